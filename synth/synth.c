/*
 * Seeded synthetic luma generator.
 *
 * This module produces the inputs that both the GPU path and the CPU oracle
 * consume.  It holds none of the coding-tree search arithmetic (no SAD, SATD,
 * prediction, lambda or bit-count code): it only renders 8-bit luma frames.
 *
 * Content model (integer-only, deterministic for a given seed):
 *   - background: three octaves of value noise with lattice spacings 64, 32
 *     and 16 pixels, weighted 4:2:1, bilinear interpolation in Q8.  It is
 *     procedural at any integer coordinate, so a global pan reveals new
 *     content instead of wrapping;
 *   - moving objects: textured rectangles (their own value noise plus a
 *     stripe pattern), each translating by a constant integer motion per
 *     frame; later rectangles are drawn over earlier ones;
 *   - sensor noise: zero-mean, approximately Gaussian (Irwin-Hall sum of 12
 *     uniforms), scaled by sigma and rounded, from a counter-based hash of
 *     (seed, frame, x, y) so the value does not depend on render order;
 *   - clip to 0..255.
 * A box filter with rounding, (sum + n*n/2) / (n*n), followed by a crop
 * produces lower ladder rungs from one high-resolution source.
 *
 * Random streams: PCG32 (PCG-XSH-RR, 64-bit state; M. E. O'Neill, 2014) for
 * the scene parameters, SplitMix64 (Steele, Lea, Flood, 2014) as the
 * stateless hash for lattice values and per-pixel noise.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SYN_MAX_RECTS 256

typedef struct {
  uint64_t state, inc;
} pcg32_t;

static uint32_t pcg32_next(pcg32_t* g) {
  uint64_t old = g->state;
  g->state = old * 6364136223846793005ULL + g->inc;
  uint32_t xorshifted = (uint32_t)(((old >> 18u) ^ old) >> 27u);
  uint32_t rot = (uint32_t)(old >> 59u);
  return (xorshifted >> rot) | (xorshifted << ((-rot) & 31u));
}

static void pcg32_seed(pcg32_t* g, uint64_t initstate, uint64_t initseq) {
  g->state = 0u;
  g->inc = (initseq << 1u) | 1u;
  pcg32_next(g);
  g->state += initstate;
  pcg32_next(g);
}

/* Uniform integer in [lo, hi] (inclusive), by rejection (no modulo bias). */
static int32_t pcg32_range(pcg32_t* g, int32_t lo, int32_t hi) {
  uint32_t span = (uint32_t)(hi - lo) + 1u;
  uint32_t limit = (uint32_t)(0x100000000ULL - (0x100000000ULL % span));
  for (;;) {
    uint32_t r = pcg32_next(g);
    if (span == 0u) return (int32_t)r;
    if (limit == 0u || r < limit) return lo + (int32_t)(r % span);
  }
}

static uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static uint32_t lattice_value(uint64_t seed, int64_t gx, int64_t gy, uint32_t salt) {
  uint64_t k = seed;
  k ^= (uint64_t)gx * 0xD1B54A32D192ED03ULL;
  k ^= (uint64_t)gy * 0xABC98388FB8FAC03ULL;
  k ^= (uint64_t)salt * 0x8CB92BA72F3D8DD7ULL;
  return (uint32_t)(splitmix64(k) & 255u);
}

/* One octave of value noise at integer coordinate (x, y), lattice 1<<lg. */
static uint32_t value_noise(uint64_t seed, int64_t x, int64_t y, int lg, uint32_t salt) {
  int64_t gx = x >> lg, gy = y >> lg; /* arithmetic shift = floor division */
  uint32_t fx = (uint32_t)(x & ((1 << lg) - 1)), fy = (uint32_t)(y & ((1 << lg) - 1));
  uint32_t wx = (fx << 8) >> lg, wy = (fy << 8) >> lg; /* Q8 weights */
  uint32_t c00 = lattice_value(seed, gx, gy, salt);
  uint32_t c10 = lattice_value(seed, gx + 1, gy, salt);
  uint32_t c01 = lattice_value(seed, gx, gy + 1, salt);
  uint32_t c11 = lattice_value(seed, gx + 1, gy + 1, salt);
  uint32_t v = c00 * (256 - wx) * (256 - wy) + c10 * wx * (256 - wy) + c01 * (256 - wx) * wy +
               c11 * wx * wy;
  return v >> 16;
}

typedef struct {
  int32_t x0, y0, w, h, vx, vy;
  int32_t period, amp, orient;
  uint64_t tex_seed;
} syn_rect;

typedef struct {
  uint64_t seed;
  int32_t width, height;
  int32_t pan_x, pan_y;    /* background content motion, pixels per frame */
  int32_t sigma_q4;        /* noise sigma in 1/16 */
  int32_t n_rects;
  syn_rect rects[SYN_MAX_RECTS];
} syn_scene;

/* Build the scene for a seed.  Rectangle sizes are U[16,160], motion per frame
 * U[-mv_max, mv_max] in each axis, global pan U[-pan_max, pan_max]. */
int syn_scene_size(void) { return (int)sizeof(syn_scene); }

int syn_scene_init(syn_scene* sc, uint64_t seed, int32_t width, int32_t height, int32_t n_rects,
                   int32_t mv_max, int32_t pan_max, int32_t sigma_q4) {
  if (!sc || width <= 0 || height <= 0 || n_rects < 0 || n_rects > SYN_MAX_RECTS || mv_max < 0 ||
      pan_max < 0 || sigma_q4 < 0)
    return -1;
  memset(sc, 0, sizeof(*sc));
  pcg32_t g;
  pcg32_seed(&g, seed, 0x5EEDull);
  sc->seed = seed;
  sc->width = width;
  sc->height = height;
  sc->sigma_q4 = sigma_q4;
  sc->pan_x = pan_max ? pcg32_range(&g, -pan_max, pan_max) : 0;
  sc->pan_y = pan_max ? pcg32_range(&g, -pan_max, pan_max) : 0;
  sc->n_rects = n_rects;
  for (int i = 0; i < n_rects; ++i) {
    syn_rect* r = &sc->rects[i];
    r->w = pcg32_range(&g, 16, 160);
    r->h = pcg32_range(&g, 16, 160);
    r->x0 = pcg32_range(&g, -r->w / 2, width - r->w / 2);
    r->y0 = pcg32_range(&g, -r->h / 2, height - r->h / 2);
    r->vx = mv_max ? pcg32_range(&g, -mv_max, mv_max) : 0;
    r->vy = mv_max ? pcg32_range(&g, -mv_max, mv_max) : 0;
    r->period = pcg32_range(&g, 4, 16);
    r->amp = pcg32_range(&g, 16, 64);
    r->orient = pcg32_range(&g, 0, 2);
    r->tex_seed = ((uint64_t)pcg32_next(&g) << 32) | pcg32_next(&g);
  }
  return 0;
}

static int32_t background(const syn_scene* sc, int64_t x, int64_t y) {
  uint32_t n64 = value_noise(sc->seed, x, y, 6, 1);
  uint32_t n32 = value_noise(sc->seed, x, y, 5, 2);
  uint32_t n16 = value_noise(sc->seed, x, y, 4, 3);
  return (int32_t)((4 * n64 + 2 * n32 + n16 + 3) / 7);
}

static int32_t rect_texture(const syn_rect* r, int32_t u, int32_t v) {
  int32_t base = (int32_t)((2 * value_noise(r->tex_seed, u, v, 4, 7) +
                            value_noise(r->tex_seed, u, v, 3, 8) + 1) / 3);
  int32_t coord = r->orient == 0 ? u : (r->orient == 1 ? v : u + v);
  int32_t stripe = ((coord / r->period) & 1) ? r->amp / 2 : -(r->amp / 2);
  return base + stripe;
}

static int32_t pixel_noise(const syn_scene* sc, int32_t t, int32_t x, int32_t y) {
  if (sc->sigma_q4 == 0) return 0;
  uint64_t ctr = sc->seed ^ 0x6A09E667F3BCC909ULL;
  ctr ^= (uint64_t)(uint32_t)t * 0x9E3779B97F4A7C15ULL;
  ctr ^= ((uint64_t)(uint32_t)y << 32) | (uint32_t)x;
  int64_t s = 0;
  for (int k = 0; k < 3; ++k) {
    uint64_t h = splitmix64(ctr + (uint64_t)k * 0xC2B2AE3D27D4EB4FULL);
    s += (int64_t)(h & 0xFFFF) + (int64_t)((h >> 16) & 0xFFFF) + (int64_t)((h >> 32) & 0xFFFF) +
         (int64_t)(h >> 48);
  }
  /* s ~ Irwin-Hall(12) * 65536 ; centre 12 * 65535 / 2 = 393210 */
  int64_t num = (int64_t)sc->sigma_q4 * (s - 393210);
  return (int32_t)((num + (1 << 19)) >> 20); /* / (16 * 65536), rounded */
}

/* Render frame t (t = 0, 1, ...) of the scene into out (width x height, row stride). */
int syn_render(const syn_scene* sc, int32_t t, uint8_t* out, int32_t stride) {
  if (!sc || !out || stride < sc->width || t < 0) return -1;
  const int32_t W = sc->width, H = sc->height;
#pragma omp parallel for schedule(static)
  for (int32_t y = 0; y < H; ++y) {
    uint8_t* row = out + (int64_t)y * stride;
    for (int32_t x = 0; x < W; ++x) {
      int32_t v = background(sc, (int64_t)x + (int64_t)sc->pan_x * t,
                             (int64_t)y + (int64_t)sc->pan_y * t);
      for (int32_t i = 0; i < sc->n_rects; ++i) {
        const syn_rect* r = &sc->rects[i];
        int32_t rx = r->x0 + r->vx * t, ry = r->y0 + r->vy * t;
        if (x >= rx && x < rx + r->w && y >= ry && y < ry + r->h) v = rect_texture(r, x - rx, y - ry);
      }
      v += pixel_noise(sc, t, x, y);
      row[x] = (uint8_t)(v < 0 ? 0 : (v > 255 ? 255 : v));
    }
  }
  return 0;
}

/* Box-filter downscale by an integer factor n, with rounding, then crop to
 * (dw, dh).  Requires dw * n <= sw and dh * n <= sh. */
int syn_box_downscale(const uint8_t* src, int32_t sw, int32_t sh, int32_t sstride, int32_t n,
                      uint8_t* dst, int32_t dw, int32_t dh, int32_t dstride) {
  if (!src || !dst || n <= 0 || dw <= 0 || dh <= 0 || (int64_t)dw * n > sw ||
      (int64_t)dh * n > sh || dstride < dw || sstride < sw)
    return -1;
  const uint32_t area = (uint32_t)(n * n);
#pragma omp parallel for schedule(static)
  for (int32_t y = 0; y < dh; ++y) {
    for (int32_t x = 0; x < dw; ++x) {
      uint32_t s = 0;
      for (int32_t j = 0; j < n; ++j) {
        const uint8_t* r = src + (int64_t)(y * n + j) * sstride + (int64_t)x * n;
        for (int32_t i = 0; i < n; ++i) s += r[i];
      }
      dst[(int64_t)y * dstride + x] = (uint8_t)((s + area / 2) / area);
    }
  }
  return 0;
}

/* Uniform white noise frame (each pixel an independent byte), used where a
 * test needs content whose block matches are unambiguous. */
int syn_white_noise(uint64_t seed, int32_t width, int32_t height, uint8_t* out, int32_t stride) {
  if (!out || width <= 0 || height <= 0 || stride < width) return -1;
#pragma omp parallel for schedule(static)
  for (int32_t y = 0; y < height; ++y)
    for (int32_t x = 0; x < width; ++x)
      out[(int64_t)y * stride + x] =
          (uint8_t)(splitmix64(seed ^ (((uint64_t)(uint32_t)y << 32) | (uint32_t)x)) >> 56);
  return 0;
}

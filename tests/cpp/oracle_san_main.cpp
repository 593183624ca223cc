// Runs every entry point of the CPU oracle on small pseudo-random pictures
// (ragged sizes down to 1x1, every search form) so that a build with
// AddressSanitizer and UndefinedBehaviorSanitizer sees each code path: out-of-
// bounds reads of the clamped windows, signed overflow in the costs, misuse of
// the per-thread job records.  Also checks J = D * 65536 + s * R per CTU.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

extern "C" {
int64_t orc_sqrt_lambda_q16(int qp);
int orc_se_bits(int v);
int64_t orc_satd(const int32_t* resid, int stride, int n);
int orc_intra_predict(const uint8_t* cur, int w, int h, int stride, int x0, int y0, int n,
                      int mode, int32_t* pred);
int orc_cu_motion_search(const uint8_t* cur, const uint8_t* ref, int w, int h, int stride,
                         int x0, int y0, int n, int R, int qp, int32_t* mx, int32_t* my,
                         int64_t* sad);
int orc_interp_qpel(const uint8_t* ref, int w, int h, int stride, int qx, int qy);
int orc_subpel_refine(const uint8_t* cur, const uint8_t* ref, int w, int h, int stride, int x0,
                      int y0, int n, int mx, int my, int qp, int32_t* qx, int32_t* qy,
                      int64_t* satd);
int orc_mv_centre(const int16_t* ref_mv, int ref_w, int ref_h, int cur_w, int cur_h, int R,
                  int r, int qpel, int x0, int y0, int n, int32_t* cx, int32_t* cy);
int orc_ctu_nodes(const uint8_t* cur, const uint8_t* ref, int w, int h, int stride, int qp,
                  int R, int flags, int ctu_x, int ctu_y, const int16_t* ref_mv, int ref_w,
                  int ref_h, int refine_r, int seed_qpel, int64_t* rec);
int orc_ctu_search(const uint8_t* cur, const uint8_t* ref, int w, int h, int stride, int qp,
                   int R, int flags, const uint8_t* bounds, const int16_t* ref_mv, int ref_w,
                   int ref_h, int refine_r, int seed_qpel, uint8_t* depth, uint8_t* mode,
                   int16_t* mv, int64_t* ctu_cost, int64_t* ctu_dist, int64_t* ctu_bits,
                   const int32_t* ctu_list, int n_list, int n_threads);
int orc_depth_bounds(const uint8_t* ref_depth, int ref_w, int ref_h, int dep_w, int dep_h,
                     int delta_lo, int delta_hi, uint8_t* bounds_out);
}

static uint64_t g_state = 0x9E3779B97F4A7C15ull;
static uint32_t rnd() {  // xorshift64*
  g_state ^= g_state >> 12;
  g_state ^= g_state << 25;
  g_state ^= g_state >> 27;
  return (uint32_t)((g_state * 0x2545F4914F6CDD1Dull) >> 32);
}

static int g_fail = 0;
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::printf("check failed at line %d: %s\n", __LINE__, #c); \
      ++g_fail;                                                   \
    }                                                             \
  } while (0)

// A smooth picture plus noise, so that searches find real minima; exact-size
// allocation so that reads past the last row or column are reported.
static std::vector<uint8_t> picture(int w, int h, int stride, int shift) {
  std::vector<uint8_t> p((size_t)stride * (h - 1) + w);
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x)
      p[(size_t)y * stride + x] =
          (uint8_t)((((x + shift) * 7) ^ (y * 13)) + (int)(rnd() % 9u));
  return p;
}

static void search_case(int w, int h, int stride, int qp, int R, int flags, bool bounded,
                        int seed_r, int qpel, int threads) {
  const std::vector<uint8_t> ref = picture(w, h, stride, 0), cur = picture(w, h, stride, 3);
  const int uw = (w + 7) / 8, uh = (h + 7) / 8, tw = (uw * 8 + 63) / 64, th = (uh * 8 + 63) / 64;
  std::vector<uint8_t> depth((size_t)uw * uh), mode((size_t)uw * uh), bounds;
  std::vector<int16_t> mv((size_t)uw * uh * 2), seed;
  std::vector<int64_t> J((size_t)tw * th), D((size_t)tw * th), B((size_t)tw * th);
  if (bounded) {
    bounds.resize((size_t)uw * uh * 2);
    for (size_t u = 0; u < (size_t)uw * uh; ++u) {
      const int lo = (int)(rnd() % 4u), hi = lo + (int)(rnd() % (4u - (unsigned)lo));
      bounds[2 * u] = (uint8_t)lo, bounds[2 * u + 1] = (uint8_t)hi;
    }
  }
  const int sw = (w + 1) / 2, sh = (h + 1) / 2;
  if (seed_r >= 0) {
    seed.resize((size_t)((sw + 7) / 8) * ((sh + 7) / 8) * 2);
    for (auto& v : seed) v = (int16_t)((int)(rnd() % (2u * 40 + 1)) - 40);
  }
  const int rc = orc_ctu_search(cur.data(), ref.data(), w, h, stride, qp, R, flags,
                                bounded ? bounds.data() : nullptr,
                                seed_r >= 0 ? seed.data() : nullptr, sw, sh,
                                seed_r >= 0 ? seed_r : 0, qpel, depth.data(), mode.data(),
                                mv.data(), J.data(), D.data(), B.data(), nullptr, 0, threads);
  CHECK(rc == 0);
  const int64_t s = orc_sqrt_lambda_q16(qp);
  for (size_t t = 0; t < J.size(); ++t) CHECK(J[t] == D[t] * 65536 + s * B[t]);
  const int max_mode = (flags & 2) ? 35 : 2;  // bit 1: angular modes
  for (size_t u = 0; u < depth.size(); ++u) CHECK(depth[u] <= 3 && mode[u] <= max_mode);
  // A listed subset (last CTU first) gives the same results for those CTUs.
  if (J.size() > 1) {
    std::vector<int64_t> J2(J.size()), D2(J.size()), B2(J.size());
    std::vector<uint8_t> d2(depth.size()), m2(depth.size());
    std::vector<int16_t> v2(mv.size());
    const int32_t list[2] = {(int32_t)J.size() - 1, 0};
    CHECK(orc_ctu_search(cur.data(), ref.data(), w, h, stride, qp, R, flags,
                         bounded ? bounds.data() : nullptr, seed_r >= 0 ? seed.data() : nullptr,
                         sw, sh, seed_r >= 0 ? seed_r : 0, qpel, d2.data(), m2.data(), v2.data(),
                         J2.data(), D2.data(), B2.data(), list, 2, 2) == 0);
    CHECK(J2[0] == J[0] && J2.back() == J.back());
  }
}

int main() {
  for (int qp : {0, 12, 32, 51}) CHECK(orc_sqrt_lambda_q16(qp) > 0);
  for (int v = -1024; v <= 1024; ++v) CHECK(orc_se_bits(v) >= 1);

  // SATD on the CU sizes, with extreme residuals.
  for (int n : {4, 8, 16, 32, 64}) {
    std::vector<int32_t> r((size_t)n * n);
    for (auto& x : r) x = (int)(rnd() % 511u) - 255;
    CHECK(orc_satd(r.data(), n, n) >= 0);
  }

  // Intra prediction at the picture's corners and edges (neighbour substitution).
  {
    const int w = 37, h = 29;
    const std::vector<uint8_t> c = picture(w, h, w, 1);
    std::vector<int32_t> pred(64 * 64);
    for (int n : {8, 16, 32})
      for (int mode = 1; mode <= 35; ++mode)
        for (int y0 : {0, 8, 24})
          for (int x0 : {0, 16, 32}) CHECK(orc_intra_predict(c.data(), w, h, w, x0, y0, n, mode, pred.data()) == 0);
  }

  // Motion search, interpolation and sub-pel refinement near and beyond the edges.
  {
    const int w = 45, h = 27;
    const std::vector<uint8_t> a = picture(w, h, w, 0), b = picture(w, h, w, 2);
    int32_t mx, my, qx, qy;
    int64_t sad, satd;
    CHECK(orc_cu_motion_search(a.data(), b.data(), w, h, w, 40, 24, 8, 9, 30, &mx, &my, &sad) == 0);
    for (int q : {-500, -3, 0, 1, 2, 3, 177, 900})
      CHECK(orc_interp_qpel(b.data(), w, h, w, q, -q) >= 0);
    CHECK(orc_subpel_refine(a.data(), b.data(), w, h, w, 40, 24, 8, mx, my, 30, &qx, &qy, &satd) == 0);
    CHECK(orc_subpel_refine(a.data(), b.data(), w, h, w, 0, 0, 16, -60, 60, 51, &qx, &qy, &satd) == 0);
    const std::vector<int16_t> seed(6 * 4 * 2, 100);
    int32_t cx, cy;
    CHECK(orc_mv_centre(seed.data(), 41, 30, 90, 61, 16, 3, 0, 80, 56, 8, &cx, &cy) == 0);
    std::vector<int64_t> rec(85 * 14);
    CHECK(orc_ctu_nodes(a.data(), b.data(), w, h, w, 27, 6, 1, 0, 0, nullptr, 0, 0, 0, 0, rec.data()) == 0);
    CHECK(orc_ctu_nodes(a.data(), b.data(), w, h, w, 27, 6, 3, 0, 0, nullptr, 0, 0, 0, 0, rec.data()) == 0);
  }

  // Whole searches: sub-unit and ragged pictures, padded strides, every search form.
  struct Sz { int w, h, stride; };
  for (Sz z : {Sz{1, 1, 1}, Sz{5, 3, 7}, Sz{17, 9, 17}, Sz{72, 40, 80}, Sz{130, 70, 131}}) {
    search_case(z.w, z.h, z.stride, 32, 0, 0, false, -1, 0, 1);
    search_case(z.w, z.h, z.stride, 51, 5, 0, true, -1, 0, 3);
    search_case(z.w, z.h, z.stride, 0, 8, 1, false, -1, 0, 2);
    search_case(z.w, z.h, z.stride, 27, 8, 0, true, 2, 0, 4);
    search_case(z.w, z.h, z.stride, 22, 6, 1, false, 6, 1, 2);
    search_case(z.w, z.h, z.stride, 37, 4, 2, true, -1, 0, 3);   // angular intra modes
    search_case(z.w, z.h, z.stride, 30, 4, 3, false, 3, 0, 2);   // angular + sub-pel, seeded
  }

  // Depth bounds at dyadic and odd ratios, up and down.
  {
    const int dims[][4] = {{960, 540, 1920, 1080}, {1280, 720, 3840, 2160}, {426, 240, 640, 360},
                           {1920, 1080, 426, 240}, {8, 8, 8192, 64}, {1, 1, 3, 5}};
    for (const auto& d : dims) {
      std::vector<uint8_t> rd((size_t)((d[0] + 7) / 8) * ((d[1] + 7) / 8));
      for (auto& x : rd) x = (uint8_t)(rnd() % 4u);
      std::vector<uint8_t> out((size_t)((d[2] + 7) / 8) * ((d[3] + 7) / 8) * 2);
      CHECK(orc_depth_bounds(rd.data(), d[0], d[1], d[2], d[3], 1, 2, out.data()) == 0);
      for (size_t u = 0; u < out.size(); u += 2) CHECK(out[u] <= out[u + 1] && out[u + 1] <= 3);
    }
  }

  if (g_fail) {
    std::printf("%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("all checks passed\n");
  return 0;
}

// HIP kernels of libmr for gfx950 (CDNA4): the per-CTU coding-tree search.
//
// Pipeline per frame pair (one job):
//   prep   : pack the current CTUs into 8x8-block-linear dwords (coded picture,
//            edge-replicated), reset the arg-min keys, mark leaf-eligible nodes
//            (inside the picture and allowed by the depth bounds);
//   search : integer full-search ME.  Persistent workgroups take (strip of
//            CTUs, dy band) items -- or, at small ranges, one CTU whose
//            quadrants go to the four wavefronts -- and stage the reference
//            window in LDS; each lane owns 4 horizontal x D vertical candidate
//            shifts and computes the 64 8x8 SADs per candidate with
//            v_qsad_pk_u16_u8 (the 4 horizontal shifts of a window dword pair
//            in one instruction, as packed 16-bit sums; current block from an
//            LDS ring), sums them into 16/32/64 SADs and keeps an exact
//            first-minimum arg-min for all 85 CUs;
//   leaf   : SATD (4x4 Hadamard) of the inter residual at the best MV and of
//            the intra DC / planar residuals, leaf mode choice, bottom-up
//            quad-tree decision with optional depth bounds, outputs.
// All arithmetic is integer and matches the CPU definition bit for bit.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>

#include "mr_device.h"

namespace mr {

// Minimum over the 64 lanes of a wavefront (all lanes active); wave-uniform result.
// The within-row steps read a valid source lane everywhere, so their "old"
// operand is never used; passing ~0 (the identity of min) lets each step fuse
// into one v_min_u32_dpp.
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
  v = min(v, dpp_mov<0xB1, 0xF>(0xFFFFFFFFu, v));   // quad_perm [1,0,3,2]
  v = min(v, dpp_mov<0x4E, 0xF>(0xFFFFFFFFu, v));   // quad_perm [2,3,0,1]
  v = min(v, dpp_mov<0x141, 0xF>(0xFFFFFFFFu, v));  // row_half_mirror
  v = min(v, dpp_mov<0x140, 0xF>(0xFFFFFFFFu, v));  // row_mirror
  v = min(v, dpp_mov<0x142, 0xA>(0xFFFFFFFFu, v));  // row_bcast:15
  v = min(v, dpp_mov<0x143, 0xC>(0xFFFFFFFFu, v));  // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Minima over the wavefront of four per-lane values at once: on return lane l
// holds the minimum over all 64 lanes of v[l & 3].  Two exchange steps leave
// each lane of a quad with the quad minimum of its own value (lane bit 0, then
// bit 1, selects which pair/value a lane keeps); rotations by 4 and 8 within a
// row and exchanges with lanes l ^ 16 and l ^ 32 keep the low two bits, so
// they complete the reduction per value.
__device__ __forceinline__ uint32_t wave_min4(uint32_t v0, uint32_t v1, uint32_t v2, uint32_t v3) {
  const int lane = threadIdx.x & 63;
  const bool b0 = (lane & 1) != 0, b1 = (lane & 2) != 0;
  uint32_t k0 = b0 ? v1 : v0, s0 = b0 ? v0 : v1;
  uint32_t k1 = b0 ? v3 : v2, s1 = b0 ? v2 : v3;
  k0 = min(k0, dpp_mov<0xB1, 0xF>(0xFFFFFFFFu, s0));  // lane ^ 1 (quad_perm [1,0,3,2])
  k1 = min(k1, dpp_mov<0xB1, 0xF>(0xFFFFFFFFu, s1));
  uint32_t k = b1 ? k1 : k0;
  const uint32_t sk = b1 ? k0 : k1;
  k = min(k, dpp_mov<0x4E, 0xF>(0xFFFFFFFFu, sk));   // lane ^ 2 (quad_perm [2,3,0,1])
  k = min(k, dpp_mov<0x124, 0xF>(0xFFFFFFFFu, k));   // row_ror:4
  k = min(k, dpp_mov<0x128, 0xF>(0xFFFFFFFFu, k));   // row_ror:8
  k = min(k, (uint32_t)__builtin_amdgcn_ds_swizzle((int)k, 0x401F));  // lane ^ 16
  k = min(k, (uint32_t)__builtin_amdgcn_ds_bpermute((lane ^ 32) << 2, (int)k));  // lane ^ 32
  return k;
}

// v_writelane_b32: clang has no builtin for it, so bind the LLVM intrinsic.
__device__ int amdgcn_writelane(int src, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

// v with lane `l` (wave-uniform) replaced by the wave-uniform value u: one
// v_writelane instead of a compare, a move and a select.
__device__ __forceinline__ uint32_t set_lane(uint32_t v, uint32_t u, int l) {
  return (uint32_t)amdgcn_writelane((int)u, l, (int)v);
}

// ---------------------------------------------------------------------------------- prep
// One workgroup of kPrepThreads threads per CTU: enough for its 85 nodes, and
// small, so that many fit a CU (each is mostly load latency and barriers).
constexpr int kPrepThreads = 128;
__device__ void prep_ctu(cjob jb, int ctu, uint32_t* csad) {
  const int tid = threadIdx.x;
  const int cx = (ctu % jb->ctus_w) * kCtu, cy = (ctu / jb->ctus_w) * kCtu;
  // With the (R, R) task left out of the search (see SearchLayout), every CU's
  // key starts at that candidate's: csad[b] = its SAD on 8x8 block b (Z-order).
  const bool corner = jb->corner != 0;  // uniform
  if (corner) {
    if (tid < 64) csad[tid] = 0;
    __syncthreads();
  }
  // 64 blocks x 16 dwords (row r, half c of block bz at dword bz * 16 + 2r + c).
  // Thread t reads dword t & 15 of CTU rows (t >> 4) + 8 i, i = 0..7, so a
  // wavefront reads 4 whole CTU rows: plain dword loads when the frame is
  // dword-aligned and the CTU lies inside it, else clamped byte loads.  A job
  // that shares another job's packed copy only reads, for the corner SADs.
  const bool pack = jb->pack_cur != 0;  // uniform
  if (pack || corner) {
    uint32_t* dst = (uint32_t*)jb->curpack + (size_t)ctu * 1024;
    const int c16 = tid & 15, x0 = cx + 4 * c16;
    const bool ref_fast = (((uintptr_t)jb->ref) & 3) == 0;
    const uint32_t frame_bytes = (uint32_t)((jb->h - 1) * jb->stride + jb->w);
    const bool fast = ((jb->stride & 3) == 0) && ((((uintptr_t)jb->cur) & 3) == 0) &&
                      cx + 64 <= jb->w && cy + 64 <= jb->h;  // uniform
#pragma unroll
    for (int i = 0; i < 64 / (kPrepThreads / 16); ++i) {
      const int ry = (tid >> 4) + (kPrepThreads / 16) * i;
      uint32_t v;
      if (fast) {
        v = *(const uint32_t*)(jb->cur + (uint32_t)((cy + ry) * jb->stride + x0));
      } else {
        const uint8_t* row = jb->cur + (uint32_t)(min(cy + ry, jb->h - 1) * jb->stride);
        v = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) v |= (uint32_t)row[min(x0 + b, jb->w - 1)] << (8 * b);
      }
      const int bx = c16 >> 1, by = ry >> 3;
      const int bz = (bx & 1) | ((by & 1) << 1) | ((bx & 2) << 1) | ((by & 2) << 2) |
                     ((bx & 4) << 2) | ((by & 4) << 3);
      if (pack) dst[bz * 16 + (ry & 7) * 2 + (c16 & 1)] = v;
      if (corner) {
        // Reference samples at (x + R, y + R), coordinates clamped to the picture.
        const int R = jb->R, xr = x0 + R;
        const uint32_t o = (uint32_t)(min(cy + ry + R, jb->h - 1) * jb->stride);
        uint32_t rv;
        if (ref_fast && xr + 3 < jb->w && o + (uint32_t)xr + 8u <= frame_bytes) {
          const uint32_t* a = (const uint32_t*)(jb->ref + ((o + (uint32_t)xr) & ~3u));
          rv = __builtin_amdgcn_alignbyte(a[1], a[0], (o + (uint32_t)xr) & 3u);
        } else {
          rv = 0;
#pragma unroll
          for (int b = 0; b < 4; ++b) rv |= (uint32_t)jb->ref[o + (uint32_t)min(xr + b, jb->w - 1)] << (8 * b);
        }
        atomicAdd(&csad[bz], __builtin_amdgcn_sad_u8(v, rv, 0u));
      }
    }
  }
  if (corner) __syncthreads();
  // Bounds of every node (min lo, max hi over its 8x8 units), bottom-up: one
  // load per unit, then three levels of 2x2 in LDS (nodes in raster order per
  // depth, at 0, 1, 5, 21).  Units outside the coded picture are neutral.
  __shared__ uint8_t nlo[kNodes], nhi[kNodes];
  const bool bounded = jb->bounds != nullptr;  // uniform
  if (bounded) {
    if (tid < 64) {
      const int ux = (cx >> 3) + (tid & 7), uy = (cy >> 3) + (tid >> 3), uw = jb->w8 >> 3;
      uint8_t lo = 3, hi = 0;
      if (ux < uw && uy < (jb->h8 >> 3)) {
        const uint8_t* b = jb->bounds + 2 * ((size_t)uy * uw + ux);
        lo = b[0], hi = b[1];
      }
      nlo[21 + tid] = lo, nhi[21 + tid] = hi;
    }
#pragma unroll
    for (int d = 2; d >= 0; --d) {
      __syncthreads();
      const int side = 1 << d, first = d == 0 ? 0 : d == 1 ? 1 : 5, child = d == 2 ? 21 : d == 1 ? 5 : 1;
      if (tid < side * side) {
        const int lx = tid % side, ly = tid / side, cs = 2 * side;
        const int c0 = child + 2 * ly * cs + 2 * lx;
        nlo[first + tid] = min(min(nlo[c0], nlo[c0 + 1]), min(nlo[c0 + cs], nlo[c0 + cs + 1]));
        nhi[first + tid] = max(max(nhi[c0], nhi[c0 + 1]), max(nhi[c0 + cs], nhi[c0 + cs + 1]));
      }
    }
    __syncthreads();
  }
  // Per node thread: its geometry and the bounds rule.
  int d = 0, lx = 0, ly = 0, n = kCtu, x0 = cx, y0 = cy;
  uint8_t e = 0;
  bool split_ok = false, leaf_ok = true;
  __shared__ uint8_t sok[kNodes];  // may split (a node crossing the picture edge must)
  if (tid < kNodes) {
    d = tid == 0 ? 0 : tid < 5 ? 1 : tid < 21 ? 2 : 3;
    const int local = tid - (d == 0 ? 0 : d == 1 ? 1 : d == 2 ? 5 : 21);
    n = kCtu >> d, lx = local % (1 << d), ly = local / (1 << d);
    x0 = cx + lx * n, y0 = cy + ly * n;
    split_ok = d < 3;
    const bool inside = x0 + n <= jb->w8 && y0 + n <= jb->h8;
    if (inside) {
      e = 1;
      if (bounded) {
        const int min_lo = nlo[tid], max_hi = nhi[tid];
        split_ok = d < 3 && d < max_hi;
        leaf_ok = d >= min_lo || !split_ok;
        e = leaf_ok ? 1 : 0;
      }
    }
    if (bounded) sok[tid] = inside ? (split_ok ? 1 : 0) : 1;
  }
  if (bounded) {
    // A node is reached only if every ancestor may split: one below a node
    // that may not is never part of the partition, so it is not eligible
    // either (no search key, refinement or SATD for it).
    __syncthreads();
    if (tid < kNodes) {
      for (int a = 0; a < d; ++a) {
        const int base = a == 0 ? 0 : a == 1 ? 1 : 5;
        if (!sok[base + (ly >> (d - a)) * (1 << a) + (lx >> (d - a))]) e = 0;
      }
    }
  }
  if (tid < kNodes) {
    jb->elig[(size_t)ctu * kNodes + tid] = e;
    jb->okbits[(size_t)ctu * kNodes + tid] = (uint8_t)((split_ok ? 1 : 0) | (leaf_ok ? 2 : 0));
    if (jb->seed_mv) {
      // Seeded search centre: the reference MV of the unit co-located with the
      // CU's centre, scaled to this picture and clamped so that the refinement
      // window stays inside the search range.
      const uint32_t sw = jb->seed_w, shh = jb->seed_h, W = jb->w, H = jb->h;
      const uint32_t px = x0 + n / 2, py = y0 + n / 2;
      const uint32_t xr = min(px * sw / W, sw - 1), yr = min(py * shh / H, shh - 1);
      const int16_t* m = jb->seed_mv + 2 * ((yr >> 3) * ((sw + 7) >> 3) + (xr >> 3));
      const int lim = jb->R - jb->seed_r, qs = 2 * jb->seed_qpel;  // quarter-pel: 4 units a pixel
      const int cxm = clampi(scale_round_dev(m[0], W, sw << qs), -lim, lim);
      const int cym = clampi(scale_round_dev(m[1], H, shh << qs), -lim, lim);
      jb->seedc[(size_t)ctu * kNodes + tid] = (uint32_t)(cxm & 0xFFFF) | ((uint32_t)cym << 16);
    }
    uint64_t key = kKeyNone;
    if (corner) {
      // The node's blocks are a Z-order run of 4^(3-d) blocks.
      const int sh = 3 - d, cnt = 1 << (2 * sh);
      const int z0 = ((lx << sh) & 1) | (((ly << sh) & 1) << 1) | (((lx << sh) & 2) << 1) |
                     (((ly << sh) & 2) << 2) | (((lx << sh) & 4) << 2) | (((ly << sh) & 4) << 3);
      uint32_t sad = 0;
      for (int k = 0; k < cnt; ++k) sad += csad[z0 + k];
      const int R = jb->R, span = 2 * R + 1;
      const uint64_t J = (uint64_t)sad * 65536u + (uint64_t)jb->s * (uint64_t)(2 * se_bits_dev(4 * R));
      key = (J << 17) | (uint64_t)(2 * R * span + 2 * R);  // raster index of (R, R)
    }
    jb->keys[(size_t)ctu * kNodes + tid] = key;
    // Eligibility as a bit mask: nodes 0..63 in the first wavefront, 64..84 in the second.
    const unsigned long long bits = __ballot(e != 0);
    if ((tid & 63) == 0) {
      uint32_t* eb = jb->eligbits + (size_t)ctu * 4;
      if (tid == 0) eb[0] = (uint32_t)bits, eb[1] = (uint32_t)(bits >> 32);
      else eb[2] = (uint32_t)bits, eb[3] = 0;
    }
  }
}


// -------------------------------------------------------------------------------- search
// Stage rows [y0, y0 + rows) x dword columns [0, Wd) of the reference, with
// coordinates clamped to the picture, into the LDS window (x origin x0).  The
// window is column-major with an odd pitch hs: dword column c, row r at
// c * hs + r, so the rows a search lane walks are immediate offsets of its
// column addresses, and lanes on consecutive columns hit distinct banks.
// Each thread owns one dword column and every per-th row of it (per = the
// workgroup's threads / Wd, at least 1), so the column's clamping is decided
// once; four rows are loaded before any is stored, keeping four loads in
// flight per thread.
__device__ void stage_window(cjob jb, int x0, int y0, int rows, int hs, uint32_t* win) {
  const int Wd = jb->win_dwords, w = jb->w, h = jb->h, stride = jb->stride;
  const uint8_t* ref = jb->ref;
  const bool dword_ok = ((stride & 3) == 0) && ((((uintptr_t)ref) & 3) == 0) && ((x0 & 3) == 0);
  const int nthr = blockDim.x;
  const int per = max(1, nthr / Wd);
  for (int pair = threadIdx.x; pair < per * Wd; pair += nthr) {
    const int p = pair / Wd, c = pair - p * Wd;
    const int x = x0 + 4 * c;
    uint32_t* dst = win + c * hs;
    if (dword_ok && x >= 0 && x + 3 < w) {
      const uint8_t* base = ref + x;
      int r = p;
      for (; r + 3 * per < rows; r += 4 * per) {
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          v[u] = *(const uint32_t*)(base + (size_t)clampi(y0 + r + u * per, 0, h - 1) * stride);
#pragma unroll
        for (int u = 0; u < 4; ++u) dst[r + u * per] = v[u];
      }
      for (; r < rows; r += per)
        dst[r] = *(const uint32_t*)(base + (size_t)clampi(y0 + r, 0, h - 1) * stride);
    } else {
      int xb[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) xb[b] = clampi(x + b, 0, w - 1);
      for (int r = p; r < rows; r += per) {
        const uint8_t* rp = ref + (size_t)clampi(y0 + r, 0, h - 1) * stride;
        uint32_t v = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) v |= (uint32_t)rp[xb[b]] << (8 * b);
        dst[r] = v;
      }
    }
  }
}

// Merge a wave's reduced 32-bit keys (one CU per lane) into its 64-bit bests.
__device__ __forceinline__ void merge_keys(uint32_t vk, const uint64_t* __restrict__ dt,
                                           uint64_t& best) {
  if (vk != 0xFFFFFFFFu) {
    const uint64_t K = ((uint64_t)(vk >> kRankBits) << 33) + dt[vk & ((1u << kRankBits) - 1)];
    best = K < best ? K : best;
  }
}

// One wavefront: steps [st_lo, st_hi) of one (CTU, band); `win` points at
// this CTU's column 0 of the staged window (dx = -R), whose dword columns are
// hs apart; `ring` is this wavefront's 512-byte LDS ring for the current CTU
// (two 16x16 regions of 64 dwords).
//
// SPLIT: the workgroup's four wavefronts take the four 32x32 quadrants of one
// CTU (quadrant = wavefront index), each over the same steps, so a CTU's work
// is spread over four SIMDs instead of one.  The 8x8..32x32 CUs lie inside a
// quadrant; the 64x64 CU's SAD per candidate is the sum of the four quadrant
// SADs, exchanged through LDS (`xch`, two buffers alternating by step, so one
// barrier per step suffices) and keyed by wavefront 0.
template <int D, bool SPLIT>
__device__ void search_wave(cjob jb, int ctu, int band, int st_lo, int st_hi, const uint32_t* win,
                            int hs, uint32_t* ring, int quad, uint32_t* xch) {
  constexpr int NREG = SPLIT ? 4 : 16;
  const int reg0 = SPLIT ? 4 * quad : 0;
  const int lane = threadIdx.x & 63;
  const int Q = jb->Q;
  const int g0 = jb->band_g0[band];  // group of the band's first task: window row 0
  const int ntasks = jb->ntasks;
  const int step0 = jb->band_step0[band];
  // Leaf-eligible nodes as an 85-bit mask in SGPRs (bit n of word n >> 5).
  const sptr32 eb = (sptr32)(jb->eligbits + (size_t)ctu * 4);
  const uint32_t em0 = eb[0], em1 = eb[1], em2 = eb[2];
  // Current CTU, 8x8-block-linear in Z-order: region r = dwords [64 r, 64 r + 64).
  const uint32_t* __restrict__ cur = jb->curpack + (size_t)ctu * 1024;
  const uint32_t* __restrict__ qtab = jb->qtab;
  const uint64_t* __restrict__ dtab = jb->dtab;
  uint64_t best8 = kKeyNone, bestB = kKeyNone;

  for (int st = st_lo; st < st_hi; ++st) {
    const int gstep = step0 + st;
    int task = gstep * kWaveSteps + lane;
    if (task >= ntasks) task = ntasks - 1;  // idle lane: its table entries are invalid
    const int g = task / Q, qd = task - g * Q;
    uint32_t kq[D][4];
    {
      const uint4* qp = (const uint4*)(qtab + ((size_t)gstep * kWaveSteps + lane) * (4 * D));
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const uint4 t = qp[j];
        kq[j][0] = t.x, kq[j][1] = t.y, kq[j][2] = t.z, kq[j][3] = t.w;
      }
    }
    const uint32_t* lbase = win + qd * hs + (g - g0) * D;  // row dy of window column qd
    // s16q[j]: the 16x16 SADs of the 4 horizontal shifts of vertical shift j,
    // packed as 16-bit fields (at most 4 x 16320 < 2^16, so packed adds are exact).
    uint64_t s16q[D];
    uint32_t s32[D][4], s64[D][4];
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int k = 0; k < 4; ++k) s64[j][k] = 0;
    uint32_t vk8 = 0xFFFFFFFFu, vkB = 0xFFFFFFFFu;
    // The first region of the current CTU into the ring; later regions are
    // fetched one region ahead (global load now, LDS write after the region's
    // compute).
    ring[lane] = cur[reg0 * 64 + lane];
    uint32_t pre = cur[(reg0 + 1) * 64 + lane];

    for (int rr = 0; rr < NREG; ++rr) {
      const int reg = reg0 + rr;
      const uint32_t* rcur = ring + (rr & 1) * 64;
      uint32_t m8[4];  // per-lane minimum key of each 8x8 block of the region
      // The region's window columns 4 zx(reg) + 0..4 from row 16 zy(reg): the
      // left blocks read columns 0..2, the right ones 2..4, the lower ones 8
      // rows further down (immediate offsets).
      const uint32_t* cb[5];
      cb[0] = lbase + 4 * zx(reg) * hs + 16 * zy(reg);
#pragma unroll
      for (int m = 1; m < 5; ++m) cb[m] = cb[m - 1] + hs;
#pragma unroll
      for (int sub = 0; sub < 4; ++sub) {
        const int bz = reg * 4 + sub;
        const int bx = zx(bz), by = zy(bz);
        uint32_t cw[16];
        {
          const uint4* cp = (const uint4*)(rcur + sub * 16);  // same address in every lane
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const uint4 t = cp[i];
            cw[4 * i] = t.x, cw[4 * i + 1] = t.y, cw[4 * i + 2] = t.z, cw[4 * i + 3] = t.w;
          }
        }
        // acq[j]: the block's SADs at the 4 horizontal shifts k of vertical
        // shift j, as 16-bit fields k (at most 64 x 255 = 16320).  One
        // v_qsad_pk_u16_u8 takes 8 window bytes (two dwords) and one current
        // dword and adds the 4 SADs of the dword against the window bytes
        // k .. k + 3, k = 0..3: the horizontal shifts without re-aligning the
        // window.  The two dwords of an 8-sample row are two such steps.
        uint64_t acq[D];
#pragma unroll
        for (int j = 0; j < D; ++j) acq[j] = 0;
        const uint32_t *c0 = cb[2 * (sub & 1)], *c1 = cb[2 * (sub & 1) + 1],
                       *c2 = cb[2 * (sub & 1) + 2];
        // The middle dword is loaded twice, once into each register pair
        // ((d1:d0) and (d2:d1) must each be an aligned pair): a second LDS read
        // instead of a v_mov per row.  c1b is c1 through an opaque zero, so
        // that the two loads are not merged.
        uint32_t zero = 0;
        asm volatile("" : "+v"(zero));
        const uint32_t* c1b = c1 + zero;
        const int r0 = 8 * (sub >> 1);
        // Window rows are loaded one row ahead of their use, so each row's LDS
        // latency overlaps the previous row's SADs.
        uint32_t n0 = c0[r0], n1 = c1[r0], n1b = c1b[r0], n2 = c2[r0];
#pragma unroll
        for (int w = 0; w < D + 7; ++w) {
          const uint32_t d0 = n0, d1 = n1, d1b = n1b, d2 = n2;
          if (w + 1 < D + 7) {
            n0 = c0[r0 + w + 1], n1 = c1[r0 + w + 1], n1b = c1b[r0 + w + 1], n2 = c2[r0 + w + 1];
          }
          __builtin_amdgcn_sched_barrier(0);
          const uint64_t p0 = ((uint64_t)d1 << 32) | d0, p1 = ((uint64_t)d2 << 32) | d1b;
#pragma unroll
          for (int j = 0; j < D; ++j) {
            const int r = w - j;
            if (r < 0 || r > 7) continue;
            acq[j] = __builtin_amdgcn_qsad_pk_u16_u8(p0, cw[2 * r], acq[j]);
            acq[j] = __builtin_amdgcn_qsad_pk_u16_u8(p1, cw[2 * r + 1], acq[j]);
          }
        }
        const int n8 = 21 + by * 8 + bx;  // 21..84
        const uint32_t ew = n8 < 32 ? em0 : (n8 < 64 ? em1 : em2);
        m8[sub] = 0xFFFFFFFFu;  // not leaf-eligible: no key
        if ((ew >> (n8 & 31)) & 1u) {
          uint32_t m = 0xFFFFFFFFu;
#pragma unroll
          for (int j = 0; j < D; ++j)
#pragma unroll
            for (int k = 0; k < 4; ++k) m = min(m, field_mad(acq[j], k, 2048u, kq[j][k]));
          m8[sub] = m;
        }
#pragma unroll
        for (int j = 0; j < D; ++j) s16q[j] = sub == 0 ? acq[j] : s16q[j] + acq[j];
      }
      // The region's four 8x8 CUs are blocks 4 reg .. 4 reg + 3, i.e. lanes
      // whose low two bits name the block: one joint wavefront reduction.
      {
        const uint32_t r = wave_min4(m8[0], m8[1], m8[2], m8[3]);
        vk8 = (lane >> 2) == reg ? r : vk8;
      }
      // Next-but-one region into the slot this region used.
      if (rr < NREG - 1) {
        ring[((rr + 1) & 1) * 64 + lane] = pre;
        if (rr < NREG - 2) pre = cur[(reg + 2) * 64 + lane];
      }
      {  // 16x16 CU of this region (nodes 5..20)
        const int lx = zx(reg), ly = zy(reg);
        if ((em0 >> (5 + ly * 4 + lx)) & 1u) {
          uint32_t m = 0xFFFFFFFFu;
#pragma unroll
          for (int j = 0; j < D; ++j)
#pragma unroll
            for (int k = 0; k < 4; ++k) m = min(m, field_mad(s16q[j], k, 2048u, kq[j][k]));
          const uint32_t mk = wave_min(m);
          vkB = set_lane(vkB, mk, reg);
        }
        if ((reg & 3) == 0) {
#pragma unroll
          for (int j = 0; j < D; ++j)
#pragma unroll
            for (int k = 0; k < 4; ++k) s32[j][k] = 0;
        }
#pragma unroll
        for (int j = 0; j < D; ++j)
#pragma unroll
          for (int k = 0; k < 4; ++k) s32[j][k] = field_mad(s16q[j], k, 1u, s32[j][k]);
      }
      if ((reg & 3) == 3) {  // 32x32 CU (nodes 1..4)
        const int qz = reg >> 2, lx = qz & 1, ly = qz >> 1;
        if ((em0 >> (1 + ly * 2 + lx)) & 1u) {
          uint32_t m = 0xFFFFFFFFu;
#pragma unroll
          for (int j = 0; j < D; ++j)
#pragma unroll
            for (int k = 0; k < 4; ++k) m = min(m, s32[j][k] * 2048u + kq[j][k]);
          const uint32_t mk = wave_min(m);
          vkB = set_lane(vkB, mk, 16 + qz);
        }
        if (!SPLIT) {
#pragma unroll
          for (int j = 0; j < D; ++j)
#pragma unroll
            for (int k = 0; k < 4; ++k) s64[j][k] += s32[j][k];
        }
      }
    }
    if (SPLIT) {
      // s32 holds this quadrant's SADs; the 64x64 SAD is the sum over the
      // four wavefronts.  The condition is uniform over the workgroup.
      if (em0 & 1u) {
        uint32_t* xb = xch + (st & 1) * (3 * 64 * 4 * D);
        if (quad != 0) {
#pragma unroll
          for (int j = 0; j < D; ++j)
#pragma unroll
            for (int k = 0; k < 4; ++k) xb[((quad - 1) * 4 * D + j * 4 + k) * 64 + lane] = s32[j][k];
        }
        __syncthreads();
        if (quad == 0) {
          uint32_t m = 0xFFFFFFFFu;
#pragma unroll
          for (int j = 0; j < D; ++j)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int jk = j * 4 + k;
              const uint32_t t = s32[j][k] + xb[jk * 64 + lane] + xb[(4 * D + jk) * 64 + lane] +
                                 xb[(8 * D + jk) * 64 + lane];
              m = min(m, t * 2048u + kq[j][k]);
            }
          const uint32_t mk = wave_min(m);
          vkB = set_lane(vkB, mk, 20);
        }
      }
    } else if (em0 & 1u) {  // 64x64 CU (node 0)
      uint32_t m = 0xFFFFFFFFu;
#pragma unroll
      for (int j = 0; j < D; ++j)
#pragma unroll
        for (int k = 0; k < 4; ++k) m = min(m, s64[j][k] * 2048u + kq[j][k]);
      const uint32_t mk = wave_min(m);
      vkB = set_lane(vkB, mk, 20);
    }
    const uint64_t* dt = dtab + (size_t)gstep * 2048;
    merge_keys(vk8, dt, best8);
    if (lane < 21) merge_keys(vkB, dt, bestB);
  }

  // Publish: lane i holds the 8x8 CU of Z-order block i; lanes 0..20 the larger CUs.
  unsigned long long* keys = (unsigned long long*)jb->keys + (size_t)ctu * kNodes;
  if (best8 != kKeyNone) atomicMin(&keys[21 + zy(lane) * 8 + zx(lane)], (unsigned long long)best8);
  if (lane < 21 && bestB != kKeyNone) {
    int node;
    if (lane < 16) node = 5 + zy(lane) * 4 + zx(lane);
    else if (lane < 20) node = 1 + ((lane - 16) >> 1) * 2 + ((lane - 16) & 1);
    else node = 0;
    atomicMin(&keys[node], (unsigned long long)bestB);
  }
}

// ---------------------------------------------------------------------------------- leaf
// Offsets of each node's reference arrays in LDS: left column 2N+1, top row 2N.
__device__ __forceinline__ int ref_offset(int node) {
  if (node == 0) return 0;
  if (node < 5) return 257 + (node - 1) * 129;
  if (node < 21) return 257 + 4 * 129 + (node - 5) * 65;
  return 257 + 4 * 129 + 16 * 65 + (node - 21) * 33;
}
constexpr int kRefTotal = 257 + 4 * 129 + 16 * 65 + 64 * 33;  // 3925

// The angular arrays exist only in the angular form: without them the
// workgroup's LDS is 19.4 KB, so 8 workgroups fit a CU's 160 KB (7 with them),
// and a 2160p frame's 2040 CTUs run in one round.
template <bool ANG>
struct LeafShared {
  uint8_t cur[64 * 64];
  int16_t refs[kRefTotal];
  int16_t mvx[kNodes], mvy[kNodes];  // integer-pel, or quarter-pel with sub-pel refinement
  uint8_t need[kNodes];  // intra SATDs wanted by a job that takes this job's
  uint32_t satq[kNodes];             // sub-pel: SATD at the refined MV
  int32_t dc[kNodes];                // DC: sum of the n top and n left neighbours
  int16_t nx0[kNodes], ny0[kNodes];  // node origin in the picture
  int16_t na[kNodes], nb[kNodes];    // available neighbours: scan interval [a, b] (a > b: none)
  uint32_t satd[kNodes][3];
  uint32_t part0[4][3];          // per-wave partial sums for the 64x64 node
  int64_t jt[kNodes], dt[kNodes], rt[kNodes];
  uint8_t leaf[kNodes];          // decision: 1 = leaf, 0 = split
  uint8_t kind[kNodes];          // 0 absent, 1 crosses edge, 2 inside
  uint8_t elig[kNodes];
  uint8_t mode[kNodes];
  int64_t lj[kNodes], ld[kNodes], lr[kNodes];
  uint8_t split_ok[kNodes], leaf_ok[kNodes];
  // Angular modes: per node the best (J, SATD, mode code); node 0's per-mode
  // SATDs arrive as per-wave partial sums.
  int64_t angj[ANG ? kNodes : 1];
  uint32_t angd[ANG ? kNodes : 1];
  uint8_t angm[ANG ? kNodes : 1];
  uint32_t ang0[4][ANG ? 33 : 1];
};

// H.265 intraPredAngle of intra modes 2..34 (index = mode) and, for the
// negative angles, invAngle = 8192 / angle rounded (index = -angle).
__constant__ int8_t kAngle[35] = {0,   0,   32,  26,  21,  17,  13,  9,   5,   2,   0,   -2,
                                  -5,  -9,  -13, -17, -21, -26, -32, -26, -21, -17, -13, -9,
                                  -5,  -2,  0,   2,   5,   9,   13,  17,  21,  26,  32};
__constant__ int16_t kInvAngle[33] = {0, 0, -4096, 0, 0, -1638, 0, 0, 0, -910, 0,
                                      0, 0, -630, 0, 0, 0, -482, 0, 0, 0, -390,
                                      0, 0, 0, 0, -315, 0, 0, 0, 0, 0, -256};

// Reference sample k (-n <= k <= 2n) of the angular prediction of a node
// whose neighbours R hold p[-1][i - 1] at R[i] (i = 0..2n, R[0] the corner)
// and p[i][-1] at R[2n + 1 + i] (i = 0..2n-1): along the top row for vertical
// modes, the left column for horizontal ones, and for k < 0 the other side
// projected onto that line (sample (k * invAngle + 128) >> 8 of it).
__device__ __forceinline__ int ang_ref(const int16_t* R, int n, bool vertical, int inv, int k) {
  if (k >= 0) return vertical ? R[k == 0 ? 0 : 2 * n + k] : R[k];
  const int j = (k * inv + 128) >> 8;
  return vertical ? R[j] : R[2 * n + j];
}

// The 16 predicted samples (row-major) of the 4x4 tile at (px0, py0) inside an
// n x n node for angular mode m: along the prediction direction, the row
// (vertical modes) or column (horizontal modes) q of the tile is (q + 1) *
// angle / 32 samples ahead of the reference line, split into an integer step
// and a 1/32 fraction shared by the four samples across it, which take
// ((32 - f) a + f b + 16) >> 5 of two neighbouring reference samples.
__device__ __forceinline__ void angular_tile(const int16_t* R, int n, int m, int px0, int py0,
                                             int pred[16]) {
  const int angle = kAngle[m];
  const bool vertical = m >= 18;
  const int inv = angle < 0 ? kInvAngle[-angle] : 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int along = (vertical ? py0 : px0) + q;
    const int pos = (along + 1) * angle, idx = pos >> 5, f = pos & 31;
    const int base = (vertical ? px0 : py0) + idx + 1;
    int r[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) r[i] = ang_ref(R, n, vertical, inv, min(base + i, 2 * n));
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int v = f ? ((32 - f) * r[i] + f * r[i + 1] + 16) >> 5 : r[i];
      if (vertical) pred[q * 4 + i] = v;
      else pred[i * 4 + q] = v;
    }
  }
}

// Sum over aligned groups of `width` lanes (4, 16 or 64; a compile-time
// constant after unrolling), every lane of a group receiving it: DPP adds
// within quads and rows of 16, then for 64 the four row sums read out of lanes
// 0, 16, 32 and 48.  Every lane of a group must be active.
__device__ __forceinline__ uint32_t group_sum(uint32_t v, int width) {
  if (width >= 4) v = add_dpp<0xB1>(v), v = add_dpp<0x4E>(v);      // quad_perm
  if (width >= 16) v = add_dpp<0x141>(v), v = add_dpp<0x140>(v);   // row half-mirror, mirror
  if (width >= 64)
    v = (uint32_t)(__builtin_amdgcn_readlane((int)v, 0) + __builtin_amdgcn_readlane((int)v, 16) +
                   __builtin_amdgcn_readlane((int)v, 32) + __builtin_amdgcn_readlane((int)v, 48));
  return v;
}

// Inter residual of a 4x4 tile whose reference samples start at (xf, yf):
// cp minus those samples, as pairs of a row's samples (16-bit halves).
__device__ __forceinline__ void inter_rows(cjob jb, int xf, int yf, const us2 (&cp)[8],
                                           bool ref_aligned, uint32_t frame_bytes,
                                           sh2 (&irp)[8]) {
  const uint8_t* __restrict__ rp = jb->ref;
  const int stride = jb->stride;
  // A tile whose 4 x 4 reference samples lie inside the frame: per row the two
  // dwords around its 4 samples (the last row's second dword inside the frame
  // too), one v_alignbyte and two byte-to-16-bit v_perm_b32; row offsets
  // (below 2^31) one stride apart.
  const uint32_t o0 = (uint32_t)yf * (uint32_t)stride + (uint32_t)xf;
  if (ref_aligned && xf >= 0 && xf + 3 < jb->w && yf >= 0 && yf + 3 < jb->h &&
      ((o0 + 3u * (uint32_t)stride) & ~3u) + 8u <= frame_bytes) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t o = o0 + (uint32_t)(q * stride);
      const uint32_t* a = (const uint32_t*)(rp + (o & ~3u));
      const uint32_t v = __builtin_amdgcn_alignbyte(a[1], a[0], o & 3u);
      const us2 r0 = __builtin_bit_cast(us2, __builtin_amdgcn_perm(0u, v, 0x0c010c00u));
      const us2 r1 = __builtin_bit_cast(us2, __builtin_amdgcn_perm(0u, v, 0x0c030c02u));
      irp[2 * q] = __builtin_bit_cast(sh2, cp[2 * q] - r0);
      irp[2 * q + 1] = __builtin_bit_cast(sh2, cp[2 * q + 1] - r1);
    }
  } else {
    uint32_t yo[4], xo[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      yo[q] = (uint32_t)(clampi(yf + q, 0, jb->h - 1) * stride);
      xo[q] = (uint32_t)clampi(xf + q, 0, jb->w - 1);
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const us2 r = {(unsigned short)rp[yo[m >> 1] + xo[2 * (m & 1)]],
                     (unsigned short)rp[yo[m >> 1] + xo[2 * (m & 1) + 1]]};
      irp[m] = __builtin_bit_cast(sh2, cp[m] - r);
    }
  }
}

// ANG: the angular-mode instantiation (a separate kernel, so that the default
// one keeps its register budget); a job's own flag still decides.
// SHARED: a job that takes its planar and DC SATDs from another job of the
// batch with the same current frame (intra_src): no neighbours, and its inter
// SATDs two depths at a time ((3, 2) and (1, 0)) in one packed transform.
template <bool ANG, bool SHARED>
__device__ void leaf_ctu(cjob jobs, cjob jb, int ctu, LeafShared<ANG>& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cx = (ctu % jb->ctus_w) * kCtu, cy = (ctu / jb->ctus_w) * kCtu;
  const int W8 = jb->w8, H8 = jb->h8;
  const int span = 2 * jb->R + 1;

  // Current CTU (coded picture, edge-replicated) from the copy the prep kernel
  // packed: 8x8 blocks in Z-order, 16 dwords each (row r, half c at 2r + c).
  // Thread t takes dwords 4t .. 4t + 3: rows 2 (t & 3) and 2 (t & 3) + 1 of
  // block t >> 2.
  {
    const uint4 v = ((const uint4*)(jb->curpack + (size_t)ctu * 1024))[tid];
    const int bz = tid >> 2, y = zy(bz) * 8 + 2 * (tid & 3), x = zx(bz) * 8;
    uint32_t* d = (uint32_t*)sh.cur;
    d[(y * 64 + x) >> 2] = v.x, d[(y * 64 + x + 4) >> 2] = v.y;
    d[((y + 1) * 64 + x) >> 2] = v.z, d[((y + 1) * 64 + x + 4) >> 2] = v.w;
  }
  if (tid < kNodes) {
    const int node = tid;
    const int d = node == 0 ? 0 : node < 5 ? 1 : node < 21 ? 2 : 3;
    const int local = node - (d == 0 ? 0 : d == 1 ? 1 : d == 2 ? 5 : 21);
    const int n = kCtu >> d, x0 = cx + (local % (1 << d)) * n, y0 = cy + (local / (1 << d)) * n;
    sh.kind[node] = (x0 >= W8 || y0 >= H8) ? 0 : ((x0 + n > W8 || y0 + n > H8) ? 1 : 2);
    const uint8_t e = jb->elig[(size_t)ctu * kNodes + node];
    sh.elig[node] = e;
    // A job whose intra SATDs serve other jobs computes them for every inside
    // node eligible in one of those (same current frame, so same CTU grid):
    // the union of their eligibility masks, read with scalar loads.
    uint32_t nw[3] = {0u, 0u, 0u};
    if (!SHARED && jb->intra) {
      const uint64_t users = jb->intra_users;  // uniform
      if (users >> 63) {
        nw[0] = nw[1] = nw[2] = 0xFFFFFFFFu;
      } else {
        for (uint64_t u = users; u; u &= u - 1) {
          const sptr32 eb = (sptr32)(jobs[__builtin_ctzll(u)].eligbits + (size_t)ctu * 4);
          nw[0] |= eb[0], nw[1] |= eb[1], nw[2] |= eb[2];
        }
      }
    }
    const uint32_t word = node < 32 ? nw[0] : node < 64 ? nw[1] : nw[2];
    sh.need[node] = sh.kind[node] == 2 && ((word >> (node & 31)) & 1u);
    int mx = 0, my = 0;
    uint32_t sq = 0;
    if (e && jb->subpel) {
      const uint32_t* o = jb->subres + ((size_t)ctu * kNodes + node) * 2;
      mx = (int16_t)(o[0] & 0xFFFFu), my = (int16_t)(o[0] >> 16), sq = o[1];
    } else if (e) {
      const uint64_t key = jb->keys[(size_t)ctu * kNodes + node];
      const int idx = (int)(key & 0x1FFFF);
      my = idx / span - jb->R;
      mx = idx - (my + jb->R) * span - jb->R;
    }
    sh.satq[node] = sq;
    sh.mvx[node] = (int16_t)mx, sh.mvy[node] = (int16_t)my;
    // bounds admissibility, as the prep kernel evaluated it
    const uint8_t ok = jb->okbits[(size_t)ctu * kNodes + node];
    sh.split_ok[node] = ok & 1, sh.leaf_ok[node] = (ok >> 1) & 1;
    // Neighbour samples after H.265 reference substitution.  In the
    // substitution's scan order (left column bottom to top, corner, top row
    // left to right; scan index k = 2n - off for the left column and k = off
    // for the top row) the available samples -- those inside the coded
    // picture -- form one interval [a, b]: an unavailable sample takes the
    // nearest available one scanned before it, or the first available one when
    // none is, i.e. the sample at clamp(k, a, b); with none available, 128.
    // Left-column entries p[-1][i - 1], i = 0..2n (i = 0 the corner), are
    // available for i in [hasT ? 0 : 1, min(2n, H8 - y0)]; top-row entries
    // p[i][-1] for i in [0, min(2n - 1, W8 - 1 - x0)].
    const bool hasL = x0 >= 1, hasT = y0 >= 1;
    int a = 1, b = 0;
    if (hasL || hasT) {
      const int iLlo = hasT ? 0 : 1, iLhi = min(2 * n, H8 - y0);
      a = hasL ? 2 * n - iLhi : 2 * n + 1;
      b = hasT ? 2 * n + 1 + min(2 * n - 1, W8 - 1 - x0) : 2 * n - iLlo;
    }
    sh.nx0[node] = (int16_t)x0, sh.ny0[node] = (int16_t)y0;
    sh.na[node] = (int16_t)a, sh.nb[node] = (int16_t)b;
    sh.dc[node] = 0;  // DC sums, accumulated below
  }
  __syncthreads();
  // Neighbour arrays, one depth level at a time: the 256 threads split evenly
  // over the level's nodes (256, 64, 16 or 4 per node), so a thread's node and
  // its entries follow from its index; samples inside the CTU come from LDS.
  // Planar and DC read p[-1][0..n] (entries 1 .. n + 1) and p[0..n][-1]
  // (entries 2n + 1 .. 3n + 1) only, so just those 2n + 2 are computed: the
  // closed form gives each one directly.
  const int stride = jb->stride;
  const bool angular = ANG && jb->angular != 0;  // uniform
  // A job whose intra SATDs serve other jobs computes them also for the nodes
  // eligible in one of those (sh.need), and writes them.
  const bool own = !SHARED && jb->intra != nullptr;  // uniform
  // Planar and DC read p[-1][0..n] and p[0..n][-1] of a node at (x0, y0):
  // with x0, y0 >= 1, x0 + n <= W8 - 1 and y0 + n <= H8 - 1 all of them are
  // available (a <= n - 1 and b >= 3n + 1 above), which holds for every node
  // of a CTU with cx, cy >= 1 and cx + 64, cy + 64 inside the coded picture:
  // then each entry is read straight from its position.
  const bool interior = !angular && cx >= 1 && cy >= 1 && cx + kCtu <= W8 - 1 &&
                        cy + kCtu <= H8 - 1;  // uniform
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    if (SHARED) break;
    // Angular prediction reads every entry: all 4n + 1 then.
    const int n = kCtu >> d, len = angular ? 4 * n + 1 : 2 * n + 2, tpn = 256 >> (2 * d);
    const int node = (d == 0 ? 0 : d == 1 ? 1 : d == 2 ? 5 : 21) + (tid >> (8 - 2 * d));
    const int j = tid & (tpn - 1);
    if (sh.elig[node] || sh.need[node]) {
      const int x0 = sh.nx0[node], y0 = sh.ny0[node], a = sh.na[node], b = sh.nb[node];
      int16_t* R = sh.refs + ref_offset(node);
      int dcs = 0;
      if (interior) {
        for (int m = j; m < len; m += tpn) {
          // m <= n: p[-1][m] (entry m + 1); m > n: p[m - n - 1][-1] (entry n + m)
          const bool left = m <= n;
          const int x = left ? x0 - 1 : x0 + m - n - 1, y = left ? y0 + m : y0 - 1;
          const int lx = x - cx, ly = y - cy;
          int v;
          if ((unsigned)lx < 64u && (unsigned)ly < 64u) v = sh.cur[ly * 64 + lx];
          else v = jb->cur[(uint32_t)(min(y, jb->h - 1) * stride + min(x, jb->w - 1))];
          R[left ? m + 1 : n + m] = (int16_t)v;
          // DC: p[-1][0..n-1] (m < n) and p[0..n-1][-1] (n < m <= 2n).
          if (m != n && m <= 2 * n) dcs += v;
        }
      } else {
        for (int m = j; m < len; m += tpn) {
          // 1 .. n + 1, then 2n + 1 .. 3n + 1 (planar, DC), or every entry (angular)
          const int off = angular ? m : (m <= n ? m + 1 : n + m);
          int v = 128;
          if (a <= b) {
            const int k = clampi(off <= 2 * n ? 2 * n - off : off, a, b);
            int x, y;
            if (k <= 2 * n) x = x0 - 1, y = y0 - 1 + (2 * n - k);  // left column / corner
            else x = x0 + (k - 2 * n - 1), y = y0 - 1;             // top row
            const int lx = x - cx, ly = y - cy;
            if ((unsigned)lx < 64u && (unsigned)ly < 64u) v = sh.cur[ly * 64 + lx];
            else v = jb->cur[(uint32_t)(min(y, jb->h - 1) * stride + min(x, jb->w - 1))];
          }
          R[off] = (int16_t)v;
          // DC: p[0..n-1][-1] (off 2n+1 .. 3n) and p[-1][0..n-1] (off 1 .. n).
          if ((off >= 1 && off <= n) || (off > 2 * n && off <= 3 * n)) dcs += v;
        }
      }
      const int g = tpn < 64 ? tpn : 64;  // the node's threads within this wavefront
      dcs = (int)group_sum((uint32_t)dcs, g);
      if ((tid & (g - 1)) == 0) atomicAdd(&sh.dc[node], dcs);
    }
  }
  __syncthreads();

  // SATD of every 4x4 tile under every eligible node: thread = tile in Z-order.
  const bool ref_aligned = (((uintptr_t)jb->ref) & 3) == 0;
  const uint32_t frame_bytes = (uint32_t)((jb->h - 1) * stride + jb->w);
  {
    const int t = tid;  // 0..255
    const int tx = (t & 1) | ((t >> 1) & 2) | ((t >> 2) & 4) | ((t >> 3) & 8);
    const int ty = ((t >> 1) & 1) | ((t >> 2) & 2) | ((t >> 3) & 4) | ((t >> 4) & 8);
    int c[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) c[i] = sh.cur[(ty * 4 + (i >> 2)) * 64 + tx * 4 + (i & 3)];
    if (SHARED) {
      // Inter SATDs only, depths (3, 2) and (1, 0) as the low and high halves
      // of one packed transform.
      us2 cp[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) cp[m] = (us2){(unsigned short)c[2 * m], (unsigned short)c[2 * m + 1]};
#pragma unroll
      for (int dp = 0; dp < 2; ++dp) {
        int nd[2];
        sh2 ir[2][8];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int d = 3 - 2 * dp - h, lg = 6 - d;
          const int lx = (tx * 4) >> lg, ly = (ty * 4) >> lg;
          nd[h] = (d == 0 ? 0 : d == 1 ? 1 : d == 2 ? 5 : 21) + ly * (1 << d) + lx;
          if (!jb->subpel && sh.elig[nd[h]]) {
            inter_rows(jb, cx + tx * 4 + sh.mvx[nd[h]], cy + ty * 4 + sh.mvy[nd[h]], cp,
                       ref_aligned, frame_bytes, ir[h]);
          } else {
#pragma unroll
            for (int m = 0; m < 8; ++m) ir[h][m] = (sh2)(0);
          }
        }
        // Per sample: (depth 3 - 2 dp residual, depth 2 - 2 dp residual).
        sh2 pr[16];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const uint32_t a = __builtin_bit_cast(uint32_t, ir[0][2 * j + q]);
            const uint32_t b = __builtin_bit_cast(uint32_t, ir[1][2 * j + q]);
            pr[4 * j + 2 * q] = __builtin_bit_cast(sh2, __builtin_amdgcn_perm(b, a, 0x05040100u));
            pr[4 * j + 2 * q + 1] = __builtin_bit_cast(sh2, __builtin_amdgcn_perm(b, a, 0x07060302u));
          }
        }
        const uint32_t pk = satd4x4_pair(pr);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int d = 3 - 2 * dp - h;
          const int width = 4 << (2 * (3 - d)), w = width > 64 ? 64 : width;
          const uint32_t v = group_sum(h == 0 ? (pk & 0xFFFFu) : (pk >> 16), w);
          if (d > 0) {
            if ((lane & (w - 1)) == 0) sh.satd[nd[h]][0] = v;
          } else if (lane == 0) {
            sh.part0[wave][0] = v;
          }
        }
      }
    } else {
    // The transform is linear and a constant block only moves its (0,0)
    // coefficient (by 16 times the constant), so the DC SATD of this tile at
    // any node follows from the tile's own coefficients: with A = sum |coef|
    // and S = the (0,0) coefficient (>= 0), SATD = (A - S + |S - 16 dc|) / 2.
    int S;
    const int A = hadamard_abs_sum(c, S);
    // The tile's samples in pairs of a row, (c[4 j + 2 q], c[4 j + 2 q + 1]) as
    // 16-bit halves: residuals and the planar prediction are packed 16-bit
    // arithmetic, two samples per operation.
    us2 cp[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) cp[m] = (us2){(unsigned short)c[2 * m], (unsigned short)c[2 * m + 1]};
#pragma unroll
    for (int d = 3; d >= 0; --d) {
      const int n = kCtu >> d, lg = 6 - d;
      const int lx = (tx * 4) >> lg, ly = (ty * 4) >> lg;
      const int node = (d == 0 ? 0 : d == 1 ? 1 : d == 2 ? 5 : 21) + ly * (1 << d) + lx;
      uint32_t v0 = 0, v1 = 0, v2 = 0;
      if (sh.elig[node] || sh.need[node]) {
        // Inter residual (zero with sub-pel refinement: that SATD comes from
        // subres) in the low halves, planar residual in the high halves; both
        // first as pairs of a row's samples (irp, prp), then regrouped per
        // sample into pr.
        sh2 irp[8];
        if (!jb->subpel && sh.elig[node]) {
          inter_rows(jb, cx + tx * 4 + sh.mvx[node], cy + ty * 4 + sh.mvy[node], cp, ref_aligned,
                     frame_bytes, irp);
        } else {
#pragma unroll
          for (int m = 0; m < 8; ++m) irp[m] = (sh2)(0);
        }
        const int16_t* L = sh.refs + ref_offset(node);
        const int16_t* T = L + 2 * n + 1;
        const int px0 = tx * 4 - lx * n, py0 = ty * 4 - ly * n;  // position inside the CU
        // Planar: the horizontal part (n-1-px) L[py+1] + (px+1) T[n] is linear
        // in px along a row and the vertical part (n-1-py) T[px] + (py+1) L[n+1]
        // linear in py along a column.  Both go in pairs of a row's samples:
        // every true value lies in [0, 2^15), so the packed 16-bit sums (mod
        // 2^16) and the unsigned shift are exact.
        const int Tn = T[n], Ln1 = L[n + 1];
        // Vertical parts of columns (0, 1) and (2, 3) at the tile's first row,
        // (n - 1 - py0) T[px] + (py0 + 1) L[n + 1], and their steps per row,
        // L[n + 1] - T[px]: packed multiply-adds (every value below 2^15).
        const us2 t01 = {(unsigned short)T[px0], (unsigned short)T[px0 + 1]};
        const us2 t23 = {(unsigned short)T[px0 + 2], (unsigned short)T[px0 + 3]};
        const us2 kv = (us2)(unsigned short)(n - 1 - py0);
        const us2 cv = (us2)(unsigned short)((py0 + 1) * Ln1), l1 = (us2)(unsigned short)Ln1;
        us2 vp0 = t01 * kv + cv, vp1 = t23 * kv + cv;
        const us2 dv0 = l1 - t01, dv1 = l1 - t23;
        const us2 sh_pl = (us2)(unsigned short)(lg + 1);
        const us2 x01 = {0, 1}, x23 = {2, 3};
        const int hc = (px0 + 1) * Tn + n;
        sh2 pr[16];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          // Horizontal part of row j at columns px0 + i: hr + i dh.
          const int Ly = L[py0 + j + 1];
          const int hr = (n - 1 - px0) * Ly + hc, dh = Tn - Ly;
          const us2 dd = (us2)(unsigned short)dh, hh = (us2)(unsigned short)hr;
          const us2 h0 = dd * x01 + hh, h1 = dd * x23 + hh;
          const us2 p0 = (h0 + vp0) >> sh_pl, p1 = (h1 + vp1) >> sh_pl;
          const uint32_t q0 = __builtin_bit_cast(uint32_t, cp[2 * j] - p0);
          const uint32_t q1 = __builtin_bit_cast(uint32_t, cp[2 * j + 1] - p1);
          const uint32_t i0 = __builtin_bit_cast(uint32_t, irp[2 * j]);
          const uint32_t i1 = __builtin_bit_cast(uint32_t, irp[2 * j + 1]);
          // sample (low half of the inter pair, low half of the planar pair), ...
          pr[4 * j] = __builtin_bit_cast(sh2, __builtin_amdgcn_perm(q0, i0, 0x05040100u));
          pr[4 * j + 1] = __builtin_bit_cast(sh2, __builtin_amdgcn_perm(q0, i0, 0x07060302u));
          pr[4 * j + 2] = __builtin_bit_cast(sh2, __builtin_amdgcn_perm(q1, i1, 0x05040100u));
          pr[4 * j + 3] = __builtin_bit_cast(sh2, __builtin_amdgcn_perm(q1, i1, 0x07060302u));
          vp0 += dv0, vp1 += dv1;
        }
        const uint32_t pk = satd4x4_pair(pr);
        v0 = pk & 0xFFFFu, v1 = pk >> 16;
        const int dcv = (sh.dc[node] + n) >> (lg + 1);
        v2 = (uint32_t)(A - S + abs(S - 16 * dcv)) >> 1;
      }
      // Tiles of a node are consecutive threads: 4^(3-d+1) of them.
      const int width = 4 << (2 * (3 - d));  // 4, 16, 64, 256
      const int w = width > 64 ? 64 : width;
      v0 = group_sum(v0, w), v1 = group_sum(v1, w), v2 = group_sum(v2, w);
      if (d > 0) {
        if ((lane & (w - 1)) == 0) sh.satd[node][0] = v0, sh.satd[node][1] = v1, sh.satd[node][2] = v2;
      } else if (lane == 0) {
        sh.part0[wave][0] = v0, sh.part0[wave][1] = v1, sh.part0[wave][2] = v2;
      }
      if (angular) {
        // Modes 2..34 two at a time (one packed SATD for both); the group's
        // first lane keeps the node's first minimum of J in mode order.
        const bool e = sh.elig[node] != 0;
        const int16_t* L = sh.refs + ref_offset(node);
        const int px0 = tx * 4 - lx * n, py0 = ty * 4 - ly * n;
        int64_t bj = INT64_MAX;
        uint32_t bd = 0;
        int bm = 0;
        for (int ma = 2; ma <= 34; ma += 2) {
          const int mb = ma < 34 ? ma + 1 : ma;
          uint32_t sa = 0, sb = 0;
          if (e) {
            int pa[16], pb[16];
            angular_tile(L, n, ma, px0, py0, pa);
            angular_tile(L, n, mb, px0, py0, pb);
            sh2 pr[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) pr[i] = (sh2){(short)(c[i] - pa[i]), (short)(c[i] - pb[i])};
            const uint32_t pk = satd4x4_pair(pr);
            sa = pk & 0xFFFFu, sb = pk >> 16;
          }
          sa = group_sum(sa, w), sb = group_sum(sb, w);
          if (d == 0) {
            if (lane == 0) {
              sh.ang0[wave][ma - 2] = sa;
              if (mb != ma) sh.ang0[wave][mb - 2] = sb;
            }
          } else {
            const int64_t ja = (int64_t)sa * 65536 + jb->s * (ma == 26 ? 4 : 7);
            if (ja < bj) bj = ja, bd = sa, bm = ma + 1;
            const int64_t jbb = (int64_t)sb * 65536 + jb->s * (mb == 26 ? 4 : 7);
            if (mb != ma && jbb < bj) bj = jbb, bd = sb, bm = mb + 1;
          }
        }
        if (d > 0 && (lane & (w - 1)) == 0)
          sh.angj[node] = bj, sh.angd[node] = bd, sh.angm[node] = (uint8_t)bm;
      }
    }
    }  // !SHARED
  }
  __syncthreads();
  if (angular && tid == 0 && sh.elig[0]) {
    int64_t bj = INT64_MAX;
    uint32_t bd = 0;
    int bm = 0;
    for (int m = 2; m <= 34; ++m) {
      const uint32_t sd = sh.ang0[0][m - 2] + sh.ang0[1][m - 2] + sh.ang0[2][m - 2] +
                          sh.ang0[3][m - 2];
      const int64_t j = (int64_t)sd * 65536 + jb->s * (m == 26 ? 4 : 7);
      if (j < bj) bj = j, bd = sd, bm = m + 1;
    }
    sh.angj[0] = bj, sh.angd[0] = bd, sh.angm[0] = (uint8_t)bm;
  }
  const int64_t s = jb->s;
  if (tid < kNodes) {
    const int node = tid;
    if (node == 0) {
      for (int m = 0; m < 3; ++m)
        sh.satd[0][m] = sh.part0[0][m] + sh.part0[1][m] + sh.part0[2][m] + sh.part0[3][m];
    }
    if (SHARED) {
      // Planar and DC SATDs of the job sharing this current frame.
      const uint32_t* is = jb->intra_src + ((size_t)ctu * kNodes + node) * 2;
      sh.satd[node][1] = is[0], sh.satd[node][2] = is[1];
    } else if (own) {
      uint32_t* io = jb->intra + ((size_t)ctu * kNodes + node) * 2;
      const bool in = sh.need[node] != 0;  // the nodes the other jobs read
      io[0] = in ? sh.satd[node][1] : 0u, io[1] = in ? sh.satd[node][2] : 0u;
    }
  }
  __syncthreads();
  if (tid < kNodes && sh.elig[tid]) {
    const int node = tid;
    // Inter: MV bits of the quarter-pel components (4 x integer MVs without sub-pel).
    const int q = jb->subpel ? 1 : 4;
    const int64_t r_inter = 1 + se_bits_dev(q * sh.mvx[node]) + se_bits_dev(q * sh.mvy[node]);
    const uint32_t si = jb->subpel ? sh.satq[node] : sh.satd[node][0];
    int64_t j = (int64_t)si * 65536 + s * r_inter, dd = si, rr = r_inter;
    uint8_t m = 0;
    const int64_t jp = (int64_t)sh.satd[node][1] * 65536 + s * 3;
    if (jp < j) j = jp, dd = sh.satd[node][1], rr = 3, m = 1;
    const int64_t jd = (int64_t)sh.satd[node][2] * 65536 + s * 4;
    if (jd < j) j = jd, dd = sh.satd[node][2], rr = 4, m = 2;
    if (angular && sh.angj[node] < j)
      j = sh.angj[node], dd = sh.angd[node], rr = sh.angm[node] == 27 ? 4 : 7, m = sh.angm[node];
    sh.lj[node] = j, sh.ld[node] = dd, sh.lr[node] = rr, sh.mode[node] = m;
  } else if (tid < kNodes) {
    // Not eligible: below a node that may not split when it may still be a
    // leaf by the bounds (its value is never used), so any finite value.
    sh.lj[tid] = 0, sh.ld[tid] = 0, sh.lr[tid] = 0, sh.mode[tid] = 0;
  }
  __syncthreads();
  // Bottom-up decision, one depth level at a time.
  for (int d = 3; d >= 0; --d) {
    const int cnt = 1 << (2 * d), base = d == 0 ? 0 : d == 1 ? 1 : d == 2 ? 5 : 21;
    if (tid < cnt) {
      const int node = base + tid;
      const int lx = tid % (1 << d), ly = tid / (1 << d);
      int64_t J = 0, Dd = 0, Rr = 0;
      uint8_t leaf = 0;
      const int k = sh.kind[node];
      int64_t cj = 0, cd = 0, cr = 0;
      if (k != 0 && d < 3) {
        const int cb = d == 0 ? 1 : d == 1 ? 5 : 21;
        for (int q = 0; q < 4; ++q) {
          const int c = cb + (2 * ly + (q >> 1)) * (2 << d) + 2 * lx + (q & 1);
          cj += sh.jt[c], cd += sh.dt[c], cr += sh.rt[c];
        }
      }
      if (k == 1) {
        J = cj, Dd = cd, Rr = cr;
      } else if (k == 2) {
        // An inside node that may be a leaf is eligible unless it cannot be
        // reached (an ancestor may not split); then its value is never used.
        const bool split_ok = sh.split_ok[node], leaf_ok = sh.leaf_ok[node];
        const int flag = d < 3 ? 1 : 0;
        int64_t lj = INT64_MAX;
        if (leaf_ok) lj = sh.lj[node] + s * flag;
        if (split_ok && (!leaf_ok || cj + s < lj)) {
          J = cj + s, Dd = cd, Rr = cr + 1;
        } else {
          J = lj, Dd = sh.ld[node], Rr = sh.lr[node] + flag, leaf = 1;
        }
      }
      sh.jt[node] = J, sh.dt[node] = Dd, sh.rt[node] = Rr, sh.leaf[node] = leaf;
    }
    __syncthreads();
  }
  // Outputs: one thread per 8x8 unit of the CTU.
  if (tid < 64) {
    const int ux = tid & 7, uy = tid >> 3;
    const int x = cx + ux * 8, y = cy + uy * 8;
    if (x < W8 && y < H8) {
      int node = 0, d = 0;
      for (; d < 3; ++d) {
        node = (d == 0 ? 0 : d == 1 ? 1 : 5) + (uy >> (3 - d)) * (1 << d) + (ux >> (3 - d));
        if (sh.leaf[node]) break;
      }
      if (d == 3) node = 21 + uy * 8 + ux;
      const size_t u = (size_t)(y >> 3) * (W8 >> 3) + (x >> 3);
      jb->depth[u] = (uint8_t)d;
      jb->mode[u] = sh.mode[node];
      jb->mv[2 * u] = sh.mvx[node];
      jb->mv[2 * u + 1] = sh.mvy[node];
    }
  }
  if (tid == 0) {
    jb->ctu_cost[ctu] = sh.jt[0];
    jb->ctu_dist[ctu] = sh.dt[0];
    jb->ctu_bits[ctu] = sh.rt[0];
  }
}


// ------------------------------------------------------------------------- depth bounds
// Bounds of dependent unit i (of duw x duh) from the co-located reference unit.
__device__ __forceinline__ void depth_bounds_unit(const uint8_t* __restrict__ ref_depth, int ref_w,
                                                  int ref_h, int dep_w, int dep_h, int dlo,
                                                  int dhi, uint8_t* __restrict__ out, int i) {
  const int duw = (dep_w + 7) >> 3;
  const int ux = i % duw, uy = i / duw;
  const int64_t xr = min((int64_t)(8 * ux + 4) * ref_w / dep_w, (int64_t)ref_w - 1);
  const int64_t yr = min((int64_t)(8 * uy + 4) * ref_h / dep_h, (int64_t)ref_h - 1);
  const int dr = ref_depth[(yr >> 3) * ((ref_w + 7) >> 3) + (xr >> 3)] & 3;
  int ds = 3;
  for (int d = 3; d >= 0; --d)
    if ((int64_t)(64 >> d) * ref_w <= (int64_t)(64 >> dr) * dep_w) ds = d;
  out[2 * i] = (uint8_t)max(0, ds - dlo);
  out[2 * i + 1] = (uint8_t)min(3, ds + dhi);
}

__global__ __launch_bounds__(256) void depth_bounds_kernel(const uint8_t* __restrict__ ref_depth,
                                                           int ref_w, int ref_h, int dep_w,
                                                           int dep_h, int dlo, int dhi,
                                                           uint8_t* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ((dep_w + 7) >> 3) * ((dep_h + 7) >> 3)) return;
  depth_bounds_unit(ref_depth, ref_w, ref_h, dep_w, dep_h, dlo, dhi, out, i);
}

// The bounds of up to kMaxBoundsJobs dependents in one launch: job blockIdx.y.
struct BoundsBatch {
  BoundsJob j[kMaxBoundsJobs];
};
__global__ __launch_bounds__(256) void depth_bounds_batch_kernel(BoundsBatch bb) {
  const BoundsJob& b = bb.j[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ((b.dep_w + 7) >> 3) * ((b.dep_h + 7) >> 3)) return;
  depth_bounds_unit(b.ref_depth, b.ref_w, b.ref_h, b.dep_w, b.dep_h, b.dlo, b.dhi, b.out, i);
}

}  // namespace mr

// Kernels over a batch of jobs (an array of JobDesc in device memory) and their
// launch wrappers.  prep and leaf run one workgroup per CTU of the flattened
// batch; search is one persistent work-queue kernel over (job, strip, band) items.
namespace mr {

// Job owning flattened CTU `flat` (jobs sorted by ctu_start).
__device__ int find_job(cjob jobs, int n_jobs, int flat) {
  int lo = 0, hi = n_jobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].ctu_start <= flat) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void store_job_kernel(JobDesc jb, JobDesc* dst) {
  if (threadIdx.x == 0) *dst = jb;
}

__global__ __launch_bounds__(kPrepThreads) void prep_kernel(const JobDesc* jobs_, int n_jobs, int n_ctus,
                                                   uint32_t* counter) {
  const cjob jobs = (cjob)jobs_;
  const int flat = xcd_contiguous_index();
  if (flat == 0 && threadIdx.x < kQueues) counter[threadIdx.x * kCounterStride] = 0;  // queue heads
  if (flat >= n_ctus) return;
  __shared__ uint32_t csad[64];
  const int j = __builtin_amdgcn_readfirstlane(find_job(jobs, n_jobs, flat));
  prep_ctu(jobs + j, flat - jobs[j].ctu_start, csad);
}

// Persistent search: each workgroup pops items until the queue is empty.  An
// item is a strip of up to `strip` horizontally adjacent CTUs and one dy band;
// the strip's reference window band is staged once in LDS and shared by the
// workgroup's `strip` wavefronts.  The item's (CTU, step) pairs are dealt to
// the wavefronts in equal contiguous shares: one CTU per wavefront for a full
// strip; a partial strip at the right picture edge splits each CTU's steps
// over several wavefronts instead of leaving some idle (partial results merge
// through the same atomic minima as bands do).  items == null: one job, items
// implicit.
//
// Queues: one per XCD, items [qo.off[q], qo.off[q + 1]).  Workgroups are
// dealt to the 8 XCDs round-robin, so a workgroup starts on queue
// blockIdx.x mod 8 (its XCD's): its first item is that queue's item
// blockIdx.x / 8, and the items past the first G_q of queue q (G_q workgroups
// start on it) are popped through the head counter[q].  A workgroup moves on
// to the next queue once its own is empty and ends when all are.  Every item
// is taken exactly once whichever XCD a workgroup runs on.
template <int D>
__device__ __forceinline__ void search_persistent(const JobDesc* jobs_, const uint2* items_,
                                                  const QueueOffsets& qo, uint32_t* counter,
                                                  uint32_t* win, int win_dwords_max) {
  __shared__ int s_item;
  const cjob jobs = (cjob)jobs_;
  const sptr32 items = (sptr32)items_;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wavefront
  const int home = blockIdx.x & (kQueues - 1);
  int empty = 0;  // thread 0: queues found empty, from the home queue on
  bool first = true;
  for (;;) {
    if (threadIdx.x == 0) {
      int it = -1;
      // The first G_q items of queue q (G_q: the workgroups that start on it)
      // are taken without an atomic, one per workgroup; the rest through
      // counter[q].  A queue with no more items than that needs no atomic at
      // all: device-scope atomics on the counters serialise across the XCDs,
      // which in a short launch costs more than the search.
      if (first) {
        first = false;
        const int k = blockIdx.x >> 3;
        if (k < qo.off[home + 1] - qo.off[home]) it = qo.off[home] + k;
      }
      while (it < 0 && empty < kQueues) {
        const int q = (home + empty) & (kQueues - 1);
        const int len = qo.off[q + 1] - qo.off[q];
        const int G = ((int)gridDim.x - q + kQueues - 1) / kQueues;
        uint32_t* head = counter + q * kCounterStride;
        // A head only grows: on the other queues (the end of the launch) a
        // device-scope read that already shows the queue empty saves the atomic.
        if (len > G && (empty == 0 || G + (int)__hip_atomic_load(head, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT) < len)) {
          const int k = G + (int)atomicAdd(head, 1u);
          if (k < len) {
            it = qo.off[q] + k;
            break;
          }
        }
        ++empty;
      }
      s_item = it;
    }
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    if (it < 0) break;  // every wavefront of the workgroup sees the same value
    int job, row, col0, band;
    if (items_) {
      const uint32_t vx = items[2 * it], vy = items[2 * it + 1];
      job = (int)vx, row = (int)(vy >> 16), col0 = (int)((vy >> 4) & 0xFFF), band = (int)(vy & 15);
    } else {
      const int nb = jobs[0].nbands, sw = jobs[0].strip;
      const int spr = (jobs[0].ctus_w + sw - 1) / sw;
      job = 0, band = it % nb;
      const int strip = it / nb;
      row = strip / spr, col0 = (strip % spr) * sw;
    }
    const cjob jb = jobs + job;
    // Window rows of the groups the band's tasks touch.
    const int g0 = jb->band_g0[band];
    const int t_last = min(jb->band_step0[band + 1] * kWaveSteps, jb->ntasks) - 1;
    const int rows = (t_last / jb->Q - g0 + 1) * D + 63;
    const int hs = rows | 1;
    stage_window(jb, col0 * kCtu - jb->R, row * kCtu - jb->R + g0 * D, rows, hs, win);
    __syncthreads();
    // This wavefront's current-CTU ring follows the largest window of the launch.
    uint32_t* ring = win + win_dwords_max + wave * (kCurRingBytes / 4);
    const int nst = jb->band_step0[band + 1] - jb->band_step0[band];
    if (jb->split) {
      // One CTU; the four wavefronts take its quadrants over all the band's
      // steps.  The 64x64 exchange sits at the end of the window area, past
      // this job's window (the plan sizes the area for both).
      search_wave<D, true>(jb, row * jb->ctus_w + col0, band, 0, nst, win, hs, ring, wave,
                           win + win_dwords_max - xch_dwords(D));
    } else {
      const int nw = jb->strip, sw = min(nw, jb->ctus_w - col0);
      int lo = wave * sw * nst / nw;
      const int hi = (wave + 1) * sw * nst / nw;
      while (lo < hi) {
        const int c = lo / nst, s0 = lo - c * nst, s1 = min(nst, s0 + (hi - lo));
        search_wave<D, false>(jb, row * jb->ctus_w + col0 + c, band, s0, s1, win + 16 * c * hs,
                              hs, ring, 0, nullptr);
        lo += s1 - s0;
      }
    }
    __syncthreads();  // the window is restaged for the next item
  }
}

// D = 2, 4: three wavefronts per SIMD (register budget 168); D = 8 keeps its
// larger register file at one or two.
template <int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void search_kernel(
    const JobDesc* jobs_, const uint2* items_, QueueOffsets qo, uint32_t* counter,
    int win_dwords_max) {
  extern __shared__ uint32_t win[];
  search_persistent<D>(jobs_, items_, qo, counter, win, win_dwords_max);
}

__global__ __launch_bounds__(256) void search_kernel_d8(const JobDesc* jobs_, const uint2* items_,
                                                        QueueOffsets qo, uint32_t* counter,
                                                        int win_dwords_max) {
  extern __shared__ uint32_t win[];
  search_persistent<8>(jobs_, items_, qo, counter, win, win_dwords_max);
}

// Job owning CTU `flat` of a leaf launch over the listed jobs (in lctu_start order).
__device__ int find_ljob(cjob jobs, const int* list, int n, int flat) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[list[mid]].lctu_start <= flat) lo = mid;
    else hi = mid - 1;
  }
  return list[lo];
}

// One workgroup per CTU of the launch: every job's CTUs (list null), or, when
// jobs share intra SATDs, two launches with lists of their own: SHARED = false
// over the jobs that take none (those whose SATDs are shared write them),
// SHARED = true over the others.  Each launch deals its own CTUs evenly to the
// XCDs.  At least four wavefronts per SIMD (at most 128 VGPRs): left free, the
// compiler gives the angular form anything from 106 to 226 registers as the
// code around it changes, and at 226 only two workgroups fit a CU.
template <bool ANG, bool SHARED>
__global__ __launch_bounds__(256) void leaf_kernel(const JobDesc* jobs_, const int* list,
                                                   int n_jobs, int n_ctus) {
  __shared__ LeafShared<ANG> sh;
  const cjob jobs = (cjob)jobs_;
  const int flat = xcd_contiguous_index();
  if (flat >= n_ctus) return;
  int j, ctu;
  if (list) {
    j = __builtin_amdgcn_readfirstlane(find_ljob(jobs, list, n_jobs, flat));
    ctu = flat - jobs[j].lctu_start;
  } else {
    j = __builtin_amdgcn_readfirstlane(find_job(jobs, n_jobs, flat));
    ctu = flat - jobs[j].ctu_start;
  }
  leaf_ctu<ANG, SHARED>(jobs, jobs + j, ctu, sh);
}

hipError_t launch_store_job(const JobDesc& jb, JobDesc* dst, hipStream_t st) {
  hipLaunchKernelGGL(store_job_kernel, dim3(1), dim3(64), 0, st, jb, dst);
  return hipGetLastError();
}

hipError_t launch_prep(const JobDesc* jobs, int n_jobs, int n_ctus, uint32_t* counter,
                       hipStream_t st) {
  hipLaunchKernelGGL(prep_kernel, dim3(n_ctus), dim3(kPrepThreads), 0, st, jobs, n_jobs, n_ctus,
                     counter);
  return hipGetLastError();
}

static const void* search_fn(int D) {
  switch (D) {
    case 2: return (const void*)search_kernel<2>;
    case 4: return (const void*)search_kernel<4>;
    case 5: return (const void*)search_kernel<5>;
    case 6: return (const void*)search_kernel<6>;
    case 8: return (const void*)search_kernel_d8;
    default: return nullptr;
  }
}

// Cached per (device, D, strip, LDS bytes): the occupancy query costs tens of
// microseconds of host time, every batch launch asks.  A kernel's dynamic-LDS
// limit (above 64 KB) is only ever raised, so a cached answer stays valid.
int search_occupancy(int D, int strip, size_t lds_bytes) {
  const void* fn = search_fn(D);
  if (!fn) return 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, size_t>, int> cache;
  static std::map<std::pair<int, const void*>, size_t> lds_limit;
  std::lock_guard<std::mutex> lk(mu);
  if (lds_bytes > 64 * 1024) {
    size_t& lim = lds_limit[{dev, fn}];
    if (lds_bytes > lim) {
      if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes) !=
          hipSuccess)
        return 0;
      lim = lds_bytes;
    }
  }
  const auto key = std::make_tuple(dev, D, strip, lds_bytes);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, 64 * strip, lds_bytes) !=
      hipSuccess)
    return 0;
  cache[key] = blocks;
  return blocks;
}

hipError_t launch_search(const JobDesc* jobs, const uint2* items, const QueueOffsets& qoff,
                         int D, int strip, int n_wg, size_t lds_bytes, uint32_t* counter,
                         hipStream_t st) {
  const dim3 grid(n_wg), block(64 * strip);
  // LDS: window (lds_bytes minus the rings) then one ring per wavefront.
  const int win_dwords_max = (int)((lds_bytes - (size_t)kCurRingBytes * strip) / 4);
  switch (D) {
    case 2: hipLaunchKernelGGL(search_kernel<2>, grid, block, lds_bytes, st, jobs, items, qoff, counter, win_dwords_max); break;
    case 4: hipLaunchKernelGGL(search_kernel<4>, grid, block, lds_bytes, st, jobs, items, qoff, counter, win_dwords_max); break;
    case 5: hipLaunchKernelGGL(search_kernel<5>, grid, block, lds_bytes, st, jobs, items, qoff, counter, win_dwords_max); break;
    case 6: hipLaunchKernelGGL(search_kernel<6>, grid, block, lds_bytes, st, jobs, items, qoff, counter, win_dwords_max); break;
    case 8: hipLaunchKernelGGL(search_kernel_d8, grid, block, lds_bytes, st, jobs, items, qoff, counter, win_dwords_max); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_leaf(const JobDesc* jobs, int n_jobs, int n_ctus, bool angular,
                       const int* llist, int n_ljobs0, int n_lctus0, int n_lctus1,
                       hipStream_t st) {
  const int* l0 = llist;
  const int nj0 = llist ? n_ljobs0 : n_jobs, nc0 = llist ? n_lctus0 : n_ctus;
  if (nc0 > 0) {
    if (angular)
      hipLaunchKernelGGL((leaf_kernel<true, false>), dim3(nc0), dim3(256), 0, st, jobs, l0, nj0,
                         nc0);
    else
      hipLaunchKernelGGL((leaf_kernel<false, false>), dim3(nc0), dim3(256), 0, st, jobs, l0, nj0,
                         nc0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (!llist || n_lctus1 <= 0) return hipSuccess;
  hipLaunchKernelGGL((leaf_kernel<false, true>), dim3(n_lctus1), dim3(256), 0, st, jobs,
                     llist + n_ljobs0, n_jobs - n_ljobs0, n_lctus1);
  return hipGetLastError();
}

// A batch's descriptor image passed by value: the kernel copies it from its
// arguments to device memory, one dword per thread.  In the stream's order, as
// a kernel, it starts as soon as the previous kernel ends, where a copy from
// host memory would first go through the copy engine (about 10 us).
struct UploadImage {
  uint32_t w[kUploadMaxBytes / 4];
};

__global__ __launch_bounds__(256) void upload_kernel(UploadImage img, uint32_t* dst, int n_words) {
  for (int i = threadIdx.x; i < n_words; i += 256) dst[i] = img.w[i];
}

hipError_t launch_upload(const uint8_t* img, size_t bytes, uint8_t* dst, hipStream_t st) {
  if (bytes > kUploadMaxBytes || (bytes & 3) != 0) return hipErrorInvalidValue;
  UploadImage u;
  std::memcpy(u.w, img, bytes);
  hipLaunchKernelGGL(upload_kernel, dim3(1), dim3(256), 0, st, u, (uint32_t*)dst,
                     (int)(bytes / 4));
  return hipGetLastError();
}

hipError_t launch_depth_bounds(const uint8_t* ref_depth, int ref_w, int ref_h, int dep_w,
                               int dep_h, int dlo, int dhi, uint8_t* out, hipStream_t st) {
  const int n = ((dep_w + 7) >> 3) * ((dep_h + 7) >> 3);
  hipLaunchKernelGGL(depth_bounds_kernel, dim3((n + 255) / 256), dim3(256), 0, st, ref_depth,
                     ref_w, ref_h, dep_w, dep_h, dlo, dhi, out);
  return hipGetLastError();
}

hipError_t launch_depth_bounds_batch(const BoundsJob* jobs, int n, hipStream_t st) {
  for (int k0 = 0; k0 < n; k0 += kMaxBoundsJobs) {
    const int m = std::min(kMaxBoundsJobs, n - k0);
    BoundsBatch bb{};
    int units = 1;
    for (int k = 0; k < m; ++k) {
      bb.j[k] = jobs[k0 + k];
      units = std::max(units, ((bb.j[k].dep_w + 7) >> 3) * ((bb.j[k].dep_h + 7) >> 3));
    }
    hipLaunchKernelGGL(depth_bounds_batch_kernel, dim3((units + 255) / 256, m), dim3(256), 0, st,
                       bb);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mr

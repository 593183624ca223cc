// HIP kernels of libmr for gfx950 (CDNA4): the seeded search (reference motion
// vectors reused as search centres with a refinement window).
//
// Each CU searches the (2r+1)^2 integer displacements around the scaled MV of
// the reference unit co-located with its centre (clamped to [-(R - r), R - r])
// with the full search's cost and tie order.  Per batch: pad_kernel copies each
// seeded job's reference with a margin and clamped coordinates, so that every
// window load is a plain dword load; refine_kernel then runs one wavefront per
// (CTU, CU depth, pass of 4 NQ + 1 candidate columns, band of window rows) and
// merges the results in the same arg-min keys the full search writes.  The
// prep and leaf kernels are the full search's.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mr_device.h"

namespace mr {

// m * num / den rounded to nearest, halves away from zero (|m| < 2^15,
// 1 <= num <= 8192, 1 <= den <= 32768: every intermediate fits 32 bits).
__device__ __forceinline__ int scale_round_dev(int m, int num, int den) {
  const uint32_t a = (uint32_t)(m < 0 ? -m : m) * (uint32_t)num;
  const int q = (int)((2u * a + (uint32_t)den) / (2u * (uint32_t)den));
  return m < 0 ? -q : q;
}

// Sums of acc[k] over aligned groups of 4^(3-d) lanes (d = 3: none; 2: quads;
// 1: rows of 16; 0: the wavefront), every lane of a group receiving its sum.
// d is uniform; independent DPP adds are interleaved across k.
template <int NP>
__device__ __forceinline__ void group_sums(uint32_t (&acc)[NP], int d) {
  if (d < 3) {
#pragma unroll
    for (int k = 0; k < NP; ++k) acc[k] = add_dpp<0xB1>(acc[k]);  // quad_perm [1,0,3,2]
#pragma unroll
    for (int k = 0; k < NP; ++k) acc[k] = add_dpp<0x4E>(acc[k]);  // quad_perm [2,3,0,1]
  }
  if (d < 2) {
#pragma unroll
    for (int k = 0; k < NP; ++k) acc[k] = add_dpp<0x141>(acc[k]);  // row_half_mirror
#pragma unroll
    for (int k = 0; k < NP; ++k) acc[k] = add_dpp<0x140>(acc[k]);  // row_mirror
  }
  if (d == 0) {
#pragma unroll
    for (int k = 0; k < NP; ++k)
      acc[k] = (uint32_t)(__builtin_amdgcn_readlane((int)acc[k], 0) +
                          __builtin_amdgcn_readlane((int)acc[k], 16) +
                          __builtin_amdgcn_readlane((int)acc[k], 32) +
                          __builtin_amdgcn_readlane((int)acc[k], 48));
  }
}

// Signed Exp-Golomb length of v without a branch on the sign.
__device__ __forceinline__ uint32_t se_len(int v) {
  const uint32_t k = 2u * (uint32_t)(v < 0 ? -v : v) - (v > 0 ? 1u : 0u);
  return 2u * (31u - (uint32_t)__builtin_clz(k + 1u)) + 1u;
}

// A reference row segment of NQ + 3 dwords, re-aligned on this lane's first
// window column (byte sh of raw[0], per lane), as the four byte shifts of its
// first NQ + 1 dwords plus one more plain dword:
// out[o][j] = window bytes 4j + o .. 4j + o + 3 (j = 0..NQ), x = bytes
// 4 NQ + 4 .. 4 NQ + 7.
template <int NQ>
__device__ __forceinline__ void shifts(const uint32_t (&raw)[NQ + 3], int sh,
                                       uint32_t (&out)[4][NQ + 1], uint32_t& x) {
  uint32_t e[NQ + 2];
#pragma unroll
  for (int m = 0; m < NQ + 2; ++m) e[m] = __builtin_amdgcn_alignbyte(raw[m + 1], raw[m], sh);
#pragma unroll
  for (int j = 0; j <= NQ; ++j) {
    out[0][j] = e[j];
#pragma unroll
    for (int o = 1; o < 4; ++o) out[o][j] = __builtin_amdgcn_alignbyte(e[j + 1], e[j], o);
  }
  x = e[NQ + 1];
}

// One wavefront: the CUs of depth d (uniform) of one CTU, one pass of
// NP = 4 NQ + 1 candidate columns, one band of window rows.  Lane b holds the
// 8x8 block at Z-order position b; the lanes of one CU sum their block SADs per
// candidate.
//
// Keys.  The arg-min key J * 2^17 + idx of candidate (dx, dy) is split as
//   T(dx) + SAD * 2^33 + U(dy),  T = s * se(4dx) * 2^17 + dx + R,
//   U = s * se(4dy) * 2^17 + (dy + R) * (2R + 1),
// so a window row is reduced with T alone and U is added once per row
// (s * se < 2^28 and every key < 2^54).
// Columns.  Pass p covers window columns p NP .. p NP + NP - 1.  Every new
// reference row is re-aligned on this lane's first column of the pass (a
// per-lane byte shift), so position k = 4q + o reads the pre-shifted dwords
// S[o][q] and S[o][q + 1], and position 4 NQ reads S[0][NQ] and X.  Columns
// past the window (last pass only, uniform) are skipped or get T = 2^62.
// Rows.  The 8 reference rows of the current dy are a ring of pre-shifted rows
// S[slot][o][j]; step u of a group of 8 uses slot (u + row) & 7 for window row
// `row`, and the row loaded during step u (8 rows below) replaces slot u, which
// step u + 1 no longer needs: the ring turns by renaming, one new row per step,
// loaded one step ahead.
template <int NQ>
__device__ void refine_wave(cjob jb, int ctu, int d, int pass, int band, int nband,
                            uint64_t (*Ts)[64]) {
  constexpr int NP = 4 * NQ + 1, NDW = NQ + 3;
  const int n = kCtu >> d, sh3 = 3 - d;
  const int b = threadIdx.x & 63;
  const int bx = zx(b), by = zy(b);
  const int ctu_x = (ctu % jb->ctus_w) * kCtu, ctu_y = (ctu / jb->ctus_w) * kCtu;
  const int lx = bx >> sh3, ly = by >> sh3;
  const int node = (d == 0 ? 0 : d == 1 ? 1 : d == 2 ? 5 : 21) + ly * (1 << d) + lx;
  const bool e = jb->elig[(size_t)ctu * kNodes + node] != 0;
  if (__ballot(e) == 0) return;  // no CU of this depth may be a leaf

  const int R = jb->R, r = jb->seed_r, lim = R - r, span = 2 * R + 1;
  const int ncand = 2 * r + 1;
  const int rem = ncand - pass * NP;  // window columns left for this pass (uniform)
  if (rem <= 0) return;
  const int bh = (ncand + nband - 1) / nband;
  const int iy0 = band * bh, iy1 = min(ncand, iy0 + bh);
  if (iy0 >= iy1) return;
  const int W = jb->w, H = jb->h;
  // Search centre of this lane's CU (all products < 2^27).
  int cxm, cym;
  {
    const uint32_t px = ctu_x + lx * n + n / 2, py = ctu_y + ly * n + n / 2;
    const uint32_t sw = jb->seed_w, shh = jb->seed_h;
    const uint32_t xr = min(px * sw / (uint32_t)W, sw - 1);
    const uint32_t yr = min(py * shh / (uint32_t)H, shh - 1);
    const int16_t* m = jb->seed_mv + 2 * ((yr >> 3) * ((sw + 7) >> 3) + (xr >> 3));
    const int qs = 2 * jb->seed_qpel;  // quarter-pel maps: 4 map units per pixel
    cxm = clampi(scale_round_dev(m[0], W, sw << qs), -lim, lim);
    cym = clampi(scale_round_dev(m[1], H, shh << qs), -lim, lim);
  }
  // This lane's block (blocks outside the coded picture belong to CUs that are
  // not searched; their loads are kept inside the padded reference).
  const int X0 = min(ctu_x + 8 * bx, jb->w8 - 8), Y0 = min(ctu_y + 8 * by, jb->h8 - 8);
  uint32_t c[16];
  {
    const uint4* cp = (const uint4*)(jb->curpack + (size_t)ctu * 1024 + b * 16);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint4 v = cp[i];
      c[4 * i] = v.x, c[4 * i + 1] = v.y, c[4 * i + 2] = v.z, c[4 * i + 3] = v.w;
    }
  }
  const int pitch = jb->pad_pitch;
  const uint32_t s = (uint32_t)jb->s;
  // This pass's first window column in the padded reference, the dword-aligned
  // column at or left of it and its byte in that dword (0..3, per lane).
  const int xs = X0 + cxm - r + jb->pad_x + pass * NP;
  const int shb = xs & 3;
  // Column key terms, one LDS slot per (position, lane): kept out of the
  // register file, which the ring of pre-shifted rows fills.
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int p = pass * NP + k;  // window column of position k (valid: 0..2r)
    const int dx = cxm - r + p;
    Ts[k][b] = p < ncand ? ((uint64_t)__umul24(s, se_len(4 * dx)) << 17) + (uint64_t)(dx + R)
                         : (1ull << 62);
  }
  const uint32_t* src = (const uint32_t*)(jb->refpad +
                                          (size_t)(Y0 + cym - r + iy0 + jb->pad_y) * pitch +
                                          (xs - shb));
  const int dwp = pitch >> 2;
  uint32_t S[8][4][NQ + 1], X[8];
#pragma unroll
  for (int row = 0; row < 8; ++row) {
    uint32_t raw[NDW];
#pragma unroll
    for (int j = 0; j < NDW; ++j) raw[j] = src[row * dwp + j];
    shifts<NQ>(raw, shb, S[row], X[row]);
  }
  const int nrow = iy1 - iy0;
  uint64_t best = kKeyNone;
  for (int g = 0; g < nrow; g += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = g + u;
      if (t >= nrow) break;
      // Keep each step's loads and shifts in its own step: hoisting them
      // across steps multiplies the live registers.
      __builtin_amdgcn_sched_barrier(0);
      const int dy = cym - r + iy0 + t;
      uint32_t nxt[NDW];
      const bool more = t + 1 < nrow;
      if (more) {
#pragma unroll
        for (int j = 0; j < NDW; ++j) nxt[j] = src[(t + 8) * dwp + j];
      }
      uint32_t acc[NP];
#pragma unroll
      for (int k = 0; k < NP; ++k) acc[k] = 0;
#pragma unroll
      for (int row = 0; row < 8; ++row) {
        const int sl = (u + row) & 7;
        // Every position, also past the window in a partial last pass: its
        // samples are inside the padded reference and its key term is 2^62.
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
#pragma unroll
          for (int o = 0; o < 4; ++o) {
            acc[4 * q + o] = __builtin_amdgcn_sad_u8(c[2 * row], S[sl][o][q], acc[4 * q + o]);
            acc[4 * q + o] =
                __builtin_amdgcn_sad_u8(c[2 * row + 1], S[sl][o][q + 1], acc[4 * q + o]);
          }
        }
        acc[4 * NQ] = __builtin_amdgcn_sad_u8(c[2 * row], S[sl][0][NQ], acc[4 * NQ]);
        acc[4 * NQ] = __builtin_amdgcn_sad_u8(c[2 * row + 1], X[sl], acc[4 * NQ]);
      }
      group_sums<NP>(acc, d);
      uint64_t rb = kKeyNone;
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        const uint64_t key = Ts[k][b] + ((uint64_t)acc[k] << 33);  // >= 2^62 past the window
        rb = key < rb ? key : rb;
      }
      // s < 2^23 and se <= 21, (dy + R) and span <= 257: 24-bit products.
      const uint64_t U = ((uint64_t)__umul24(s, se_len(4 * dy)) << 17) +
                         (uint64_t)__umul24((uint32_t)(dy + R), (uint32_t)span);
      rb += U;
      best = rb < best ? rb : best;
      if (more) shifts<NQ>(nxt, shb, S[u], X[u]);
    }
  }
  // Passes and bands of one CU meet in its key (reset to all ones by prep).
  if (e && (b & ((1 << (2 * sh3)) - 1)) == 0)
    atomicMin((unsigned long long*)&jb->keys[(size_t)ctu * kNodes + node],
              (unsigned long long)best);
}

// Seeded job owning CTU `flat` among the seeded jobs' CTUs (rlist lists the
// seeded jobs in rctu_start order; null: job 0 alone).
__device__ int find_rjob(cjob jobs, const int* rlist, int n_rjobs, int flat) {
  if (!rlist) return 0;
  int lo = 0, hi = n_rjobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[rlist[mid]].rctu_start <= flat) lo = mid;
    else hi = mid - 1;
  }
  return rlist[lo];
}

// Padded reference of every job that has one (seeded or sub-pel): jobs in y,
// rows of each job's [h8 + 2 pad_y][pad_pitch] bytes grid-strided in x, and
// 8-byte pieces of a row over the threads (pad_pitch is a multiple of 8).
__global__ __launch_bounds__(256) void pad_kernel(const JobDesc* jobs_, const int* plist,
                                                  int n_pjobs) {
  for (int k = blockIdx.y; k < n_pjobs; k += gridDim.y) {
    const cjob jb = (cjob)jobs_ + (plist ? plist[k] : 0);
    const int PY = jb->pad_y, w = jb->w, h = jb->h, stride = jb->stride, P = jb->pad_x;
    const int pitch = jb->pad_pitch, rows = jb->h8 + 2 * PY, pieces = pitch >> 3;
    const uint8_t* ref = jb->ref;
    const bool dword_ok = ((stride & 3) == 0) && ((((uintptr_t)ref) & 3) == 0);
    for (int row = blockIdx.x; row < rows; row += gridDim.x) {
      const uint8_t* rp = ref + (size_t)clampi(row - PY, 0, h - 1) * stride;
      uint2* dst = (uint2*)(jb->refpad + (size_t)row * pitch);
      for (int c = threadIdx.x; c < pieces; c += blockDim.x) {
        uint32_t v[2];
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          const int x = 8 * c + 4 * half - P;
          if (dword_ok && x >= 0 && x + 3 < w) {
            v[half] = *(const uint32_t*)(rp + x);
          } else {
            uint32_t u = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) u |= (uint32_t)rp[clampi(x + b, 0, w - 1)] << (8 * b);
            v[half] = u;
          }
        }
        dst[c] = make_uint2(v[0], v[1]);
      }
    }
  }
}

// One single-wavefront workgroup per (CTU, CU depth) in x (depths of a CTU
// adjacent), pass of 4 NQ + 1 candidate columns in y, band of window rows in z.
// NQ = 1 (5 columns) when every job has r <= 2, else 2 (9 columns).
template <int NQ>
__device__ __forceinline__ void refine_body(const JobDesc* jobs_, const int* rlist, int n_rjobs,
                                            int n_rctus) {
  __shared__ uint64_t Ts[4 * NQ + 1][64];
  const cjob jobs = (cjob)jobs_;
  // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous
  // eighth of the (CTU, depth) list so that its L2 holds one band of the
  // frames.  (A bijection on [0, gridDim.x) whatever the dispatch order.)
  // Within its eighth an XCD runs the depth-0 items first and the depth-3
  // items last: a 64x64 CU's cross-lane sums make its wavefront the longest,
  // an 8x8 CU's the shortest, and the last of about three rounds of
  // wavefronts per slot is only partly full.
  const int gx = gridDim.x, x = blockIdx.x;
  const int q = gx >> 3, rm = gx & 7, xcd = x & 7, k = x >> 3;
  const int a = xcd * q + min(xcd, rm), len = q + (xcd < rm ? 1 : 0);  // this XCD's range
  int lin = a, rest = k;
#pragma unroll
  for (int dd = 0; dd < 4; ++dd) {
    const int first = a + ((dd - a) & 3);  // first index >= a of depth dd
    const int cnt = first < a + len ? (a + len - first + 3) >> 2 : 0;
    if (rest >= 0 && rest < cnt) lin = first + 4 * rest;
    rest -= cnt;
  }
  const int flat = lin >> 2, d = lin & 3;
  if (flat >= n_rctus) return;
  const int j = __builtin_amdgcn_readfirstlane(find_rjob(jobs, rlist, n_rjobs, flat));
  refine_wave<NQ>(jobs + j, flat - jobs[j].rctu_start, d, blockIdx.y, blockIdx.z, gridDim.z, Ts);
}

// 5 columns per pass: four wavefronts per SIMD (register budget 128).
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void refine_kernel_q1(
    const JobDesc* jobs_, const int* rlist, int n_rjobs, int n_rctus) {
  refine_body<1>(jobs_, rlist, n_rjobs, n_rctus);
}

// 9 columns per pass: the ring of 8 pre-shifted rows takes 104 registers;
// three wavefronts per SIMD (register budget 168).
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void refine_kernel_q2(
    const JobDesc* jobs_, const int* rlist, int n_rjobs, int n_rctus) {
  refine_body<2>(jobs_, rlist, n_rjobs, n_rctus);
}

hipError_t launch_pad(const JobDesc* jobs, const int* plist, int n_pjobs, int max_rows,
                      hipStream_t st) {
  hipLaunchKernelGGL(pad_kernel, dim3((unsigned)std::max(1, std::min(max_rows, 65535)),
                                      (unsigned)std::min(n_pjobs, 65535)),
                     dim3(256), 0, st, jobs, plist, n_pjobs);
  return hipGetLastError();
}

hipError_t launch_refine(const JobDesc* jobs, const int* rlist, int n_rjobs, int n_rctus,
                         int max_r, hipStream_t st) {
  if ((int64_t)n_rctus * 4 > INT32_MAX) return hipErrorInvalidValue;
  // Grid: (CTU, depth) x passes of 4 NQ + 1 columns x bands of about 10 window rows.
  const int ncand = 2 * max_r + 1;
  const int nq = ncand <= 5 ? 1 : 2;
  const int npass = (ncand + 4 * nq) / (4 * nq + 1);
  const int nband = std::min(8, (ncand + 9) / 10);
  const dim3 grid(4 * n_rctus, npass, nband), block(64);
  if (nq == 1)
    hipLaunchKernelGGL(refine_kernel_q1, grid, block, 0, st, jobs, rlist, n_rjobs, n_rctus);
  else
    hipLaunchKernelGGL(refine_kernel_q2, grid, block, 0, st, jobs, rlist, n_rjobs, n_rctus);
  return hipGetLastError();
}

}  // namespace mr

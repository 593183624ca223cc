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

// Signed Exp-Golomb length of v without a branch on the sign.
__device__ __forceinline__ uint32_t se_len(int v) {
  const uint32_t k = 2u * (uint32_t)(v < 0 ? -v : v) - (v > 0 ? 1u : 0u);
  return 2u * (31u - (uint32_t)__builtin_clz(k + 1u)) + 1u;
}

// A reference row segment of NQ + 3 dwords, re-aligned on this lane's first
// window column (byte sh of raw[0], per lane), as NQ + 1 overlapping dword
// pairs: P[q] = window bytes 4q .. 4q + 7.
template <int NQ>
__device__ __forceinline__ void align_pairs(const uint32_t (&raw)[NQ + 3], int sh,
                                            uint64_t (&P)[NQ + 1]) {
  uint32_t e[NQ + 2];
#pragma unroll
  for (int m = 0; m < NQ + 2; ++m) e[m] = __builtin_amdgcn_alignbyte(raw[m + 1], raw[m], sh);
#pragma unroll
  for (int q = 0; q <= NQ; ++q) P[q] = ((uint64_t)e[q + 1] << 32) | e[q];
}

// The minimum 32-bit key SAD * 2^9 + Kr[k] over a window row's NP = 4 NQ + 1
// candidates, whose block SADs this lane holds as NQ packed quads (16-bit
// fields k = positions 4q + k) and one 32-bit SAD (position 4 NQ).  The SADs
// are first summed over aligned groups of 4^(3-d) lanes (d = 3: none; 2: quads;
// 1: rows of 16; 0: the wavefront) with DPP adds; d is uniform.  A field holds
// an 8x8 SAD (<= 16320) and, after the quad level, a 16x16 SAD (<= 65280):
// below 2^16, so 32-bit adds on two fields are exact.
// For d <= 1, after the quad level the four lanes of a quad hold the same
// sums, so they share the candidates out: lane k (= b & 3) takes positions
// k + 4i (i < NQ) and, if k = 0, position 4 NQ (unpacked to 32 bits, one
// select and one field extract each), with key terms Kl.  Lanes 4 apart hold
// the same positions: rotations by 4 and 8 within the row add the row's
// quads, and for d = 0 the lane-wise swaps of the row pairs and of the halves
// add the rows.  The quad's minimum then covers every position.  Every lane of
// a group ends with the group's minimum.
template <int NQ>
__device__ __forceinline__ uint32_t row_min_key(uint64_t (&aq)[NQ], uint32_t a8, int d,
                                                const uint32_t (&Kr)[4 * NQ + 1], int b,
                                                const uint32_t (&Kl)[NQ + 1]) {
  constexpr int NP = 4 * NQ + 1;
  uint32_t w[2 * NQ + 1];
#pragma unroll
  for (int q = 0; q < NQ; ++q) w[2 * q] = (uint32_t)aq[q], w[2 * q + 1] = (uint32_t)(aq[q] >> 32);
  w[2 * NQ] = a8;
  if (d < 3) {
#pragma unroll
    for (int i = 0; i <= 2 * NQ; ++i) w[i] = add_dpp<0xB1>(w[i]);  // quad_perm [1,0,3,2]
#pragma unroll
    for (int i = 0; i <= 2 * NQ; ++i) w[i] = add_dpp<0x4E>(w[i]);  // quad_perm [2,3,0,1]
  }
  uint32_t m = 0xFFFFFFFFu;
  if (d >= 2) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const uint64_t v = ((uint64_t)w[2 * q + 1] << 32) | w[2 * q];
#pragma unroll
      for (int k = 0; k < 4; ++k) m = min(m, field_mad(v, k, 1u << kRankBitsR, Kr[4 * q + k]));
    }
    m = min(m, (w[2 * NQ] << kRankBitsR) + Kr[4 * NQ]);
  } else {
    const bool first = (b & 3) == 0;
    const uint32_t fsh = (uint32_t)(b & 1) * 16u;
    uint32_t v[NQ + 1];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      // The high dword of the pair for lanes with b & 2 (a lane mask constant):
      // one v_cndmask (written out, so that the choice stays a select of two
      // registers instead of an indexed array).
      uint32_t x;
      asm("v_cndmask_b32_e64 %0, %1, %2, %3"
          : "=v"(x)
          : "v"(w[2 * i]), "v"(w[2 * i + 1]), "s"(0xCCCCCCCCCCCCCCCCull));
      v[i] = (x >> fsh) & 0xFFFFu;
    }
    v[NQ] = first ? w[2 * NQ] : 0u;
#pragma unroll
    for (int i = 0; i <= NQ; ++i) v[i] = add_dpp<0x124>(v[i]);  // row_ror:4
#pragma unroll
    for (int i = 0; i <= NQ; ++i) v[i] = add_dpp<0x128>(v[i]);  // row_ror:8
    if (d == 0) {
#pragma unroll
      for (int i = 0; i <= NQ; ++i) {
        const auto s = __builtin_amdgcn_permlane16_swap(v[i], v[i], false, false);  // rows 0|1, 2|3
        v[i] = s[0] + s[1];
      }
#pragma unroll
      for (int i = 0; i <= NQ; ++i) {
        const auto s = __builtin_amdgcn_permlane32_swap(v[i], v[i], false, false);  // halves
        v[i] = s[0] + s[1];
      }
    }
    // SAD < 2^21: SAD * 2^9 + Kl stays below 2^32, also past the window.
#pragma unroll
    for (int i = 0; i <= NQ; ++i) m = min(m, (v[i] << kRankBitsR) + Kl[i]);
    m = min(m, dpp_mov<0xB1, 0xF>(m, m));  // quad_perm [1,0,3,2]
    m = min(m, dpp_mov<0x4E, 0xF>(m, m));  // quad_perm [2,3,0,1]
  }
  return m;
}

// One wavefront: the CUs of depth d (uniform) of one CTU, one pass of
// NP = 4 NQ + 1 candidate columns, one band of window rows.  Lane b holds the
// 8x8 block at Z-order position b; the lanes of one CU sum their block SADs per
// candidate.
//
// Keys.  A candidate's arg-min key J * 2^17 + idx is
//   (SAD + (c(dx) >> 16)) * 2^33 + rd[rank(dx + R)] + ru[dy + R]
// with the job's tables (c = s * se(4 v); rank orders the columns of the
// whole range by (c & 0xFFFF, dx)), so inside one window row the 32-bit
// (SAD + (c(dx) >> 16)) * 2^9 + rank(dx + R) = SAD * 2^9 + rk[dx + R] orders the
// candidates exactly as their keys do: one shift-add and a minimum per
// candidate, and one 64-bit decode per row.  Columns past the window (last
// pass only, uniform) get rk = 2^31, above every valid row key (< 2^30).
// Columns.  Pass p covers window columns p NP .. p NP + NP - 1.  Every new
// reference row is re-aligned on this lane's first column of the pass (a
// per-lane byte shift) and kept as NQ + 1 dword pairs P[q] (bytes 4q .. 4q + 7).
// One v_qsad_pk_u16_u8 of P[q] and a current dword adds that dword's SADs at
// the 4 byte shifts 4q .. 4q + 3 into 16-bit fields, so positions 0 .. 4 NQ - 1
// take 2 NQ of them per row and position 4 NQ two v_sad_u8.  The ring of 8
// rows then holds 16 (NQ + 1) registers instead of 13 NQ + 8 pre-shifted ones:
// more wavefronts per SIMD.
// Rows.  The 8 reference rows of the current dy are a ring of aligned rows
// P[slot][q]; step u of a group of 8 uses slot (u + row) & 7 for window row
// `row`, and the row loaded during step u (8 rows below) replaces slot u, which
// step u + 1 no longer needs: the ring turns by renaming, one new row per step,
// loaded one step ahead.  A row's two table loads are used one step later.
template <int NQ>
__device__ void refine_wave(cjob jb, int ctu, int d, int pass, int band, int nband,
                            uint32_t (*Ks)[64]) {
  constexpr int NP = 4 * NQ + 1, NDW = NQ + 3;
  const int n = kCtu >> d, sh3 = 3 - d;
  const int b = threadIdx.x & 63;
  const int bx = zx(b), by = zy(b);
  const int ctu_x = (ctu % jb->ctus_w) * kCtu, ctu_y = (ctu / jb->ctus_w) * kCtu;
  const int lx = bx >> sh3, ly = by >> sh3;
  const int node = (d == 0 ? 0 : d == 1 ? 1 : d == 2 ? 5 : 21) + ly * (1 << d) + lx;
  const int R = jb->R, r = jb->seed_r;
  const int ncand = 2 * r + 1;
  const int rem = ncand - pass * NP;  // window columns left for this pass (uniform)
  if (rem <= 0) return;
  const int bh = (ncand + nband - 1) / nband;
  const int iy0 = band * bh, iy1 = min(ncand, iy0 + bh);
  if (iy0 >= iy1) return;
  // The eligibility flags, the search centre of this lane's CU (scaled and
  // clamped by the prep kernel) and the current block are loaded together:
  // the wavefront's first global loads.
  const bool e = jb->elig[(size_t)ctu * kNodes + node] != 0;
  const uint32_t cc = jb->seedc[(size_t)ctu * kNodes + node];
  uint32_t c[16];
  {
    const uint4* cp = (const uint4*)(jb->curpack + (size_t)ctu * 1024 + b * 16);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint4 v = cp[i];
      c[4 * i] = v.x, c[4 * i + 1] = v.y, c[4 * i + 2] = v.z, c[4 * i + 3] = v.w;
    }
  }
  // Consume every load here, so that the compiler keeps them above the exit
  // test (one round of latency instead of three).
  asm volatile("" ::"v"(cc), "v"(c[0]), "v"(c[4]), "v"(c[8]), "v"(c[12]));
  if (__ballot(e) == 0) return;  // no CU of this depth may be a leaf
  const int cxm = (int)(int16_t)(cc & 0xFFFFu), cym = (int)cc >> 16;  // within [r - R, R - r]
  // This lane's block (blocks outside the coded picture belong to CUs that are
  // not searched; their loads are kept inside the padded reference).
  const int X0 = min(ctu_x + 8 * bx, jb->w8 - 8), Y0 = min(ctu_y + 8 * by, jb->h8 - 8);
  const int pitch = jb->pad_pitch;
  const uint32_t* __restrict__ rk = (const uint32_t*)(jb->rtab + kRtabRk);
  const uint64_t* __restrict__ rd = (const uint64_t*)(jb->rtab + kRtabRd);
  const uint64_t* __restrict__ ru = (const uint64_t*)(jb->rtab + kRtabRu);
  // This pass's first window column in the padded reference, the dword-aligned
  // column at or left of it and its byte in that dword (0..3, per lane).
  const int xs = X0 + cxm - r + jb->pad_x + pass * NP;
  const int shb = xs & 3;
  // Column key terms of this lane's positions: in registers for the row minima
  // (Kr), and in LDS (Ks), from where the lanes of a quad take their shares at
  // d <= 1.
  uint32_t Kr[NP];
  if (pass * NP + NP <= ncand) {  // uniform: every column of the pass is in the window
    const uint32_t* kp = rk + (cxm - r + pass * NP + R);  // entries 0..2R
    uint32_t kv[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) kv[k] = kp[k];
#pragma unroll
    for (int k = 0; k < NP; ++k) Ks[k][b] = Kr[k] = kv[k];
  } else {
    // All loads first (indices clamped into the table), then the selects.
    uint32_t kv[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) kv[k] = rk[min(cxm - r + pass * NP + k + R, 2 * R)];
#pragma unroll
    for (int k = 0; k < NP; ++k)  // window column pass NP + k (valid: 0..2r)
      Ks[k][b] = Kr[k] = pass * NP + k < ncand ? kv[k] : 0x80000000u;
  }
  // For d <= 1, the key terms of this lane's share of the positions (this
  // lane's own column of Ks; 2^31 for the slot that lanes k != 0 leave empty).
  uint32_t Kl[NQ + 1];
  if (d <= 1) {
#pragma unroll
    for (int i = 0; i < NQ; ++i) Kl[i] = Ks[(b & 3) + 4 * i][b];
    Kl[NQ] = (b & 3) == 0 ? Ks[4 * NQ][b] : 0x80000000u;
  } else {
#pragma unroll
    for (int i = 0; i <= NQ; ++i) Kl[i] = 0;
  }
  // Window row `row` of this lane: a 32-bit byte offset from the (uniform)
  // padded reference, so that each load is one add and a scalar base.  Rows
  // up to nrow + 7 are read (one past the last band row's ring refill), at
  // most h8 + 2R + 8 < h8 + 2 pad_y padded rows.
  const uint8_t* __restrict__ rp = jb->refpad;
  const uint32_t pitch_u = (uint32_t)pitch;
  const uint32_t off0 = (uint32_t)(Y0 + cym - r + iy0 + jb->pad_y) * pitch_u + (uint32_t)(xs - shb);
  uint64_t P[8][NQ + 1];
#pragma unroll
  for (int row = 0; row < 8; ++row) {
    const uint32_t* s = (const uint32_t*)(rp + (off0 + (uint32_t)row * pitch_u));
    uint32_t raw[NDW];
#pragma unroll
    for (int j = 0; j < NDW; ++j) raw[j] = s[j];
    align_pairs<NQ>(raw, shb, P[row]);
  }
  const int nrow = iy1 - iy0;
  uint64_t best = kKeyNone;
  // The previous row's minimum and its table entries.  Before the first row:
  // a key above every real one (< 2^54) and below kKeyNone.
  uint32_t next_off = off0 + 8u * pitch_u;  // the ring's next row
  uint32_t pm = 0xFFFFFFFFu;
  uint64_t pd = 0, pu = 0;
  for (int g = 0; g < nrow; g += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = g + u;
      if (t >= nrow) break;
      // Keep each step's loads and shifts in its own step: hoisting them
      // across steps multiplies the live registers.
      __builtin_amdgcn_sched_barrier(0);
      const int dy = cym - r + iy0 + t;
      // The ring's next row, loaded unconditionally (also after the band's
      // last row: in bounds, unused) so that the wait for the previous row's
      // table entries need not also wait for it.
      uint32_t nxt[NDW];
      const bool more = t + 1 < nrow;
      {
        const uint32_t* s = (const uint32_t*)(rp + next_off);
        next_off += pitch_u;
#pragma unroll
        for (int j = 0; j < NDW; ++j) nxt[j] = s[j];
      }
      // Every position, also past the window in a partial last pass: its
      // samples are inside the padded reference and its key term is 2^31.
      uint64_t aq[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) aq[q] = 0;
      uint32_t a8 = 0;
#pragma unroll
      for (int row = 0; row < 8; ++row) {
        const int sl = (u + row) & 7;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          aq[q] = __builtin_amdgcn_qsad_pk_u16_u8(P[sl][q], c[2 * row], aq[q]);
          aq[q] = __builtin_amdgcn_qsad_pk_u16_u8(P[sl][q + 1], c[2 * row + 1], aq[q]);
        }
        a8 = __builtin_amdgcn_sad_u8(c[2 * row], (uint32_t)P[sl][NQ], a8);
        a8 = __builtin_amdgcn_sad_u8(c[2 * row + 1], (uint32_t)(P[sl][NQ] >> 32), a8);
      }
      const uint32_t m = row_min_key<NQ>(aq, a8, d, Kr, b, Kl);
      {
        const uint64_t K = ((uint64_t)(pm >> kRankBitsR) << 33) + pd + pu;
        best = K < best ? K : best;
      }
      pm = m;
      // 32-bit byte offsets from the (uniform) tables: one add per load.
      pd = *(const uint64_t*)((const uint8_t*)rd + (m & ((1u << kRankBitsR) - 1)) * 8u);
      pu = *(const uint64_t*)((const uint8_t*)ru + (uint32_t)(dy + R) * 8u);  // dy >= -R
      if (more) align_pairs<NQ>(nxt, shb, P[u]);
    }
  }
  {
    const uint64_t K = ((uint64_t)(pm >> kRankBitsR) << 33) + pd + pu;
    best = K < best ? K : best;
  }
  // Passes and bands of one CU meet in its key (reset to all ones by prep),
  // from the lane that holds the CU's sums: its first lane, lane 63 for d = 0.
  if (e && (d == 0 ? b == 63 : (b & ((1 << (2 * sh3)) - 1)) == 0))
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

// The refinement key tables of a seeded job (layout with kRtabBytes): one
// 256-thread block.  Ranks are counts of smaller (c & 0xFFFF, i) keys, read
// from LDS (the same address in every lane).
__device__ void build_refine_tables(cjob jb) {
  constexpr int NQ4 = (kRtabSpan + 3) / 4;
  __shared__ uint4 key4[NQ4];
  uint32_t* key = (uint32_t*)key4;
  const int R = jb->R, n = 2 * R + 1, nq = (n + 3) >> 2;
  const uint32_t s = (uint32_t)jb->s;
  uint32_t* rk = (uint32_t*)(jb->rtab + kRtabRk);
  uint64_t* rd = (uint64_t*)(jb->rtab + kRtabRd);
  uint64_t* ru = (uint64_t*)(jb->rtab + kRtabRu);
  for (int i = threadIdx.x; i < 4 * nq; i += blockDim.x) {
    if (i < n) {
      const uint32_t c = __umul24(s, se_len(4 * (i - R)));  // s < 2^23, se <= 21
      key[i] = ((c & 0xFFFFu) << kRankBitsR) | (uint32_t)i;  // < 2^25
      ru[i] = ((uint64_t)c << 17) + (uint64_t)(i * n);
    } else {
      key[i] = 0xFFFFFFFFu;  // padding: never below a key
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const uint32_t ki = key[i];
    uint32_t rank = 0;
#pragma unroll 8
    for (int q = 0; q < nq; ++q) {
      const uint4 v = key4[q];
      rank += (v.x < ki ? 1u : 0u) + (v.y < ki ? 1u : 0u) + (v.z < ki ? 1u : 0u) +
              (v.w < ki ? 1u : 0u);
    }
    const uint32_t c = __umul24(s, se_len(4 * (i - R)));
    rk[i] = ((c >> 16) << kRankBitsR) + rank;
    rd[rank] = ((uint64_t)(c & 0xFFFFu) << 17) | (uint64_t)i;
  }
  __syncthreads();
}

// Padded reference of every job that has one (seeded or sub-pel): blocks
// 0 .. n_pjobs - 1 build the seeded jobs' key tables; then one block per row of
// each job's [h8 + 2 pad_y][pad_pitch] bytes, for the jobs that copy their
// reference (a job whose reference another job of the batch pads, same frame
// and margins, shares that copy and has no blocks), with 8-byte pieces of the
// row over the threads (pad_pitch is a multiple of 8).
__global__ __launch_bounds__(256) void pad_kernel(const JobDesc* jobs_, const int* plist,
                                                  int n_pjobs) {
  const cjob jobs = (cjob)jobs_;
  const int b = blockIdx.x;
  if (b < n_pjobs) {  // the first blocks to start build the key tables
    const cjob jb = jobs + (plist ? plist[b] : 0);
    if (jb->seed_mv) build_refine_tables(jb);
    return;
  }
  // Row block r: the padding job whose rows hold r (the last in list order
  // whose first row is at most r: one that pads nothing has the next one's).
  const int r = b - n_pjobs;
  int lo = 0, hi = n_pjobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[plist ? plist[mid] : 0].pad_row_start <= r) lo = mid;
    else hi = mid - 1;
  }
  const cjob jb = jobs + (plist ? plist[lo] : 0);
  const int PY = jb->pad_y, w = jb->w, h = jb->h, stride = jb->stride, P = jb->pad_x;
  const int pitch = jb->pad_pitch, pieces = pitch >> 3, row = r - jb->pad_row_start;
  const uint8_t* ref = jb->ref;
  const bool dword_ok = ((stride & 3) == 0) && ((((uintptr_t)ref) & 3) == 0);
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
        for (int k = 0; k < 4; ++k) u |= (uint32_t)rp[clampi(x + k, 0, w - 1)] << (8 * k);
        v[half] = u;
      }
    }
    dst[c] = make_uint2(v[0], v[1]);
  }
}

// One single-wavefront workgroup per (CTU, CU depth) in x (depths of a CTU
// adjacent), pass of 4 NQ + 1 candidate columns in y, band of window rows in z.
// NQ = 1 (5 columns) when every job has r <= 2, else 2 (9 columns).
template <int NQ>
__device__ __forceinline__ void refine_body(const JobDesc* jobs_, const int* rlist, int n_rjobs,
                                            int n_rctus) {
  __shared__ uint32_t Ks[4 * NQ + 1][64];
  const cjob jobs = (cjob)jobs_;
  // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous
  // eighth of the (CTU, depth) list so that its L2 holds one band of the
  // frames.  (A bijection on [0, gridDim.x) whatever the dispatch order.)
  // Within its eighth an XCD runs the depth-0 items first and the depth-3
  // items last: a 64x64 CU's cross-lane sums make its wavefront the longest,
  // an 8x8 CU's the shortest, so the last wavefronts to start are short.
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
  const int flat = lin >> 2, d = __builtin_amdgcn_readfirstlane(lin & 3);
  if (flat >= n_rctus) return;
  const int j = __builtin_amdgcn_readfirstlane(find_rjob(jobs, rlist, n_rjobs, flat));
  refine_wave<NQ>(jobs + j, flat - jobs[j].rctu_start, d, blockIdx.y, blockIdx.z, gridDim.z, Ks);
}

// 5 columns per pass.
__global__ __launch_bounds__(64) void refine_kernel_q1(const JobDesc* jobs_, const int* rlist,
                                                       int n_rjobs, int n_rctus) {
  refine_body<1>(jobs_, rlist, n_rjobs, n_rctus);
}

// 9 columns per pass: the ring of 8 aligned rows takes 48 registers; four
// wavefronts per SIMD (register budget 128).
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void refine_kernel_q2(
    const JobDesc* jobs_, const int* rlist, int n_rjobs, int n_rctus) {
  refine_body<2>(jobs_, rlist, n_rjobs, n_rctus);
}

hipError_t launch_pad(const JobDesc* jobs, const int* plist, int n_pjobs, int total_rows,
                      hipStream_t st) {
  if (n_pjobs < 1 || total_rows < 0 || (int64_t)n_pjobs + total_rows > INT32_MAX)
    return hipErrorInvalidValue;
  // One block per job (its key tables), then one per padded row of every job
  // that copies its reference.
  hipLaunchKernelGGL(pad_kernel, dim3((unsigned)(n_pjobs + total_rows)), dim3(256), 0, st, jobs,
                     plist, n_pjobs);
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

// HIP kernel of libmr for gfx950 (CDNA4): quarter-pel refinement of every
// CU's integer motion vector (SATD for quarter-pel motion estimation).
//
// Prediction samples follow the H.265 luma fractional-sample interpolation for
// 8-bit video: an 8-tap horizontal filter on the reference samples, an 8-tap
// vertical filter on those sums shifted right by 6, and the default
// uni-prediction rounding (v + 32) >> 6 clipped to 0..255.  Phase 0 uses the
// unit filter (64 at tap 3), which makes integer and one-axis positions the
// same formula.  Per CU: a half-pel stage then a quarter-pel stage, each over
// the current best and its 8 neighbours at the stage's step, J = SATD * 65536 +
// s * (se(qx) + se(qy)), the centre keeping ties, then raster order.
//
// One workgroup (256 threads) per CTU of a sub-pel job; thread t holds the
// 4x4 tile at Z-order position t, so the tiles of one CU are consecutive
// lanes (4, 16, 64 or 256 of them).  For each CU depth a thread loads a 12x12
// patch of the padded reference around its tile at the CU's integer MV, which
// covers both stages (|qx - 4 mx| <= 3), into its own column of an LDS array
// (read back row by row in every horizontal pass).  A stage shares the
// horizontal pass among the 3 candidates of each column and does the vertical
// pass with packed 16-bit dot products; its columns are a loop, not unrolled.
// Patch in LDS and one column's sums live at a time keep the kernel at 168
// registers: three wavefronts per SIMD instead of two.
#include <hip/hip_runtime.h>

#include "mr_device.h"

namespace mr {

// Taps of phase ph as signed bytes, taps 0..3 (lo) and 4..7 (hi), little endian.
__device__ __forceinline__ uint32_t taps8_lo(int ph) {
  return ph == 0 ? 0x40000000u : ph == 1 ? 0x3AF604FFu : ph == 2 ? 0x28F504FFu : 0x11FB0100u;
}
__device__ __forceinline__ uint32_t taps8_hi(int ph) {
  return ph == 0 ? 0x00000000u : ph == 1 ? 0x0001FB11u : ph == 2 ? 0xFF04F528u : 0xFF04F63Au;
}
// Taps of phase ph times 16 as signed 16-bit pairs (2p, 2p + 1), p = 0..3: a
// vertical sum then carries its prediction in its high 16 bits ((16 v) >> 16
// == v >> 12), where one v_perm_b32 packs two candidates' predictions.
__device__ __forceinline__ uint32_t taps16(int ph, int p) {
  const int t0 = (int)(int8_t)(((p < 2 ? taps8_lo(ph) : taps8_hi(ph)) >> (16 * (p & 1))) & 0xFF);
  const int t1 = (int)(int8_t)(((p < 2 ? taps8_lo(ph) : taps8_hi(ph)) >> (16 * (p & 1) + 8)) & 0xFF);
  return ((uint32_t)(16 * t0) & 0xFFFFu) | ((uint32_t)(16 * t1) << 16);
}

typedef short short2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int dot2(uint32_t a, uint32_t b, int c) {
  return __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, a), __builtin_bit_cast(short2_t, b),
                                c, false);
}

// The first product of a dot-product chain, with an inline-constant
// accumulator in the three-operand encoding: the builtins select the
// two-operand form, whose accumulator is its destination, and copy the
// constant into it first.
__device__ __forceinline__ int dot4_plus32(uint32_t a, uint32_t b) {
  int r;
  asm("v_dot4_i32_i8 %0, %1, %2, 32" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Sum over the aligned group of 4^(4-d) tiles of CU depth d (d >= 1: inside one
// wavefront; d = 0: the whole workgroup through red[]).  Every lane of a group
// receives the sum.
__device__ __forceinline__ uint32_t tile_group_sum(uint32_t v, int d, uint32_t* red, int k) {
  v = add_dpp<0xB1>(v);  // quad_perm [1,0,3,2]
  v = add_dpp<0x4E>(v);  // quad_perm [2,3,0,1]
  if (d == 3) return v;
  v = add_dpp<0x141>(v);  // row_half_mirror
  v = add_dpp<0x140>(v);  // row_mirror
  if (d == 2) return v;
  v = (uint32_t)(__builtin_amdgcn_readlane((int)v, 0) + __builtin_amdgcn_readlane((int)v, 16) +
                 __builtin_amdgcn_readlane((int)v, 32) + __builtin_amdgcn_readlane((int)v, 48));
  if (d == 1) return v;
  return v + red[k];  // d == 0: red[k] holds the other wavefronts' sums (see caller)
}

__device__ void subpel_ctu(cjob jb, int ctu) {
  __shared__ uint32_t red[4][9];
  __shared__ uint32_t Ps[12][3][256];  // patch dwords: [row][dword][thread], conflict-free
  const int t = threadIdx.x, wave = t >> 6;
  const int tx = (t & 1) | ((t >> 1) & 2) | ((t >> 2) & 4) | ((t >> 3) & 8);
  const int ty = ((t >> 1) & 1) | ((t >> 2) & 2) | ((t >> 3) & 4) | ((t >> 4) & 8);
  const int ctu_x = (ctu % jb->ctus_w) * kCtu, ctu_y = (ctu / jb->ctus_w) * kCtu;
  // Tiles outside the coded picture belong to CUs that are not refined; their
  // addresses are kept inside the padded reference.
  const int X = min(ctu_x + 4 * tx, jb->w8 - 4), Y = min(ctu_y + 4 * ty, jb->h8 - 4);
  const int R = jb->R, span = 2 * R + 1;
  const uint64_t s = (uint64_t)jb->s;
  // Current tile (coded picture) from the packed CTU: block t >> 2, rows
  // (t >> 1 & 1) * 4 + i, dword t & 1; as sample - 128, like the predictions,
  // in both 16-bit halves (c2) for the packed residuals of two candidates.
  uint32_t c2[16];
  {
    const uint32_t* cp = jb->curpack + (size_t)ctu * 1024 + (t >> 2) * 16 + ((t >> 1) & 1) * 8 +
                         (t & 1);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t w = cp[2 * i] ^ 0x80808080u;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        c2[4 * i + k] = ((uint32_t)(int)(int8_t)((w >> (8 * k)) & 0xFF) & 0xFFFFu) * 0x10001u;
    }
  }
  const int pitch = jb->pad_pitch;
  for (int d = 0; d < 4; ++d) {
    const int sh = 4 - d;  // tile-coordinate shift of a CU of depth d
    const int lx = tx >> sh, ly = ty >> sh;
    const int node = (d == 0 ? 0 : d == 1 ? 1 : d == 2 ? 5 : 21) + ly * (1 << d) + lx;
    const bool e = jb->elig[(size_t)ctu * kNodes + node] != 0;
    // d = 0 is one CU for the whole workgroup (e uniform); d >= 1 stays in a wavefront.
    if (__ballot(e) == 0) continue;
    int mx = 0, my = 0;
    if (e) {
      const int idx = (int)(jb->keys[(size_t)ctu * kNodes + node] & 0x1FFFF);
      my = idx / span - R;
      mx = idx - (my + R) * span - R;
    }
    // 12x12 patch at (X + mx - 4, Y + my - 4), as signed bytes (sample - 128),
    // into this thread's column of Ps (no other thread reads it).
    {
      const int col = X + mx - 4 + jb->pad_x;
      const int sb = col & 3;
      const uint8_t* base = jb->refpad + (size_t)(Y + my - 4 + jb->pad_y) * pitch + (col - sb);
#pragma unroll
      for (int r = 0; r < 12; ++r) {
        const uint32_t* rp = (const uint32_t*)(base + (size_t)r * pitch);
        const uint32_t d0 = rp[0], d1 = rp[1], d2 = rp[2], d3 = rp[3];
        Ps[r][0][t] = __builtin_amdgcn_alignbyte(d1, d0, sb) ^ 0x80808080u;
        Ps[r][1][t] = __builtin_amdgcn_alignbyte(d2, d1, sb) ^ 0x80808080u;
        Ps[r][2][t] = __builtin_amdgcn_alignbyte(d3, d2, sb) ^ 0x80808080u;
      }
    }
    int cqx = 4 * mx, cqy = 4 * my;
    uint32_t csatd = 0, csatd_tile = 0;
#pragma unroll 1
    for (int step = 2; step >= 1; --step) {
      uint32_t sat[9];
#pragma unroll 1
      for (int ix = 0; ix < 3; ++ix) {
        const int qx = cqx + step * (ix - 1);
        const int fx = qx & 3, f = ((qx - fx) >> 2) - mx;  // f in {-1, 0}
        const uint32_t tlo = taps8_lo(fx), thi = taps8_hi(fx);
        // Horizontal pass: h[r][k] for patch rows r = 0..11, tile columns k,
        // taps at patch bytes k + f + 1 .. k + f + 8; packed as 16-bit pairs of
        // consecutive rows Q[r][k] = (h[r][k], h[r + 1][k]).
        //
        // Offsets.  With samples as (sample - 128) each sum is the plain
        // H.265 sum minus 128 * 64; it carries + 32 instead.  Every vertical
        // filter's taps sum to 64, so the vertical sum is the plain one minus
        // 128 * 4096 plus 2048, and the prediction (plain + 2048) >> 12 is that
        // sum >> 12, plus 128.  The horizontal chains start from 32 and the
        // vertical ones from 0, both inline constants.
        const int o = f + 1;  // first tap of column 0 at patch byte o (0 or 1, per lane)
        uint32_t Q[12][4];  // Q[11] = (h[11], 0) pads the vertical window
        int hprev[4];
#pragma unroll
        for (int r = 0; r < 12; ++r) {
          // Patch row r from byte o on: a0 = bytes 0..3, a1 = 4..7, a2 = 8..10 (+1 unused).
          const uint32_t p0 = Ps[r][0][t], p1 = Ps[r][1][t], p2 = Ps[r][2][t];
          const uint32_t a0 = __builtin_amdgcn_alignbyte(p1, p0, o);
          const uint32_t a1 = __builtin_amdgcn_alignbyte(p2, p1, o);
          const uint32_t a2 = __builtin_amdgcn_alignbyte(p2, p2, o);
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const uint32_t lo = k == 0 ? a0 : __builtin_amdgcn_alignbyte(a1, a0, k);
            const uint32_t hi = k == 0 ? a1 : __builtin_amdgcn_alignbyte(a2, a1, k);
            const int h = __builtin_amdgcn_sdot4((int)lo, (int)tlo, dot4_plus32(hi, thi), false);
            // (low halves of) hprev | h << 16 in one v_perm_b32
            if (r > 0) Q[r - 1][k] = __builtin_amdgcn_perm((uint32_t)h, (uint32_t)hprev[k], 0x05040100u);
            hprev[k] = h;
          }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) Q[11][k] = (uint32_t)hprev[k] & 0xFFFFu;
        // Vertical pass of candidate row iy (qy = cqy + step (iy - 1)): its
        // per-lane taps, then per tile sample a sum v, 16 times the plain H.265
        // sum minus 128 * 4096 plus 2048, so that v >> 16 is the prediction -
        // 128 before clipping (((v >> 6) + 32) >> 6 == (v + 2048) >> 12 for the
        // plain sum, arithmetic shifts).
        auto vtaps = [&](int iy, uint32_t tw[5]) {
          const int qy = cqy + step * (iy - 1);
          const int fy = qy & 3, g = ((qy - fy) >> 2) - my;  // g in {-1, 0}
          // Filter tap j applies to patch row i + g + 1 + j.  Over the window
          // of rows i .. i + 9 (pairs Q[i + 2p], p = 0..4) that is window tap
          // j + g + 1: the taps move by one row for g = 0 instead of the rows.
          uint32_t prev = 0;
#pragma unroll
          for (int p = 0; p < 5; ++p) {
            const uint32_t cur = p < 4 ? taps16(fy, p) : 0u;
            tw[p] = g == 0 ? __builtin_amdgcn_alignbyte(cur, prev, 2) : cur;
            prev = cur;
          }
        };
        auto vsum = [&](const uint32_t tw[5], int i, int k) {
          int v = 0;
#pragma unroll
          for (int p = 0; p < 5; ++p) v = dot2(Q[i + 2 * p][k], tw[p], v);
          return v;
        };
        // The quarter-pel stage's centre is the half-pel stage's best, whose
        // SATD is already known.  The first two candidates of the column share
        // one packed 16-bit transform.
        const bool centre_known = step == 1 && ix == 1;
        {
          uint32_t ta[5], tb[5];
          vtaps(0, ta);
          vtaps(centre_known ? 2 : 1, tb);
          sh2 pr[16];
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int va = vsum(ta, i >> 2, i & 3), vb = vsum(tb, i >> 2, i & 3);
            // (va >> 16, vb >> 16) as 16-bit halves, clipped, subtracted from the sample
            sh2 p = __builtin_bit_cast(sh2, __builtin_amdgcn_perm((uint32_t)vb, (uint32_t)va,
                                                                  0x07060302u));
            p = __builtin_elementwise_min(__builtin_elementwise_max(p, (sh2)(-128)), (sh2)(127));
            pr[i] = __builtin_bit_cast(sh2, c2[i]) - p;
          }
          const uint32_t pk = satd4x4_pair(pr);
          sat[ix] = pk & 0xFFFFu;
          if (centre_known) sat[6 + ix] = pk >> 16;
          else sat[3 + ix] = pk >> 16;
        }
        if (centre_known) {
          sat[4] = csatd_tile;
        } else {
          uint32_t tc[5];
          vtaps(2, tc);
          int rc[16];
#pragma unroll
          for (int i = 0; i < 16; ++i)
            rc[i] = (int)(short)c2[i] - clampi(vsum(tc, i >> 2, i & 3) >> 16, -128, 127);
          sat[6 + ix] = satd4x4(rc);
        }
      }
      const uint32_t tile_sat[9] = {sat[0], sat[1], sat[2], sat[3], sat[4], sat[5], sat[6],
                                    sat[7], sat[8]};
      // Sum each candidate's SATD over the CU's tiles.
      if (d == 0) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          uint32_t v = add_dpp<0xB1>(sat[k]);
          v = add_dpp<0x4E>(v);
          v = add_dpp<0x141>(v);
          v = add_dpp<0x140>(v);
          v = (uint32_t)(__builtin_amdgcn_readlane((int)v, 0) + __builtin_amdgcn_readlane((int)v, 16) +
                         __builtin_amdgcn_readlane((int)v, 32) + __builtin_amdgcn_readlane((int)v, 48));
          if ((t & 63) == 0) red[wave][k] = v;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 9; ++k) sat[k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
        __syncthreads();  // red is reused by the next stage
      } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) sat[k] = tile_group_sum(sat[k], d, nullptr, 0);
      }
      // First minimum: the centre, then the 8 neighbours in raster order.
      int bk = 4;
      uint64_t bj = (uint64_t)sat[4] * 65536 + s * (uint64_t)(se_bits_dev(cqx) + se_bits_dev(cqy));
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        if (k == 4) continue;
        const int qx = cqx + step * (k % 3 - 1), qy = cqy + step * (k / 3 - 1);
        const uint64_t j = (uint64_t)sat[k] * 65536 + s * (uint64_t)(se_bits_dev(qx) + se_bits_dev(qy));
        if (j < bj) bj = j, bk = k;
      }
      cqx += step * (bk % 3 - 1);
      cqy += step * (bk / 3 - 1);
      csatd = sat[bk];
      // This tile's share of the best candidate's SATD (the next stage's centre).
      csatd_tile = tile_sat[0];
#pragma unroll
      for (int k = 1; k < 9; ++k) csatd_tile = bk == k ? tile_sat[k] : csatd_tile;
    }
    const int gsz = 1 << (2 * (4 - d));  // tiles per CU
    if (e && (t & (gsz - 1)) == 0) {
      uint32_t* o = jb->subres + ((size_t)ctu * kNodes + node) * 2;
      o[0] = ((uint32_t)cqx & 0xFFFFu) | ((uint32_t)cqy << 16);
      o[1] = csatd;
    }
  }
}

// Sub-pel job owning CTU `flat` among the sub-pel jobs' CTUs (slist: those jobs
// in sctu_start order; null: job 0 alone).
__device__ int find_sjob(cjob jobs, const int* slist, int n_sjobs, int flat) {
  if (!slist) return 0;
  int lo = 0, hi = n_sjobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[slist[mid]].sctu_start <= flat) lo = mid;
    else hi = mid - 1;
  }
  return slist[lo];
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void subpel_kernel(
    const JobDesc* jobs_, const int* slist, int n_sjobs, int n_sctus) {
  const cjob jobs = (cjob)jobs_;
  const int flat = xcd_contiguous_index();
  if (flat >= n_sctus) return;
  const int j = __builtin_amdgcn_readfirstlane(find_sjob(jobs, slist, n_sjobs, flat));
  subpel_ctu(jobs + j, flat - jobs[j].sctu_start);
}

hipError_t launch_subpel(const JobDesc* jobs, const int* slist, int n_sjobs, int n_sctus,
                         hipStream_t st) {
  hipLaunchKernelGGL(subpel_kernel, dim3(n_sctus), dim3(256), 0, st, jobs, slist, n_sjobs,
                     n_sctus);
  return hipGetLastError();
}

}  // namespace mr

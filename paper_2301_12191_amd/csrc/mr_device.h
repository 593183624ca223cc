// Device helpers shared by the HIP kernels of libmr (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mr_internal.h"

namespace mr {

typedef const __attribute__((address_space(4))) uint32_t* sptr32;  // scalar (uniform) loads
typedef const __attribute__((address_space(4))) JobDesc* cjob;     // job descriptor, scalar loads

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Workgroups are dealt round-robin to the 8 XCDs: this maps blockIdx.x to an
// index such that each XCD takes a contiguous eighth of [0, gridDim.x), so
// neighbouring CTUs share one L2 (a bijection whatever the dispatch order).
__device__ __forceinline__ int xcd_contiguous_index() {
  const int gx = gridDim.x, x = blockIdx.x;
  const int q = gx >> 3, rm = gx & 7, xcd = x & 7, k = x >> 3;
  return xcd * q + min(xcd, rm) + k;
}

// m * num / den rounded to nearest, halves away from zero (|m| < 2^15,
// 1 <= num <= 8192, 1 <= den <= 32768: every intermediate fits 32 bits).
__device__ __forceinline__ int scale_round_dev(int m, int num, int den) {
  const uint32_t a = (uint32_t)(m < 0 ? -m : m) * (uint32_t)num;
  const int q = (int)((2u * a + (uint32_t)den) / (2u * (uint32_t)den));
  return m < 0 ? -q : q;
}

// Z-order (Morton) position -> (x, y) for 6-bit indices.
__device__ __forceinline__ int zx(int z) { return (z & 1) | ((z >> 1) & 2) | ((z >> 2) & 4); }
__device__ __forceinline__ int zy(int z) { return ((z >> 1) & 1) | ((z >> 2) & 2) | ((z >> 3) & 4); }

template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t old, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWMASK, 0xF, false);
}

// Bits of the signed Exp-Golomb code of v.
__device__ __forceinline__ int se_bits_dev(int v) {
  const uint32_t k = v > 0 ? 2u * (uint32_t)v - 1u : 2u * (uint32_t)(-v);
  return 2 * (31 - __builtin_clz(k + 1u)) + 1;
}

// Field k (0..3) of four packed 16-bit values, times m (< 2^16, uniform), plus
// a: one v_mad_u32_u16 whose op_sel picks the high half of the dword holding
// the field, instead of an extract and a multiply-add.
__device__ __forceinline__ uint32_t field_mad(uint64_t v, int k, uint32_t m, uint32_t a) {
  const uint32_t x = (uint32_t)(v >> (32 * (k >> 1)));
  uint32_t r;
  if (k & 1)
    asm("v_mad_u32_u16 %0, %1, %2, %3 op_sel:[1,0,0,0]" : "=v"(r) : "v"(x), "s"(m), "v"(a));
  else
    asm("v_mad_u32_u16 %0, %1, %2, %3" : "=v"(r) : "v"(x), "s"(m), "v"(a));
  return r;
}

// v plus the value of another lane (DPP permutation CTRL) in one v_add_u32.
template <int CTRL>
__device__ __forceinline__ uint32_t add_dpp(uint32_t v) {
  return v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

// max(|a|, |b|) = max(a, b, -a, -b) = max(a, b, -min(a, b)): a min, a
// negation and a three-input max instead of two absolute values and a max.
__device__ __forceinline__ int max_abs2(int a, int b) { return max(max(a, b), -min(a, b)); }

// SATD of a 4x4 residual: sum |H d H^T| / 2 via butterflies.  The last
// column stage is folded into |x + y| + |x - y| = 2 max(|x|, |y|).
__device__ __forceinline__ uint32_t satd4x4(const int d[16]) {
  int t[16];
#pragma unroll
  for (int i = 0; i < 4; ++i) {  // rows
    const int a0 = d[4 * i] + d[4 * i + 1], a1 = d[4 * i] - d[4 * i + 1];
    const int a2 = d[4 * i + 2] + d[4 * i + 3], a3 = d[4 * i + 2] - d[4 * i + 3];
    t[4 * i] = a0 + a2, t[4 * i + 1] = a1 + a3, t[4 * i + 2] = a0 - a2, t[4 * i + 3] = a1 - a3;
  }
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {  // columns
    const int a0 = t[j] + t[4 + j], a1 = t[j] - t[4 + j];
    const int a2 = t[8 + j] + t[12 + j], a3 = t[8 + j] - t[12 + j];
    s += max_abs2(a0, a2) + max_abs2(a1, a3);
  }
  return s;
}

// Two 4x4 residuals at once in packed 16-bit lanes (v_pk_* ops).  Row then
// column butterflies; the last column stage is folded into
// |x + y| + |x - y| = 2 max(|x|, |y|), so each half returns sum |H d H^T| / 2
// directly.  Residuals within +-255 keep every intermediate within +-2040 and
// each half's result within 16320.
typedef short sh2 __attribute__((ext_vector_type(2)));
typedef unsigned short us2 __attribute__((ext_vector_type(2)));

// max(|a|, |b|) per 16-bit half, as max(max(a, b), -min(a, b)): four packed
// operations instead of five.
__device__ __forceinline__ sh2 pk_max_abs2(sh2 a, sh2 b) {
  return __builtin_elementwise_max(__builtin_elementwise_max(a, b),
                                   (sh2)(0) - __builtin_elementwise_min(a, b));
}

__device__ __forceinline__ uint32_t satd4x4_pair(const sh2 d[16]) {
  sh2 t[16];
#pragma unroll
  for (int i = 0; i < 4; ++i) {  // rows
    const sh2 a0 = d[4 * i] + d[4 * i + 1], a1 = d[4 * i] - d[4 * i + 1];
    const sh2 a2 = d[4 * i + 2] + d[4 * i + 3], a3 = d[4 * i + 2] - d[4 * i + 3];
    t[4 * i] = a0 + a2, t[4 * i + 1] = a1 + a3, t[4 * i + 2] = a0 - a2, t[4 * i + 3] = a1 - a3;
  }
  sh2 s = (sh2)(0);
#pragma unroll
  for (int j = 0; j < 4; ++j) {  // columns
    const sh2 a0 = t[j] + t[4 + j], a1 = t[j] - t[4 + j];
    const sh2 a2 = t[8 + j] + t[12 + j], a3 = t[8 + j] - t[12 + j];
    s += pk_max_abs2(a0, a2) + pk_max_abs2(a1, a3);
  }
  return __builtin_bit_cast(uint32_t, s);  // low half: d.x residual, high half: d.y
}

// sum |H c H^T| over all 16 coefficients of a 4x4 block and its (0,0)
// coefficient S (the sum of the block), with the same folded last stage.
__device__ __forceinline__ int hadamard_abs_sum(const int c[16], int& S) {
  int t[16];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int a0 = c[4 * i] + c[4 * i + 1], a1 = c[4 * i] - c[4 * i + 1];
    const int a2 = c[4 * i + 2] + c[4 * i + 3], a3 = c[4 * i + 2] - c[4 * i + 3];
    t[4 * i] = a0 + a2, t[4 * i + 1] = a1 + a3, t[4 * i + 2] = a0 - a2, t[4 * i + 3] = a1 - a3;
  }
  int m = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int a0 = t[j] + t[4 + j], a1 = t[j] - t[4 + j];
    const int a2 = t[8 + j] + t[12 + j], a3 = t[8 + j] - t[12 + j];
    m += max_abs2(a0, a2) + max_abs2(a1, a3);
    if (j == 0) S = a0 + a2;
  }
  return 2 * m;
}

}  // namespace mr

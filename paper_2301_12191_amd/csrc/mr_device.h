// Device helpers shared by the HIP kernels of libmr (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mr_internal.h"

namespace mr {

typedef const __attribute__((address_space(4))) uint32_t* sptr32;  // scalar (uniform) loads
typedef const __attribute__((address_space(4))) JobDesc* cjob;     // job descriptor, scalar loads

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

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

}  // namespace mr

// bfloat16 helpers of the matrix-core kernels (v_mfma_f32_32x32x16_bf16:
// lane l supplies A[l % 32][8 (l / 32) .. 8 (l / 32) + 7] and
// B[8 (l / 32) .. + 7][l % 32] of a K = 16 step, eight bfloat16 each; the
// sixteen accumulators of lane l hold D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]).
#pragma once
#include "common.hpp"

namespace cc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Round to the nearest bfloat16 (ties to even); NaN stays NaN.
__device__ __forceinline__ uint16_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_f(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ float round_bf16(float f) { return bf16_f(bf16_bits(f)); }

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}
__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }
__device__ __forceinline__ f32x16 mfma_bf16(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

}  // namespace cc

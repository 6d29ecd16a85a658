// Shared device-side definitions of the gfx950 Cool-chic kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cc {

constexpr int MAXL = 7;          // latent levels supported
constexpr int UPS_K = 8;         // taps of each 1-D stride-2 transposed conv
constexpr int UPS_P = UPS_K / 2 - 1;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Latent-pyramid geometry: level l is lh[l] x lw[l], starting at loff[l] in
// the packed buffer.
struct Geo {
  int H, W, L;
  int n_lat;
  int lh[MAXL + 1], lw[MAXL + 1], loff[MAXL + 1];
};

// Quantisation proxy: 0 = round half to even (straight-through gradient),
// 1 = additive noise y + u, 2 = values used as given (already quantised).
__device__ __forceinline__ float quantise(const float* __restrict__ y, const float* __restrict__ u, int q,
                                          int mode) {
  float v = y[q];
  if (mode == 0) return __builtin_rintf(v);
  if (mode == 1) return v + u[q];
  return v;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Wave-local ordering of LDS traffic: stops the compiler from moving LDS
// accesses across it and waits for this wave's outstanding LDS operations, so
// that data one lane wrote is visible to the other lanes of the same wave.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// D = A x B + C with A 32x2, B 2x32 (one float per lane each), 16 accumulators.
// Lane l supplies A[l%32][l/32] and B[l/32][l%32]; accumulator r of lane l is
// D[8*(r/4) + 4*(l/32) + r%4][l%32].
__device__ __forceinline__ f32x16 mfma32x32x2(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
// D = A x B + C with A 16x4, B 4x16; lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator r of lane l is D[4*(l/16) + r][l%16].
__device__ __forceinline__ f32x4 mfma16x16x4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row index, within a 32-row MFMA block, of accumulator r of a lane in half g.
__device__ __forceinline__ constexpr int dfeat(int r, int g) { return 8 * (r >> 2) + 4 * g + (r & 3); }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ __forceinline__ bool finitef(float v) { return __builtin_isfinite(v); }

// One work-group of a batched launch: the image whose argument block it
// uses, its block index and the block count of that image's share, and a
// kernel-specific extra index.
struct WorkItem {
  int img, bid, nblk, aux;
};

}  // namespace cc

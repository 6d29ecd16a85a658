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

// Soft rounding (Agustsson & Theis 2020) of sharpness a: floor(x) + 1/2 +
// tanh(a r) / (2 tanh(a/2)), r = x - floor(x) - 1/2, and its derivative.
__device__ __forceinline__ float soft_round(float x, float a) {
  const float fl = floorf(x);
  return fl + 0.5f + tanhf(a * (x - fl - 0.5f)) / (2.0f * tanhf(0.5f * a));
}
__device__ __forceinline__ float soft_round_grad(float x, float a) {
  const float t = tanhf(a * (x - floorf(x) - 0.5f));
  return a * (1.0f - t * t) / (2.0f * tanhf(0.5f * a));
}

// Quantisation proxy: 0 = round half to even (straight-through gradient),
// 1 = additive noise y + u, 2 = values used as given (already quantised),
// 3 = C3's proxy s(s(y) + u), s the soft rounding of sharpness alpha (read
// by each kernel from u[N_lat]).
constexpr int QMODE_SOFT = 3;
__device__ __forceinline__ bool uses_noise(int mode) { return mode == 1 || mode == QMODE_SOFT; }

__device__ __forceinline__ float quantise_raw(float yv, float uv, int mode, float alpha = 0.0f) {
  if (mode == 0) return __builtin_rintf(yv);
  if (mode == 1) return yv + uv;
  if (mode == QMODE_SOFT) return soft_round(soft_round(yv, alpha) + uv, alpha);
  return yv;
}

__device__ __forceinline__ float quantise(const float* __restrict__ y, const float* __restrict__ u, int q, int mode,
                                          float alpha = 0.0f) {
  return quantise_raw(y[q], uses_noise(mode) ? u[q] : 0.0f, mode, alpha);
}

// dy_hat / dy of the proxy (1 except for the soft one).
__device__ __forceinline__ float quantise_grad(float yv, float uv, int mode, float alpha) {
  if (mode != QMODE_SOFT) return 1.0f;
  return soft_round_grad(soft_round(yv, alpha) + uv, alpha) * soft_round_grad(yv, alpha);
}

// The soft proxy's sharpness, stored after the noise of the N_lat latents.
__device__ __forceinline__ float proxy_alpha(const float* __restrict__ u, int mode, int n_lat) {
  return mode == QMODE_SOFT ? u[n_lat] : 0.0f;
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

// Fills n LDS values (n <= NQ * NT): store(p, load(p)) for p = tid, tid + NT,
// ..., with every global read of the thread issued before its first LDS
// write (a plain loop would wait for each read in turn).
template <int NQ, int NT, typename Load, typename Store>
__device__ __forceinline__ void batched_stage(int tid, int n, Load load, Store store) {
  float r[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int p = tid + NT * q;
    r[q] = p < n ? load(p) : 0.0f;
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int p = tid + NT * q;
    if (p < n) store(p, r[q]);
  }
}

// Stages n values of a latent stack into LDS the same way: for p, src(p)
// gives (idx, plane): plane < 0 reads the latent y[idx] (quantised with
// mode; the noise u[idx] is read too in mode 1), plane >= 0 the float
// planes[idx] (already a stack channel).  All reads first, then the writes.
template <int NQ, int NT, typename Src, typename Store>
__device__ __forceinline__ void batched_stage_stack(int tid, int n, const float* __restrict__ y,
                                                    const float* __restrict__ u, int mode, float alpha,
                                                    const float* __restrict__ planes, Src src, Store store) {
  float ry[NQ], ru[NQ];
  bool lat[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int p = tid + NT * q;
    ry[q] = 0.0f;
    ru[q] = 0.0f;
    lat[q] = false;
    if (p < n) {
      int idx;
      bool is_lat;
      src(p, idx, is_lat);
      lat[q] = is_lat;
      if (is_lat) {
        ry[q] = y[idx];
        if (uses_noise(mode)) ru[q] = u[idx];
      } else {
        ry[q] = planes[idx];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int p = tid + NT * q;
    if (p < n) store(p, lat[q] ? quantise_raw(ry[q], ru[q], mode, alpha) : ry[q]);
  }
}

// Causal neighbour sets (dy, dx), raster order: the C positions of the 7x7
// window that precede the latent, nearest first (ties in raster order).
// (compile-time tables: with the loops over k unrolled, every offset is an
// immediate)
template <int C>
__device__ __forceinline__ constexpr int ctx_dy(int k) {
  constexpr signed char t8[8] = {-2, -2, -2, -1, -1, -1, 0, 0};
  constexpr signed char t16[16] = {-3, -3, -3, -2, -2, -2, -2, -2, -1, -1, -1, -1, -1, 0, 0, 0};
  constexpr signed char t24[24] = {-3, -3, -3, -3, -3, -3, -3, -2, -2, -2, -2, -2,
                                   -2, -2, -1, -1, -1, -1, -1, -1, -1, 0,  0,  0};
  return C == 8 ? t8[k] : (C == 16 ? t16[k] : t24[k]);
}
template <int C>
__device__ __forceinline__ constexpr int ctx_dx(int k) {
  constexpr signed char t8[8] = {-1, 0, 1, -1, 0, 1, -2, -1};
  constexpr signed char t16[16] = {-1, 0, 1, -2, -1, 0, 1, 2, -2, -1, 0, 1, 2, -3, -2, -1};
  constexpr signed char t24[24] = {-3, -2, -1, 0, 1, 2, 3, -3, -2, -1, 0, 1, 2, 3, -3, -2, -1, 0, 1, 2, 3, -3, -2, -1};
  return C == 8 ? t8[k] : (C == 16 ? t16[k] : t24[k]);
}

// One work-group of a batched launch: the image whose argument block it
// uses, its block index and the block count of that image's share, and a
// kernel-specific extra index.
struct WorkItem {
  int img, bid, nblk, aux;
};

}  // namespace cc

// Laplace rate of one latent and its derivatives (device, float32).
#pragma once

#include "common.hpp"

namespace cc {

// Clamp range of the log-scale s (scale b = exp(s) in [0.01, 100]).
constexpr float LOG_SCALE_MIN = -4.605170186f;  // ln 0.01
constexpr float LOG_SCALE_MAX = 4.605170186f;   // ln 100
constexpr float INV_LN2 = 1.4426950408889634f;

struct Rate {
  float r;   // -log2 P(y_hat), bits
  float dd;  // dr/dd with d = y_hat - mu  (so dr/dy_hat = dd, dr/dmu = -dd)
  float ds;  // dr/ds, zero where s is outside the clamp range
};

// Rate of the Laplace(mu, b) mass over [y_hat - 1/2, y_hat + 1/2],
// b = exp(clamp(s)).  With d = y_hat - mu, x = |d| - 1/2:
//  |d| >= 1/2 : P = (1/2) e^{-x/b} (1 - e^{-1/b})
//               r = x / (b ln2) + 1 - log2(1 - e^{-1/b})
//               dr/dd = sign(d) / (b ln2)
//               dr/ds = (1/b) (1 / (e^{1/b} - 1) - x) / ln2
//  |d| <  1/2 : with A = e^{-(1/2 + d)/b}, B = e^{-(1/2 - d)/b},
//               P = 1 - (A + B)/2 = -(expm1(-(1/2+d)/b) + expm1(-(1/2-d)/b)) / 2
//               dr/dd = -(A - B) / (2 b P ln2)
//               dr/ds = (A (1/2 + d) + B (1/2 - d)) / (2 b P ln2)
// Both branches agree at |d| = 1/2 (value and d-derivative).
//
// Evaluated with the hardware base-2 exponential, logarithm and reciprocal;
// e^t - 1 for |t| < 1/4 comes from its Taylor series to t^7 (relative error
// below 1e-8 there), so that 1 - e^{-1/b} and P keep full relative precision
// for wide scales.  Over |y_hat - mu| <= 20 and s in [-7, 7] the rate is
// within 7e-6 bits of the exact value below 100 bits (FP32 resolution above).
constexpr float LOG2E_F = 1.4426950408889634f;

__device__ __forceinline__ float exp_hw(float t) { return __builtin_amdgcn_exp2f(t * LOG2E_F); }

__device__ __forceinline__ float expm1_hw(float t) {
  const float p =
      t * __builtin_fmaf(t, __builtin_fmaf(t, __builtin_fmaf(t, __builtin_fmaf(t, __builtin_fmaf(t, __builtin_fmaf(
                                  t, 1.0f / 5040.0f, 1.0f / 720.0f), 1.0f / 120.0f), 1.0f / 24.0f), 1.0f / 6.0f), 0.5f), 1.0f);
  return fabsf(t) < 0.25f ? p : exp_hw(t) - 1.0f;
}

template <bool GRAD>
__device__ __forceinline__ Rate laplace_rate(float yq, float mu, float s) {
  const bool inside = (s >= LOG_SCALE_MIN) && (s <= LOG_SCALE_MAX);
  const float sc = fminf(fmaxf(s, LOG_SCALE_MIN), LOG_SCALE_MAX);
  const float ib = exp_hw(-sc);  // 1 / b
  const float d = yq - mu;
  const float ad = fabsf(d);
  Rate o;
  if (ad >= 0.5f) {
    const float x = ad - 0.5f;
    const float E = -expm1_hw(-ib);  // 1 - e^{-1/b}
    o.r = x * ib * INV_LN2 + 1.0f - __builtin_amdgcn_logf(E);
    if (GRAD) {
      o.dd = copysignf(ib * INV_LN2, d);
      o.ds = inside ? ib * (__builtin_amdgcn_rcpf(expm1_hw(ib)) - x) * INV_LN2 : 0.0f;
    }
  } else {
    const float ma = expm1_hw(-(0.5f + d) * ib), mb = expm1_hw(-(0.5f - d) * ib);  // A - 1, B - 1
    const float P = -0.5f * (ma + mb);
    o.r = -__builtin_amdgcn_logf(P);
    if (GRAD) {
      const float k = 0.5f * ib * INV_LN2 * __builtin_amdgcn_rcpf(P);
      o.dd = -(ma - mb) * k;
      o.ds = inside ? ((1.0f + ma) * (0.5f + d) + (1.0f + mb) * (0.5f - d)) * k : 0.0f;
    }
  }
  if (!GRAD) { o.dd = 0.0f; o.ds = 0.0f; }
  return o;
}

}  // namespace cc

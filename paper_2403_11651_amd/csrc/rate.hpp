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
template <bool GRAD>
__device__ __forceinline__ Rate laplace_rate(float yq, float mu, float s) {
  const bool inside = (s >= LOG_SCALE_MIN) && (s <= LOG_SCALE_MAX);
  const float sc = fminf(fmaxf(s, LOG_SCALE_MIN), LOG_SCALE_MAX);
  const float ib = expf(-sc);  // 1 / b
  const float d = yq - mu;
  const float ad = fabsf(d);
  Rate o;
  if (ad >= 0.5f) {
    const float x = ad - 0.5f;
    const float E = -expm1f(-ib);  // 1 - e^{-1/b}
    o.r = x * ib * INV_LN2 + 1.0f - log2f(E);
    if (GRAD) {
      o.dd = copysignf(ib * INV_LN2, d);
      o.ds = inside ? ib * (1.0f / expm1f(ib) - x) * INV_LN2 : 0.0f;
    }
  } else {
    const float ea = -(0.5f + d) * ib, eb = -(0.5f - d) * ib;
    const float A = expf(ea), B = expf(eb);
    const float P = -0.5f * (expm1f(ea) + expm1f(eb));
    o.r = (P > 0.5f) ? -log1pf(-0.5f * (A + B)) * INV_LN2 : -log2f(P);
    if (GRAD) {
      const float k = 0.5f * ib * INV_LN2 / P;
      o.dd = -(A - B) * k;
      o.ds = inside ? (A * (0.5f + d) + B * (0.5f - d)) * k : 0.0f;
    }
  }
  if (!GRAD) { o.dd = 0.0f; o.ds = 0.0f; }
  return o;
}

}  // namespace cc

// Quantisation of the decoder parameters, for gfx950 (Section II: after the
// encoding the network parameters are quantised and entropy coded with an
// ad-hoc probability model).  Each module (ARM, upsampling, synthesis) sits
// on a grid of step 2^-k: q = rint(theta 2^k), theta_hat = q 2^-k (both exact
// in float32).  Its rate is the sum of -log2 of the Laplace(0, b) mass of
// every q over [q - 1/2, q + 1/2], with b = max(mean |q|, 0.01) (the
// maximum-likelihood scale of the block).  One work-group per module; sums in
// a fixed order.
#include "common.hpp"
#include "kernels.hpp"

namespace cc {

namespace {

__device__ float block_sum_256(float v, float* s_tmp) {
  const int tid = threadIdx.x;
  s_tmp[tid] = v;
  __syncthreads();
  for (int stride = 128; stride >= 1; stride >>= 1) {
    if (tid < stride) s_tmp[tid] += s_tmp[tid + stride];
    __syncthreads();
  }
  const float out = s_tmp[0];
  __syncthreads();
  return out;
}

// -log2 of the Laplace(0, b) mass over [q - 1/2, q + 1/2] (q an integer):
// q = 0: -log2(1 - e^(-1/(2b))); |q| >= 1: (|q| - 1/2) / (b ln 2) + 1 -
// log2(1 - e^(-1/b)).
__device__ __forceinline__ float param_bits(float q, float b) {
  const float aq = fabsf(q);
  if (aq == 0.0f) return -log2f(-expm1f(-0.5f / b));
  return (aq - 0.5f) / (b * 0.6931471805599453f) + 1.0f - log2f(-expm1f(-1.0f / b));
}

}  // namespace

__global__ __launch_bounds__(256) void param_quant_kernel(ParamQArgs a) {
  __shared__ float s_tmp[256];
  const int m = blockIdx.x, tid = threadIdx.x, n = a.n[m];
  const float* __restrict__ src = a.src[m];
  float* __restrict__ dst = a.dst[m];
  const float up = ldexpf(1.0f, a.k[m]), down = ldexpf(1.0f, -a.k[m]);
  float sabs = 0.0f;
  for (int i = tid; i < n; i += 256) {
    const float q = __builtin_rintf(src[i] * up);
    sabs += fabsf(q);
  }
  sabs = block_sum_256(sabs, s_tmp);
  const float b = n > 0 ? fmaxf(sabs / (float)n, PARAM_B_MIN) : PARAM_B_MIN;
  float bits = 0.0f;
  for (int i = tid; i < n; i += 256) {
    const float q = __builtin_rintf(src[i] * up);
    bits += param_bits(q, b);
    dst[i] = q * down;  // after every read of src[i] (dst may alias src)
  }
  bits = block_sum_256(bits, s_tmp);
  if (tid == 0) a.bits[m] = n > 0 ? bits : 0.0f;
}

}  // namespace cc

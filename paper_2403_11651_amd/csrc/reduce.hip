// Deterministic reductions of per-block partials, the loss of Eq. (1), and the
// Adam update.  Every sum runs in a fixed order, so results are bit-identical
// from run to run.
#include "common.hpp"
#include "kernels.hpp"

namespace cc {

// Column sums of several [rows][ld] partial matrices: 16 columns per block,
// 16 row groups per column combined in fixed order.
__global__ __launch_bounds__(256) void reduce_cols_kernel(ReduceArgs a) {
  __shared__ float s_p[RED_RG][RED_COLS];
  const int tid = threadIdx.x, cl = tid % RED_COLS, rg = tid / RED_COLS;
  const int gc = blockIdx.x * RED_COLS + cl;
  int sg = -1;
  for (int k = 0; k < a.nseg; ++k)
    if (gc >= a.col_start[k] && gc < a.col_start[k + 1]) sg = k;
  float acc = 0.0f;
  if (sg >= 0) {
    const RedSeg& S = a.seg[sg];
    const int col = gc - a.col_start[sg];
    for (int r = rg; r < S.rows; r += RED_RG) acc += S.src[(size_t)r * S.ld + col];
  }
  s_p[rg][cl] = acc;
  __syncthreads();
  bool bad = false;
  if (rg == 0 && sg >= 0) {
    float v = 0.0f;
    for (int k = 0; k < RED_RG; ++k) v += s_p[k][cl];
    a.seg[sg].dst[gc - a.col_start[sg]] = v;
    bad = !finitef(v);
  }
  const bool any = __syncthreads_or(bad);
  if (tid == 0) a.flags[blockIdx.x] = any ? 1.0f : 0.0f;
}

__device__ float block_sum_fixed(const float* src, int n, float* s_tmp) {
  const int tid = threadIdx.x;
  float acc = 0.0f;
  for (int i = tid; i < n; i += 256) acc += src[i];
  s_tmp[tid] = acc;
  __syncthreads();
  for (int stride = 128; stride >= 1; stride >>= 1) {
    if (tid < stride) s_tmp[tid] += s_tmp[tid + stride];
    __syncthreads();
  }
  const float v = s_tmp[0];
  __syncthreads();
  return v;
}

// loss4 = {D + lambda R / (HW), D, R, non-finite flag} (Eq. (1); D = SSE / 3HW).
__global__ __launch_bounds__(256) void finalize_kernel(FinalArgs a) {
  __shared__ float s_tmp[256];
  const float R = a.have_rate ? block_sum_fixed(a.rpart, a.nr, s_tmp) : 0.0f;
  const float sse = a.have_sse ? block_sum_fixed(a.spart, a.ns, s_tmp) : 0.0f;
  const float fl = a.nflags ? block_sum_fixed(a.flags, a.nflags, s_tmp) : 0.0f;
  if (threadIdx.x == 0) {
    const float D = sse * a.inv_3hw;
    const float L = D + a.lambda * R * a.inv_hw;
    a.loss4[0] = L;
    a.loss4[1] = D;
    a.loss4[2] = R;
    a.loss4[3] = (fl > 0.0f || !finitef(L) || !finitef(D) || !finitef(R)) ? 1.0f : 0.0f;
  }
}

// Adam (Kingma & Ba) with bias correction; t = step[0] + 1.
__global__ __launch_bounds__(256) void adam_kernel(AdamArgs a) {
  const int t = a.step[0] + 1;
  const float bc1 = 1.0f - powf(a.beta1, (float)t);
  const float bc2 = 1.0f - powf(a.beta2, (float)t);
  const float k1 = 1.0f / bc1, k2 = 1.0f / bc2;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * 256) {
    const float g = a.g[i];
    const float m = a.beta1 * a.m[i] + (1.0f - a.beta1) * g;
    const float v = a.beta2 * a.v[i] + (1.0f - a.beta2) * g * g;
    a.m[i] = m;
    a.v[i] = v;
    a.theta[i] -= a.lr * (m * k1) / (sqrtf(v * k2) + a.eps);
  }
}

// Advances the step counter after the update kernel has read it.
__global__ void adam_advance_kernel(int32_t* step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) step[0] += 1;
}

}  // namespace cc

// Deterministic reductions of per-block partials, the loss of Eq. (1), and the
// Adam update.  Every sum runs in a fixed order, so results are bit-identical
// from run to run.
#include "common.hpp"
#include "kernels.hpp"

namespace cc {

// Adam (Kingma & Ba) on one value with the bias corrections k1 = 1 / (1 -
// beta1^t), k2 = 1 / (1 - beta2^t); every kernel that updates parameters
// uses these two functions, so fused and separate updates agree bit for bit.
__device__ __forceinline__ void adam_coeffs(float beta1, float beta2, int t, float& k1, float& k2) {
  k1 = 1.0f / (1.0f - powf(beta1, (float)t));
  k2 = 1.0f / (1.0f - powf(beta2, (float)t));
}
__device__ __forceinline__ void adam_apply(float lr, float beta1, float beta2, float eps, float k1, float k2,
                                           float& th, float g, float& m, float& v) {
  // explicit FMAs: the rounding does not depend on how the caller inlines it
  m = __builtin_fmaf(beta1, m, (1.0f - beta1) * g);
  v = __builtin_fmaf(beta2, v, (1.0f - beta2) * g * g);
  th = __builtin_fmaf(-lr, (m * k1) / (sqrtf(v * k2) + eps), th);
}

// g_y[q] += sum of the extended-frame gradients of every ARM tile whose frame
// contains latent q (own tile, left / right neighbours, and the three tiles of
// the next tile row), in fixed order; with the fused Adam, the latent is then
// updated from that gradient.
template <typename AD>
__device__ bool arm_fold_one(const FoldArgs& a, int q, const AD& ad, float k1, float k2) {
  if (q >= a.q1) return true;
  int l = 0;
  while (l + 1 < a.geo.L && q >= a.geo.loff[l + 1]) ++l;
  const int wl = a.geo.lw[l], local = q - a.geo.loff[l];
  const int i = local / wl, j = local % wl;
  const int ti = i / ARM_TH, tj = j / ARM_TW;
  // all six candidate frames are read at once (0 where the tile does not
  // exist or its frame misses q), then added in fixed order
  float f[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int ta = ti + k / 3, tb = tj + k % 3 - 1;
    const int fa = i - (ta * ARM_TH - 3), fb = j - (tb * ARM_TW - 3);
    const bool ok = ta < a.tiles.nth[l] && tb >= 0 && tb < a.tiles.ntw[l] && fa >= 0 && fa < ARM_EH && fb >= 0 &&
                    fb < ARM_EW;
    const int tile = a.tiles.base[l] + ta * a.tiles.ntw[l] + tb;
    f[k] = ok ? a.gext[(size_t)tile * ARM_EXT + fa * ARM_EW + fb] : 0.0f;
  }
  const float gy = a.g_y[q];
  float th = 0.0f, m = 0.0f, vv = 0.0f;
  if (ad.on) { th = a.th[q]; m = a.m[q]; vv = a.v[q]; }
  float G = 0.0f;
#pragma unroll
  for (int k = 0; k < 6; ++k) G += f[k];
  float v = gy + G;
  // the gradient so far is w.r.t. y_hat; the soft proxy's derivative takes it to y
  if (a.quant == QMODE_SOFT) v *= quantise_grad(a.y[q], a.u[q], a.quant, a.u[a.geo.n_lat]);
  a.g_y[q] = v;
  if (ad.on) {
    adam_apply(ad.lr, ad.beta1, ad.beta2, ad.eps, k1, k2, th, v, m, vv);
    a.th[q] = th; a.m[q] = m; a.v[q] = vv;
  }
  return finitef(v);
}

// Three block sums in one pass: each thread adds its strided share of every
// array in index order (the loads of a share are issued together), then one
// fixed tree per array.
__device__ void block_sum3(const float* const src[3], const int n[3], float* s_tmp, float out[3]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float acc = 0.0f;
#pragma unroll 8
    for (int i = tid; i < n[k]; i += 256) acc += src[k][i];
    s_tmp[k * 256 + tid] = acc;
  }
  __syncthreads();
  for (int stride = 128; stride >= 1; stride >>= 1) {
    if (tid < stride) {
#pragma unroll
      for (int k = 0; k < 3; ++k) s_tmp[k * 256 + tid] += s_tmp[k * 256 + tid + stride];
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) out[k] = s_tmp[k * 256];
}

// loss4 = {D + lambda R / (HW), D, R, non-finite flag} (Eq. (1); D = SSE / 3HW).
__device__ __forceinline__ void finalize_body(const FinalArgs& a) {
  __shared__ float s_tmp[3 * 256];
  const float* const src[3] = {a.rpart, a.spart, a.flags};
  const int n[3] = {a.have_rate ? a.nr : 0, a.have_sse ? a.ns : 0, a.nflags};
  float sums[3];
  block_sum3(src, n, s_tmp, sums);
  const float R = sums[0], sse = sums[1], fl = sums[2];
  if (threadIdx.x == 0) {
    // explicit rounding steps, so that every kernel built from this body
    // (single image or batched) computes the loss the same way
    const float D = sse * a.inv_3hw;
    const float L = __builtin_fmaf(a.lambda * R, a.inv_hw, D);
    a.loss4[0] = L;
    a.loss4[1] = D;
    a.loss4[2] = R;
    const bool bad = fl > 0.0f || !finitef(L) || !finitef(D) || !finitef(R);
    if (bad || !a.sticky) a.loss4[3] = bad ? 1.0f : 0.0f;
  }
}

// Column sums of [rows][ld] partial matrices, and the ARM fold (see
// CombineArgs).  A reduction block owns cpb columns of one segment; its
// 256 / cpb row groups each sum a strided set of rows, then a fixed-order
// tree combines the row groups.
__device__ __forceinline__ void combine_body(const CombineArgs& a, const int bid) {
  __shared__ float s_p[256];
  const int tid = threadIdx.x;
  if (bid == a.loss_block) {
    finalize_body(a.fin);
    return;
  }
  float k1 = 0.0f, k2 = 0.0f;
  if (a.adam.on) {
    const int t = *a.adam.t_slot;
    adam_coeffs(a.adam.beta1, a.adam.beta2, t, k1, k2);
    if (a.adam.store_step && bid == 0 && tid == 0) *a.adam.step = t;
  }
  const int n_red = a.block_start[a.nseg];
  bool bad = false;
  if (bid >= n_red) {
    bad = !arm_fold_one(a.fold, a.fold.q0 + (bid - n_red) * 256 + tid, a.adam, k1, k2);
  } else {
    int sg = 0;
    while (sg + 1 < a.nseg && bid >= a.block_start[sg + 1]) ++sg;
    const RedSeg& S = a.seg[sg];
    const int cpb = S.cpb, ngroups = 256 / cpb;
    const int cl = tid % cpb, rg = tid / cpb;
    const int col = (bid - a.block_start[sg]) * cpb + cl;
    float acc = 0.0f;
    if (col < S.cols) {
#pragma unroll 4
      for (int r = rg; r < S.rows; r += ngroups) acc += S.src[(size_t)r * S.ld + col];
    }
    s_p[tid] = acc;
    __syncthreads();
    for (int stride = ngroups / 2; stride >= 1; stride >>= 1) {
      if (rg < stride) s_p[tid] += s_p[tid + stride * cpb];
      __syncthreads();
    }
    if (rg == 0 && col < S.cols) {
      const float v = s_p[cl];
      S.dst[col] = v;
      bad = !finitef(v);
      if (a.adam.on && S.th) {
        float th = S.th[col], m = S.m[col], vv = S.v[col];
        adam_apply(a.adam.lr, a.adam.beta1, a.adam.beta2, a.adam.eps, k1, k2, th, v, m, vv);
        S.th[col] = th; S.m[col] = m; S.v[col] = vv;
      }
    }
  }
  const bool any = __syncthreads_or(bad);
  if (tid == 0) {
    if (a.flags) a.flags[bid] = any ? 1.0f : 0.0f;
    else if (any) *a.bad = 1.0f;
  }
}
__global__ __launch_bounds__(256) void combine_kernel(CombineArgs a) { combine_body(a, blockIdx.x); }
__global__ __launch_bounds__(256) void combine_kernel_batch(const CombineArgs* __restrict__ d,
                                                            const WorkItem* __restrict__ w) {
  const WorkItem it = w[blockIdx.x];
  combine_body(d[it.img], it.bid);
}

__global__ __launch_bounds__(256) void finalize_kernel(FinalArgs a) { finalize_body(a); }

// Adam (Kingma & Ba) with bias correction; t = step[0] + 1.  Every block reads
// step[0] before it adds itself to the completion counter step[1]; the block
// that completes the count advances step[0] and clears the counter, so the
// next launch sees the new step.  VEC: all four arrays are 16-byte aligned
// and are read and written four values at a time.
__device__ __forceinline__ void adam_one(const AdamArgs& a, float k1, float k2, float& th, float g, float& m,
                                         float& v) {
  adam_apply(a.lr, a.beta1, a.beta2, a.eps, k1, k2, th, g, m, v);
}

template <bool VEC>
__global__ __launch_bounds__(256) void adam_kernel(AdamArgs a) {
  const int t = a.step[0] + 1;
  float k1, k2;
  adam_coeffs(a.beta1, a.beta2, t, k1, k2);
  const int64_t stride = (int64_t)gridDim.x * 256, first = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int64_t done = 0;
  if (VEC) {
    // ADAM_U float4 groups per thread and pass, all loads issued before any
    // store (the four arrays do not overlap)
    const int64_t n4 = a.n / 4;
    float4* __restrict__ th4 = reinterpret_cast<float4*>(a.theta);
    const float4* __restrict__ g4 = reinterpret_cast<const float4*>(a.g);
    float4* __restrict__ m4 = reinterpret_cast<float4*>(a.m);
    float4* __restrict__ v4 = reinterpret_cast<float4*>(a.v);
    const int64_t base = (int64_t)blockIdx.x * 256 * ADAM_U + threadIdx.x;
    for (int64_t i0 = base; i0 < n4; i0 += stride * ADAM_U) {
      float4 th[ADAM_U], g[ADAM_U], m[ADAM_U], v[ADAM_U];
#pragma unroll
      for (int u = 0; u < ADAM_U; ++u) {
        const int64_t i = i0 + u * 256;
        if (i < n4) { th[u] = th4[i]; g[u] = g4[i]; m[u] = m4[i]; v[u] = v4[i]; }
      }
#pragma unroll
      for (int u = 0; u < ADAM_U; ++u) {
        const int64_t i = i0 + u * 256;
        if (i < n4) {
          adam_one(a, k1, k2, th[u].x, g[u].x, m[u].x, v[u].x);
          adam_one(a, k1, k2, th[u].y, g[u].y, m[u].y, v[u].y);
          adam_one(a, k1, k2, th[u].z, g[u].z, m[u].z, v[u].z);
          adam_one(a, k1, k2, th[u].w, g[u].w, m[u].w, v[u].w);
          m4[i] = m[u];
          v4[i] = v[u];
          th4[i] = th[u];
        }
      }
    }
    done = n4 * 4;
  }
  for (int64_t i = done + first; i < a.n; i += stride) {
    float th = a.theta[i], m = a.m[i], v = a.v[i];
    adam_one(a, k1, k2, th, a.g[i], m, v);
    a.m[i] = m;
    a.v[i] = v;
    a.theta[i] = th;
  }
  if (threadIdx.x == 0) {
    const int prev = atomicAdd(&a.step[1], 1);  // after this block's read of step[0] (t is used above)
    if (prev == (int)gridDim.x - 1) {
      atomicExch(&a.step[0], t);
      atomicExch(&a.step[1], 0);
    }
  }
}
template __global__ void adam_kernel<true>(AdamArgs);
template __global__ void adam_kernel<false>(AdamArgs);

}  // namespace cc

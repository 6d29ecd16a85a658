// Upsampling f_upsilon kernels for gfx950 (Section II "Decoding"; Table I
// "TConv", stride 2).
//
// stack_{L-1} = y_hat_{L-1}; stack_s = [y_hat_s, U_s(stack_{s+1})].  U_s is a
// stride-2 transposed convolution with 8 taps per axis, applied as the outer
// product of a vertical and a horizontal kernel, with input indices clamped
// to the grid (replicate border):
//     out[i][j] = sum_{ky, kx} v[ky] h[kx] in[clamp((i+3-ky)/2)][clamp((j+3-kx)/2)]
// over the taps with (i+3-ky) and (j+3-kx) even (4 x 4 taps per output).
// The step s = 0 is fused into the synthesis kernels; these kernels produce
// the steps s >= 1 and the adjoint of every step.
#include "common.hpp"
#include "kernels.hpp"

namespace cc {

__global__ __launch_bounds__(256) void ups_fwd_kernel(UpsFwdArgs a) {
  const int s = a.s, L = a.geo.L;
  const int h = a.geo.lh[s], w = a.geo.lw[s], hi = a.geo.lh[s + 1], wi = a.geo.lw[s + 1];
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= h * w) return;
  const int i = idx / w, j = idx % w;
  int ro[4], co[4];
  float vt[4], ht[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int ky = 2 * q + 1 - (i & 1), kx = 2 * q + 1 - (j & 1);
    ro[q] = clampi((i + UPS_P - ky) >> 1, 0, hi - 1);
    co[q] = clampi((j + UPS_P - kx) >> 1, 0, wi - 1);
    vt[q] = a.taps[ky];
    ht[q] = a.taps[UPS_K + kx];
  }
  const int nch = L - 1 - s;  // channels of stack_{s+1}
  const int lo = a.geo.loff[s + 1];
  float acc = 0.0f;
#pragma unroll
  for (int q1 = 0; q1 < 4; ++q1) {
    float ra = 0.0f;
#pragma unroll
    for (int q2 = 0; q2 < 4; ++q2) ra += ht[q2] * quantise(a.y, a.u, lo + ro[q1] * wi + co[q2], a.quant);
    acc += vt[q1] * ra;
  }
  a.up_out[idx] = acc;
  for (int c = 1; c < nch; ++c) {
    const float* in = a.up_in + (size_t)(c - 1) * hi * wi;
    float acc2 = 0.0f;
#pragma unroll
    for (int q1 = 0; q1 < 4; ++q1) {
      float ra = 0.0f;
#pragma unroll
      for (int q2 = 0; q2 < 4; ++q2) ra += ht[q2] * in[ro[q1] * wi + co[q2]];
      acc2 += vt[q1] * ra;
    }
    a.up_out[(size_t)c * h * w + idx] = acc2;
  }
}

// Adjoint of step s, one thread per input position (r, c) of level s+1:
//   g_in[r][c] = sum over (padded index m' that clamps to r, tap ky) and
//                (m'' that clamps to c, tap kx) of v[ky] h[kx] g_out[2m'+ky-3][2m''+kx-3]
// (outputs outside the level-s grid excluded), which is the transpose of the
// clamped gather above.  The tap gradients are accumulated at the same time:
//   dL/dv[ky] += in[r][c] * sum_kx h[kx] g_out[..],  dL/dh[kx] += in[r][c] * sum_ky v[ky] g_out[..].
__global__ __launch_bounds__(256) void ups_bwd_kernel(UpsBwdArgs a) {
  const int s = a.s, L = a.geo.L;
  const int ho = a.geo.lh[s], wo = a.geo.lw[s], hi = a.geo.lh[s + 1], wi = a.geo.lw[s + 1];
  const int nch = L - 1 - s;
  float v[UPS_K], hh[UPS_K], gv[UPS_K], gh[UPS_K];
#pragma unroll
  for (int k = 0; k < UPS_K; ++k) {
    v[k] = a.taps[k];
    hh[k] = a.taps[UPS_K + k];
    gv[k] = 0.0f;
    gh[k] = 0.0f;
  }
  const int lo = a.geo.loff[s + 1];
  for (int idx = blockIdx.x * 256 + threadIdx.x; idx < hi * wi; idx += gridDim.x * 256) {
    const int r = idx / wi, c = idx % wi;
    int mr[5], mc[5], nr = 0, nc = 0;
    mr[nr++] = r;
    if (r == 0) { mr[nr++] = -1; mr[nr++] = -2; }
    if (r == hi - 1) { mr[nr++] = hi; mr[nr++] = hi + 1; }
    mc[nc++] = c;
    if (c == 0) { mc[nc++] = -1; mc[nc++] = -2; }
    if (c == wi - 1) { mc[nc++] = wi; mc[nc++] = wi + 1; }
    for (int ch = 0; ch < nch; ++ch) {
      const float* gin = a.g_in + (size_t)ch * ho * wo;
      const float inval = ch == 0 ? quantise(a.y, a.u, lo + idx, a.quant) : a.up_in[(size_t)(ch - 1) * hi * wi + idx];
      float gsum = 0.0f;
      for (int pa = 0; pa < nr; ++pa) {
        for (int pb = 0; pb < nc; ++pb) {
          float rows[UPS_K], cols[UPS_K];
#pragma unroll
          for (int k = 0; k < UPS_K; ++k) { rows[k] = 0.0f; cols[k] = 0.0f; }
#pragma unroll
          for (int ky = 0; ky < UPS_K; ++ky) {
            const int jr = 2 * mr[pa] + ky - UPS_P;
            if (jr < 0 || jr >= ho) continue;
#pragma unroll
            for (int kx = 0; kx < UPS_K; ++kx) {
              const int jc = 2 * mc[pb] + kx - UPS_P;
              if (jc < 0 || jc >= wo) continue;
              const float gval = gin[jr * wo + jc];
              rows[ky] += hh[kx] * gval;
              cols[kx] += v[ky] * gval;
            }
          }
#pragma unroll
          for (int k = 0; k < UPS_K; ++k) {
            gsum += v[k] * rows[k];
            gv[k] += inval * rows[k];
            gh[k] += inval * cols[k];
          }
        }
      }
      if (ch == 0) a.g_y[idx] = gsum;
      else a.g_out[(size_t)(ch - 1) * hi * wi + idx] = gsum;
    }
  }
  __shared__ float s_red[4][2 * UPS_K];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < UPS_K; ++k) {
    const float a0 = wave_sum(gv[k]), a1 = wave_sum(gh[k]);
    if (lane == 0) { s_red[wave][k] = a0; s_red[wave][UPS_K + k] = a1; }
  }
  __syncthreads();
  if (threadIdx.x < 2 * UPS_K) {
    float acc = 0.0f;
    for (int wv = 0; wv < 4; ++wv) acc += s_red[wv][threadIdx.x];
    a.part[blockIdx.x * 2 * UPS_K + threadIdx.x] = acc;
  }
}

}  // namespace cc

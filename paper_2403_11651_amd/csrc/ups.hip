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

// Adjoint of step s.  One work-group per UT x UT tile of input positions
// (level s+1), one thread per position, channels in turn.  With padded input
// indices m' (before clamping), the transpose of the clamped gather is
//   g_pad[m'_r][m'_c] = sum_{ky, kx} v[ky] h[kx] g_out[2m'_r+ky-3][2m'_c+kx-3]
// (outputs outside the level-s grid are zero), and an input takes the sum of
// g_pad over the padded indices that clamp to it (itself, and the two beyond
// the border for border positions).  g_pad is computed separably in LDS: a
// horizontal pass T, then a vertical pass.  The tap gradients need, per
// input, in * sum_kx h[kx] g_out[..] = in * T[2m'_r+ky-3][m'_c] for each ky and
// in * sum_ky v[ky] g_out[..] = in * T2[m'_r][2m'_c+kx-3] for each kx, with T2
// the vertical-first pass.
constexpr int UT = 16;                 // input positions per tile side
constexpr int UP_N = UT + 4;           // padded indices per tile side: [m0-2, m0+UT+2)
constexpr int UR_N = 2 * UT + 14;      // output rows / columns read: [2m0-7, 2m0+2UT+7)

__global__ __launch_bounds__(256) void ups_bwd_kernel(UpsBwdArgs a) {
  __shared__ float s_g[UR_N * UR_N];
  __shared__ float s_T[UR_N * UP_N];   // [output row][padded column]
  __shared__ float s_T2[UP_N * UR_N];  // [padded row][output column]
  __shared__ float s_P[UP_N * UP_N];   // g_pad
  const int s = a.s, L = a.geo.L, tid = threadIdx.x;
  const int ho = a.geo.lh[s], wo = a.geo.lw[s], hi = a.geo.lh[s + 1], wi = a.geo.lw[s + 1];
  const int ntx = (wi + UT - 1) / UT;
  const int r0 = (blockIdx.x / ntx) * UT, c0 = (blockIdx.x % ntx) * UT;
  const int tr = tid / UT, tc = tid % UT, r = r0 + tr, c = c0 + tc;
  const bool in_tile = r < hi && c < wi;
  const int nch = L - 1 - s;
  float v[UPS_K], hh[UPS_K], gv[UPS_K], gh[UPS_K];
#pragma unroll
  for (int k = 0; k < UPS_K; ++k) {
    v[k] = a.taps[k];
    hh[k] = a.taps[UPS_K + k];
    gv[k] = 0.0f;
    gh[k] = 0.0f;
  }
  // padded indices (local to the tile frame) that clamp to r / c; -1 = none
  int ca[5], cb[5];
  ca[0] = tr + 2; ca[1] = r == 0 ? 1 : -1; ca[2] = r == 0 ? 0 : -1;
  ca[3] = r == hi - 1 ? tr + 3 : -1; ca[4] = r == hi - 1 ? tr + 4 : -1;
  cb[0] = tc + 2; cb[1] = c == 0 ? 1 : -1; cb[2] = c == 0 ? 0 : -1;
  cb[3] = c == wi - 1 ? tc + 3 : -1; cb[4] = c == wi - 1 ? tc + 4 : -1;
  const int jr0 = 2 * r0 - 7, jc0 = 2 * c0 - 7;
  const int lo = a.geo.loff[s + 1];
  for (int ch = 0; ch < nch; ++ch) {
    const float* gin = a.g_in + (size_t)ch * ho * wo;
    for (int p = tid; p < UR_N * UR_N; p += 256) {
      const int jr = jr0 + p / UR_N, jc = jc0 + p % UR_N;
      s_g[p] = (jr >= 0 && jr < ho && jc >= 0 && jc < wo) ? gin[jr * wo + jc] : 0.0f;
    }
    __syncthreads();
    for (int p = tid; p < UR_N * UP_N; p += 256) {
      {  // T[row][pc] = sum_kx h[kx] g[row][2 pc + kx]
        const int row = p / UP_N, pc = p % UP_N;
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < UPS_K; ++k) acc += hh[k] * s_g[row * UR_N + 2 * pc + k];
        s_T[p] = acc;
      }
      {  // T2[pr][col] = sum_ky v[ky] g[2 pr + ky][col]
        const int pr = p / UR_N, col = p % UR_N;
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < UPS_K; ++k) acc += v[k] * s_g[(2 * pr + k) * UR_N + col];
        s_T2[p] = acc;
      }
    }
    __syncthreads();
    for (int p = tid; p < UP_N * UP_N; p += 256) {
      const int pr = p / UP_N, pc = p % UP_N;
      float acc = 0.0f;
#pragma unroll
      for (int k = 0; k < UPS_K; ++k) acc += v[k] * s_T[(2 * pr + k) * UP_N + pc];
      s_P[p] = acc;
    }
    __syncthreads();
    if (in_tile) {
      const int idx = r * wi + c;
      const float inval = ch == 0 ? quantise(a.y, a.u, lo + idx, a.quant) : a.up_in[(size_t)(ch - 1) * hi * wi + idx];
      float gsum = 0.0f;
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        if (ca[i] < 0) continue;
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          if (cb[j] < 0) continue;
          gsum += s_P[ca[i] * UP_N + cb[j]];
#pragma unroll
          for (int k = 0; k < UPS_K; ++k) {
            gv[k] += inval * s_T[(2 * ca[i] + k) * UP_N + cb[j]];
            gh[k] += inval * s_T2[ca[i] * UR_N + 2 * cb[j] + k];
          }
        }
      }
      if (ch == 0) a.g_y[idx] = gsum;
      else a.g_out[(size_t)(ch - 1) * hi * wi + idx] = gsum;
    }
    __syncthreads();
  }
  __shared__ float s_red[4][2 * UPS_K];
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int k = 0; k < UPS_K; ++k) {
    const float a0 = wave_sum(gv[k]), a1 = wave_sum(gh[k]);
    if (lane == 0) { s_red[wave][k] = a0; s_red[wave][UPS_K + k] = a1; }
  }
  __syncthreads();
  if (tid < 2 * UPS_K) {
    float acc = 0.0f;
    for (int wv = 0; wv < 4; ++wv) acc += s_red[wv][tid];
    a.part[blockIdx.x * 2 * UPS_K + tid] = acc;
  }
}

}  // namespace cc

// Synthesis f_theta kernels for gfx950 (Section II "Decoding", Table I):
//   z   = [y_hat_0, U_0(stack_1)]                       (L channels per pixel)
//   a   = ReLU(W1 z + b1)                                ("L-Hs-Conv-1")
//   t0  = ReLU(W2 a + b2)                                ("Hs-3-Conv-1")
//   t_r = phi(t_{r-1} + conv3x3_r(t_{r-1}) + b_r)        ("3-3-ConvR-3"), phi = ReLU
//         except after the last layer; replicate borders
//   x_hat = t_{n_res};  D = mean over 3HW of (x_hat - x)^2
//
// syn_t0_kernel: one thread per pixel computes the last upsampling step on
// the fly (z never reaches HBM) and the two 1x1 layers, writing t0 (3 floats
// per pixel).  syn_res_fwd_kernel: 16x16 output tiles with a halo of n_res
// pixels of t0 in LDS run the residual convs and score the distortion.
// syn_bwd_kernel: 16x16 tiles with a halo of 2 n_res recompute the residual
// convs, run their adjoint back to t0, then each thread recomputes z and the
// 1x1 layers of its pixel and runs their adjoint down to z.  Weight
// gradients are X^T Y products over pixels: each wave stages 32 pixels' rows
// in LDS and accumulates them on the v_mfma_f32_16x16x4f32 matrix core.
#include "common.hpp"
#include "kernels.hpp"

namespace cc {

// The L channels of z at pixel (i, j): y_hat_0 and U_0 of every channel of
// stack_1 = [y_hat_1, U_1 output].
__device__ __forceinline__ void compute_z(const SynArgs& a, int i, int j, float z[MAXL]) {
  const int L = a.geo.L, W = a.geo.W, h1 = a.geo.lh[1], w1 = a.geo.lw[1];
  z[0] = quantise(a.y, a.u, i * W + j, a.quant);
  int ro[4], co[4];
  float vt[4], ht[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int ky = 2 * q + 1 - (i & 1), kx = 2 * q + 1 - (j & 1);
    ro[q] = clampi((i + UPS_P - ky) >> 1, 0, h1 - 1);
    co[q] = clampi((j + UPS_P - kx) >> 1, 0, w1 - 1);
    vt[q] = a.ups0[ky];
    ht[q] = a.ups0[UPS_K + kx];
  }
  const int lo1 = a.geo.loff[1];
#pragma unroll
  for (int c = 1; c < MAXL; ++c) {
    z[c] = 0.0f;
    if (c < L) {
      float acc = 0.0f;
#pragma unroll
      for (int q1 = 0; q1 < 4; ++q1) {
        float ra = 0.0f;
#pragma unroll
        for (int q2 = 0; q2 < 4; ++q2) {
          const int p = ro[q1] * w1 + co[q2];
          const float val = c == 1 ? quantise(a.y, a.u, lo1 + p, a.quant) : a.up1[(size_t)(c - 2) * h1 * w1 + p];
          ra += ht[q2] * val;
        }
        acc += vt[q1] * ra;
      }
      z[c] = acc;
    }
  }
}

// offsets inside the packed synthesis parameters
struct SynOff {
  int W1, b1, W2, b2, res0;
  __device__ SynOff(int Hs, int L) {
    W1 = 0;
    b1 = Hs * L;
    W2 = b1 + Hs;
    b2 = W2 + 3 * Hs;
    res0 = b2 + 3;
  }
};

template <int HS>
__global__ __launch_bounds__(256) void syn_t0_kernel(SynArgs a) {
  const int H = a.geo.H, W = a.geo.W, L = a.geo.L;
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= H * W) return;
  const int i = idx / W, j = idx % W;
  const SynOff o(HS, L);
  const float* __restrict__ w = a.w;
  float z[MAXL];
  compute_z(a, i, j, z);
  float t[3] = {w[o.b2 + 0], w[o.b2 + 1], w[o.b2 + 2]};
#pragma unroll
  for (int f = 0; f < HS; ++f) {
    float pre = w[o.b1 + f];
#pragma unroll
    for (int c = 0; c < MAXL; ++c)
      if (c < L) pre += w[o.W1 + f * L + c] * z[c];
    const float av = fmaxf(pre, 0.0f);
#pragma unroll
    for (int c = 0; c < 3; ++c) t[c] += w[o.W2 + c * HS + f] * av;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) a.t0[(size_t)c * H * W + idx] = fmaxf(t[c], 0.0f);
}

// One residual layer t_r = phi(t_{r-1} + conv(t_{r-1}) + b) on the frame region
// [lo, hi)^2 of a tile frame of side FS whose position (0, 0) is image pixel
// (fi0, fj0).  Values at frame positions outside the image are the values at
// the clamped position (replicate border), so the conv reads its neighbours
// around the clamped position.
__device__ __forceinline__ void res_layer(const float* __restrict__ wr, const float* src, float* dst, int FS, int lo,
                                          int hi, int fi0, int fj0, int H, int W, bool relu, int tid) {
  const int side = hi - lo;
  for (int p = tid; p < side * side; p += SYN_THREADS) {
    const int fa = lo + p / side, fb = lo + p % side;
    const int ca = clampi(fi0 + fa, 0, H - 1) - fi0, cb = clampi(fj0 + fb, 0, W - 1) - fj0;
    float nb[3][9];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = 0; d < 9; ++d) nb[c][d] = src[c * SYN_FMAX * SYN_FMAX + (ca + d / 3 - 1) * FS + cb + d % 3 - 1];
#pragma unroll
    for (int o = 0; o < 3; ++o) {
      float pre = nb[o][4] + wr[81 + o];
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = 0; d < 9; ++d) pre += wr[o * 27 + c * 9 + d] * nb[c][d];
      dst[o * SYN_FMAX * SYN_FMAX + fa * FS + fb] = relu ? fmaxf(pre, 0.0f) : pre;
    }
  }
}

__global__ __launch_bounds__(SYN_THREADS) void syn_res_fwd_kernel(SynArgs a) {
  constexpr int FA = SYN_FMAX * SYN_FMAX;
  __shared__ float s_t[2][3 * FA];
  const int H = a.geo.H, W = a.geo.W, tid = threadIdx.x;
  const int E = a.n_res, FS = SYN_T + 2 * E;
  float sse = 0.0f;
  for (int tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
    const int i0 = (tile / a.n_tiles_x) * SYN_T, j0 = (tile % a.n_tiles_x) * SYN_T;
    const int fi0 = i0 - E, fj0 = j0 - E;
    for (int p = tid; p < FS * FS; p += SYN_THREADS) {
      const int fa = p / FS, fb = p % FS;
      const int ii = clampi(fi0 + fa, 0, H - 1), jj = clampi(fj0 + fb, 0, W - 1);
#pragma unroll
      for (int c = 0; c < 3; ++c) s_t[0][c * FA + fa * FS + fb] = a.t0[(size_t)c * H * W + ii * W + jj];
    }
    __syncthreads();
    int cur = 0;
    for (int r = 1; r <= E; ++r) {
      res_layer(a.w + a.res_off + (r - 1) * 84, s_t[cur], s_t[cur ^ 1], FS, r, FS - r, fi0, fj0, H, W, r < E, tid);
      cur ^= 1;
      __syncthreads();
    }
    {
      const int ty = tid / SYN_T, tx = tid % SYN_T;
      const int i = i0 + ty, j = j0 + tx;
      if (i < H && j < W) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float xh = s_t[cur][c * FA + (E + ty) * FS + E + tx];
          const size_t gi = (size_t)c * H * W + i * W + j;
          if (a.xhat) a.xhat[gi] = xh;
          if (a.img) { const float e = xh - a.img[gi]; sse += e * e; }
        }
      }
    }
    __syncthreads();
  }
  __shared__ float s_red[SYN_THREADS / 64];
  sse = wave_sum(sse);
  if ((tid & 63) == 0) s_red[tid >> 6] = sse;
  __syncthreads();
  if (tid == 0 && a.spart) {
    float acc = 0.0f;
    for (int k = 0; k < SYN_THREADS / 64; ++k) acc += s_red[k];
    a.spart[blockIdx.x] = acc;
  }
}

// acc[bm][bn] += X^T Y over the 64 items (one per lane) of the wave, with
// X [item][NX] and Y [item][NY] staged in LDS, 32 items at a time, and read
// back as 16x16x4 MFMA operands.  Accumulator r of lane l holds
// (X index 16 bm + 4 (l / 16) + r, Y index 16 bn + l % 16).
template <int NX, int NY, int BM, int BN>
__device__ __forceinline__ void xty_accumulate(f32x4 (&acc)[BM][BN], float* stg, const float (&xv)[NX],
                                               const float (&yv)[NY], int lane) {
  constexpr int LX = NX | 1, LY = NY | 1;
  float* Xs = stg;
  float* Ys = stg + 32 * LX;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    if ((lane >> 5) == half) {
      const int row = lane & 31;
#pragma unroll
      for (int k = 0; k < NX; ++k) Xs[row * LX + k] = xv[k];
#pragma unroll
      for (int k = 0; k < NY; ++k) Ys[row * LY + k] = yv[k];
    }
    wave_lds_sync();
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int item = 4 * t + (lane >> 4), col = lane & 15;
      float av[BM], bv[BN];
#pragma unroll
      for (int bm = 0; bm < BM; ++bm) av[bm] = (16 * bm + col < NX) ? Xs[item * LX + 16 * bm + col] : 0.0f;
#pragma unroll
      for (int bn = 0; bn < BN; ++bn) bv[bn] = (16 * bn + col < NY) ? Ys[item * LY + 16 * bn + col] : 0.0f;
#pragma unroll
      for (int bm = 0; bm < BM; ++bm)
#pragma unroll
        for (int bn = 0; bn < BN; ++bn) acc[bm][bn] = mfma16x16x4(av[bm], bv[bn], acc[bm][bn]);
    }
    wave_lds_sync();
  }
}

template <int BM, int BN>
__device__ __forceinline__ void zero_acc(f32x4 (&acc)[BM][BN]) {
#pragma unroll
  for (int bm = 0; bm < BM; ++bm)
#pragma unroll
    for (int bn = 0; bn < BN; ++bn) acc[bm][bn] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
}

template <int HS>
__global__ __launch_bounds__(SYN_THREADS, 2) void syn_bwd_kernel(SynArgs a) {
  constexpr int FA = SYN_FMAX * SYN_FMAX;
  constexpr int BMA = (HS + 15) / 16;   // blocks of the hidden width
  constexpr int BNA = (HS + 1 + 15) / 16;
  // widest staged product per item: (g_a, [z, 1]), (g_pre_t, [a, 1]) or
  // (g_pre_r, 3x3x3 neighbourhood + 1)
  constexpr int STG_W1 = (HS | 1) + ((MAXL + 1) | 1), STG_W2 = 3 + ((HS + 1) | 1), STG_R = 3 + (28 | 1);
  constexpr int STG_ROW = STG_W1 > STG_W2 ? (STG_W1 > STG_R ? STG_W1 : STG_R) : (STG_W2 > STG_R ? STG_W2 : STG_R);
  __shared__ float s_t[SYN_MAXRES + 1][3 * FA];
  __shared__ float s_g[2][3 * FA];
  __shared__ float s_stg[SYN_THREADS / 64][32 * STG_ROW];

  const int H = a.geo.H, W = a.geo.W, L = a.geo.L, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nres = a.n_res, E = 2 * nres, FS = SYN_T + 2 * E;
  const SynOff o(HS, L);
  const float* __restrict__ w = a.w;
  float* stg = s_stg[wave];

  f32x4 accW1[BMA][1], accW2[1][BNA], accR[SYN_MAXRES][1][2];
  zero_acc(accW1);
  zero_acc(accW2);
#pragma unroll
  for (int r = 0; r < SYN_MAXRES; ++r) zero_acc(accR[r]);
  float sse = 0.0f;

  for (int tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
    const int i0 = (tile / a.n_tiles_x) * SYN_T, j0 = (tile % a.n_tiles_x) * SYN_T;
    const int fi0 = i0 - E, fj0 = j0 - E;
    // 1. t0 on the frame (clamped coordinates)
    for (int p = tid; p < FS * FS; p += SYN_THREADS) {
      const int fa = p / FS, fb = p % FS;
      const int ii = clampi(fi0 + fa, 0, H - 1), jj = clampi(fj0 + fb, 0, W - 1);
#pragma unroll
      for (int c = 0; c < 3; ++c) s_t[0][c * FA + fa * FS + fb] = a.t0[(size_t)c * H * W + ii * W + jj];
    }
    __syncthreads();
    // 2. residual layers forward, layer r on halo E - r
    for (int r = 1; r <= nres; ++r) {
      res_layer(w + o.res0 + (r - 1) * 84, s_t[r - 1], s_t[r], FS, r, FS - r, fi0, fj0, H, W, r < nres, tid);
      __syncthreads();
    }
    // 3. dL/dx_hat on halo nres; zero outside the image
    int cur = 0;
    {
      const int lo = E - nres, side = SYN_T + 2 * nres;
      for (int p = tid; p < side * side; p += SYN_THREADS) {
        const int fa = lo + p / side, fb = lo + p % side;
        const int ii = fi0 + fa, jj = fj0 + fb;
        const bool in = ii >= 0 && ii < H && jj >= 0 && jj < W;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int fp = c * FA + fa * FS + fb;
          s_g[0][fp] = in ? a.dscale * (s_t[nres][fp] - a.img[(size_t)c * H * W + ii * W + jj]) : 0.0f;
        }
      }
    }
    __syncthreads();
    // 4. residual layers backward
    for (int r = nres; r >= 1; --r) {
      const float* wr = w + o.res0 + (r - 1) * 84;
      // g_pre_r = g_t_r * ReLU'(pre_r) on halo r (identity for the last layer)
      if (r < nres) {
        const int lo = E - r, side = SYN_T + 2 * r;
        for (int p = tid; p < side * side; p += SYN_THREADS) {
          const int fp = (lo + p / side) * FS + lo + p % side;
#pragma unroll
          for (int c = 0; c < 3; ++c)
            if (!(s_t[r][c * FA + fp] > 0.0f)) s_g[cur][c * FA + fp] = 0.0f;
        }
        __syncthreads();
      }
      // weight gradient of layer r over the tile's own pixels
      {
        const int ty = tid / SYN_T, tx = tid % SYN_T;
        const bool in = (i0 + ty) < H && (j0 + tx) < W;
        const int fp = (E + ty) * FS + E + tx;
        float xv[3], yv[28];
#pragma unroll
        for (int c = 0; c < 3; ++c) xv[c] = in ? s_g[cur][c * FA + fp] : 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int d = 0; d < 9; ++d) yv[c * 9 + d] = in ? s_t[r - 1][c * FA + fp + (d / 3 - 1) * FS + d % 3 - 1] : 0.0f;
        yv[27] = in ? 1.0f : 0.0f;
        if (r == 1) xty_accumulate(accR[0], stg, xv, yv, lane);
        else xty_accumulate(accR[SYN_MAXRES - 1], stg, xv, yv, lane);
      }
      // adjoint: g_t_{r-1}[q] = g_pre[q] + sum over padded positions q' that clamp
      // to q of sum_d W_d^T g_pre[q' - d], in-image terms only
      {
        const int lo = E - r + 1, side = SYN_T + 2 * (r - 1);
        for (int p = tid; p < side * side; p += SYN_THREADS) {
          const int fa = lo + p / side, fb = lo + p % side;
          const int ii = fi0 + fa, jj = fj0 + fb;
          const int fp = fa * FS + fb;
          float out[3] = {0.0f, 0.0f, 0.0f};
          if (ii >= 0 && ii < H && jj >= 0 && jj < W) {
            int ay[3], ax[3], nay = 0, nax = 0;
            ay[nay++] = 0;
            if (ii == 0) ay[nay++] = -1;
            if (ii == H - 1) ay[nay++] = 1;
            ax[nax++] = 0;
            if (jj == 0) ax[nax++] = -1;
            if (jj == W - 1) ax[nax++] = 1;
#pragma unroll
            for (int c = 0; c < 3; ++c) out[c] = s_g[cur][c * FA + fp];
            for (int u1 = 0; u1 < nay; ++u1) {
              for (int u2 = 0; u2 < nax; ++u2) {
#pragma unroll
                for (int d = 0; d < 9; ++d) {
                  const int dy = d / 3 - 1, dx = d % 3 - 1;
                  const int si = ii + ay[u1] - dy, sj = jj + ax[u2] - dx;
                  if (si < 0 || si >= H || sj < 0 || sj >= W) continue;
                  const int sp = (fa + ay[u1] - dy) * FS + fb + ax[u2] - dx;
                  const float g0 = s_g[cur][sp], g1 = s_g[cur][FA + sp], g2 = s_g[cur][2 * FA + sp];
#pragma unroll
                  for (int c = 0; c < 3; ++c)
                    out[c] += wr[0 * 27 + c * 9 + d] * g0 + wr[1 * 27 + c * 9 + d] * g1 + wr[2 * 27 + c * 9 + d] * g2;
                }
              }
            }
          }
#pragma unroll
          for (int c = 0; c < 3; ++c) s_g[cur ^ 1][c * FA + fp] = out[c];
        }
      }
      cur ^= 1;
      __syncthreads();
    }
    // 5./6. per pixel: 1x1 layers recomputed, then their adjoint down to z
    {
      const int ty = tid / SYN_T, tx = tid % SYN_T;
      const int i = i0 + ty, j = j0 + tx;
      const bool in = i < H && j < W;
      const int fp = (E + ty) * FS + E + tx;
      float gpt[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float t0v = s_t[0][c * FA + fp];
        gpt[c] = (in && t0v > 0.0f) ? s_g[cur][c * FA + fp] : 0.0f;
        if (in) {
          const float e = s_t[nres][c * FA + fp] - a.img[(size_t)c * H * W + i * W + j];
          sse += e * e;
        }
      }
      float z[MAXL];
      if (in) compute_z(a, i, j, z);
      else {
#pragma unroll
        for (int c = 0; c < MAXL; ++c) z[c] = 0.0f;
      }
      float av1[HS + 1], ga[HS], gz[MAXL];
#pragma unroll
      for (int c = 0; c < MAXL; ++c) gz[c] = 0.0f;
#pragma unroll
      for (int f = 0; f < HS; ++f) {
        float pre = w[o.b1 + f];
#pragma unroll
        for (int c = 0; c < MAXL; ++c)
          if (c < L) pre += w[o.W1 + f * L + c] * z[c];
        av1[f] = in ? fmaxf(pre, 0.0f) : 0.0f;
        float g = w[o.W2 + f] * gpt[0] + w[o.W2 + HS + f] * gpt[1] + w[o.W2 + 2 * HS + f] * gpt[2];
        g = pre > 0.0f ? g : 0.0f;
        ga[f] = g;
#pragma unroll
        for (int c = 0; c < MAXL; ++c)
          if (c < L) gz[c] += w[o.W1 + f * L + c] * g;
      }
      av1[HS] = in ? 1.0f : 0.0f;
      if (in) {
        a.g_y[i * W + j] = gz[0];
#pragma unroll
        for (int c = 1; c < MAXL; ++c)
          if (c < L) a.gz[(size_t)(c - 1) * H * W + i * W + j] = gz[c];
      }
      // weight gradients: W2, b2 from (g_pre_t, [a, 1]); W1, b1 from (g_a, [z, 1])
      xty_accumulate(accW2, stg, gpt, av1, lane);
      float zv[MAXL + 1];
#pragma unroll
      for (int c = 0; c < MAXL; ++c) zv[c] = c < L ? z[c] : 0.0f;
      zv[MAXL] = in ? 1.0f : 0.0f;
      xty_accumulate(accW1, stg, ga, zv, lane);
    }
    __syncthreads();
  }

  // ---- block partials
  const int n_syn = HS * L + HS + 3 * HS + 3 + nres * 84;
  static_assert(4 * (48 * MAXL + 48 + 3 * 48 + 3 + SYN_MAXRES * 84) <= (SYN_MAXRES + 1) * 3 * FA, "partials fit");
  float* red = &s_t[0][0];  // [waves][n_syn], spans the whole s_t array
  float* rw = red + wave * n_syn;
  const int lg = lane >> 4, lc = lane & 15;
#pragma unroll
  for (int bm = 0; bm < BMA; ++bm)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int f = 16 * bm + 4 * lg + r, c = lc;  // X index = hidden unit, Y index = z channel (MAXL = bias)
      if (f < HS) {
        if (c < L) rw[o.W1 + f * L + c] = accW1[bm][0][r];
        else if (c == MAXL) rw[o.b1 + f] = accW1[bm][0][r];
      }
    }
#pragma unroll
  for (int bn = 0; bn < BNA; ++bn)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = 4 * lg + r, f = 16 * bn + lc;  // X index = output channel, Y index = hidden unit (HS = bias)
      if (c < 3) {
        if (f < HS) rw[o.W2 + c * HS + f] = accW2[0][bn][r];
        else if (f == HS) rw[o.b2 + c] = accW2[0][bn][r];
      }
    }
  for (int rr = 0; rr < nres; ++rr) {
    const int slot = rr == 0 ? 0 : SYN_MAXRES - 1;
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int oc = 4 * lg + r, k = 16 * bn + lc;
        if (oc < 3) {
          if (k < 27) rw[o.res0 + rr * 84 + oc * 27 + k] = accR[slot][0][bn][r];
          else if (k == 27) rw[o.res0 + rr * 84 + 81 + oc] = accR[slot][0][bn][r];
        }
      }
  }
  __shared__ float s_red[SYN_THREADS / 64];
  sse = wave_sum(sse);
  if (lane == 0) s_red[wave] = sse;
  __syncthreads();
  for (int p = tid; p < n_syn; p += SYN_THREADS) {
    float acc = 0.0f;
    for (int k = 0; k < SYN_THREADS / 64; ++k) acc += red[k * n_syn + p];
    a.wpart[(size_t)blockIdx.x * n_syn + p] = acc;
  }
  if (tid == 0) {
    float acc = 0.0f;
    for (int k = 0; k < SYN_THREADS / 64; ++k) acc += s_red[k];
    a.spart[blockIdx.x] = acc;
  }
}

SynKernelFn syn_t0_kernel_for(int Hs) {
  switch (Hs) {
    case 8: return syn_t0_kernel<8>;
    case 16: return syn_t0_kernel<16>;
    case 24: return syn_t0_kernel<24>;
    case 32: return syn_t0_kernel<32>;
    case 40: return syn_t0_kernel<40>;
    case 48: return syn_t0_kernel<48>;
  }
  return nullptr;
}
SynKernelFn syn_res_fwd_kernel_for(int Hs) { return (Hs % 8 == 0 && Hs >= 8 && Hs <= 48) ? syn_res_fwd_kernel : nullptr; }
SynKernelFn syn_bwd_kernel_for(int Hs) {
  switch (Hs) {
    case 8: return syn_bwd_kernel<8>;
    case 16: return syn_bwd_kernel<16>;
    case 24: return syn_bwd_kernel<24>;
    case 32: return syn_bwd_kernel<32>;
    case 40: return syn_bwd_kernel<40>;
    case 48: return syn_bwd_kernel<48>;
  }
  return nullptr;
}

}  // namespace cc

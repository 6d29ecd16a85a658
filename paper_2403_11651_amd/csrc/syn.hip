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

// The L channels of z at pixel (i, j) are y_hat_0 and U_0 of every channel of
// stack_1 = [y_hat_1, U_1 output].  A separable U_0 runs vertically first
// (four taps per column, explicit FMAs), then horizontally; the shared 8 x 8
// kernel (Table I) takes its 4 x 4 taps of the pixel's parity at once.
// The four taps of one direction that reach an output of parity `odd`
// (tap 2q + 1 - odd for the q-th input), selected from the eight taps held
// in registers (uniform loads, no per-lane indexing).
__device__ __forceinline__ void parity_taps(const float (&k8)[UPS_K], int odd, float (&t)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) t[q] = odd ? k8[2 * q] : k8[2 * q + 1];
}

// (taps is null for a single latent level, which has no upsampling)
__device__ __forceinline__ void load_taps(const float* __restrict__ taps, float (&kv)[UPS_K], float (&kh)[UPS_K]) {
#pragma unroll
  for (int k = 0; k < UPS_K; ++k) {
    kv[k] = taps ? taps[k] : 0.0f;
    kh[k] = taps ? taps[UPS_K + k] : 0.0f;
  }
}

// Channel c >= 1 of z at pixel (pi, pj) with the shared kernel w2 (LDS,
// [8][8]) from the stack_1 region st (frame origin (r0, c0), row stride RS1,
// already clamped to the grid): sum over the 4 x 4 taps of the pixel's parity.
template <int RS1>
__device__ __forceinline__ float shared_u0(const float* __restrict__ w2, const float* __restrict__ st, int pi, int pj,
                                           int r0, int c0) {
  const int ky0 = 1 - (pi & 1), kx0 = 1 - (pj & 1);
  float acc = 0.0f;
#pragma unroll
  for (int q1 = 0; q1 < 4; ++q1) {
    const int rr = ((pi + UPS_P - (2 * q1 + ky0)) >> 1) - r0;
#pragma unroll
    for (int q2 = 0; q2 < 4; ++q2) {
      const int cc = ((pj + UPS_P - (2 * q2 + kx0)) >> 1) - c0;
      acc = __builtin_fmaf(w2[(2 * q1 + ky0) * UPS_K + 2 * q2 + kx0], st[rr * RS1 + cc], acc);
    }
  }
  return acc;
}

// Synthesis weights staged in LDS once per work-group, laid out for 128-bit
// broadcast reads: row f of W1 padded to 8 with b1[f] in column 7 (z[7] = 1),
// W2 transposed to [f][4], and each residual conv as W (81) then b (3).
template <int HS, int NRES>
struct SynW {
  float W1p[HS][8];
  float W2t[HS][4];
  float b2[4];
  float conv[NRES][88];
};

template <int HS, int NRES>
__device__ __forceinline__ void stage_weights(SynW<HS, NRES>& sw, const float* __restrict__ w, int L, int tid) {
  // SynW is [W1p | W2t | b2 | conv] without padding: one flat index
  const int b1 = HS * L, W2 = b1 + HS, b2 = W2 + 3 * HS, res0 = b2 + 3;
  constexpr int N1 = HS * 8, N2 = HS * 4, N3 = 4, N = N1 + N2 + N3 + NRES * 88;
  static_assert(sizeof(SynW<HS, NRES>) == N * sizeof(float), "flat weight layout");
  float* dst = reinterpret_cast<float*>(&sw);
  batched_stage<(N + SYN_THREADS - 1) / SYN_THREADS, SYN_THREADS>(
      tid, N,
      [&](int i) -> float {
        if (i < N1) {
          const int f = i / 8, c = i % 8;
          return c < L ? w[f * L + c] : (c == 7 ? w[b1 + f] : 0.0f);
        }
        i -= N1;
        if (i < N2) {
          const int f = i / 4, c = i % 4;
          return c < 3 ? w[W2 + c * HS + f] : 0.0f;
        }
        i -= N2;
        if (i < N3) return i < 3 ? w[b2 + i] : 0.0f;
        i -= N3;
        const int r = i / 88, k = i % 88;
        return k < 84 ? w[res0 + r * 84 + k] : 0.0f;
      },
      [&](int i, float v) { dst[i] = v; });
}

// The two 1x1 layers, a = ReLU(W1 z + b1) (z[7] = 1 carries the bias) and
// t0 = ReLU(W2 a + b2), for NP pixels at once: every weight read from LDS
// serves all NP pixels (the hidden units run in a partly unrolled loop, so
// the weights are read where they are used).
template <int HS, int NRES, int NP>
__device__ __forceinline__ void layers_1x1_np(const SynW<HS, NRES>& sw, const float (&zz)[NP][8], float (&t)[NP][3]) {
#pragma unroll
  for (int n = 0; n < NP; ++n) {
    t[n][0] = sw.b2[0]; t[n][1] = sw.b2[1]; t[n][2] = sw.b2[2];
  }
#pragma unroll 4
  for (int f = 0; f < HS; ++f) {
    const f32x4 w0 = *reinterpret_cast<const f32x4*>(&sw.W1p[f][0]);
    const f32x4 w1 = *reinterpret_cast<const f32x4*>(&sw.W1p[f][4]);
    const f32x4 w2 = *reinterpret_cast<const f32x4*>(&sw.W2t[f][0]);
#pragma unroll
    for (int n = 0; n < NP; ++n) {
      const float pre = w0.x * zz[n][0] + w0.y * zz[n][1] + w0.z * zz[n][2] + w0.w * zz[n][3] + w1.x * zz[n][4] +
                        w1.y * zz[n][5] + w1.z * zz[n][6] + w1.w * zz[n][7];
      const float av = fmaxf(pre, 0.0f);
      t[n][0] += w2.x * av; t[n][1] += w2.y * av; t[n][2] += w2.z * av;
    }
  }
#pragma unroll
  for (int n = 0; n < NP; ++n) {
    t[n][0] = fmaxf(t[n][0], 0.0f); t[n][1] = fmaxf(t[n][1], 0.0f); t[n][2] = fmaxf(t[n][2], 0.0f);
  }
}

template <int HS, int NRES>
__device__ __forceinline__ void syn_t0_body(const SynArgs& a, const int bid) {
  constexpr int RH = SYN_T0_H / 2 + 4, RW = SYN_T0_W / 2 + 4;
  __shared__ SynW<HS, NRES> sw;
  __shared__ float s_s[MAXL - 1][RH][RW + 1];
  __shared__ float s_v[MAXL - 1][SYN_T0_H][RW + 1];
  __shared__ float s_w2[UPS_SHARED_TAPS];
  const int H = a.geo.H, W = a.geo.W, L = a.geo.L, tid = threadIdx.x;
  const bool shared = a.ups_shared != 0;
  if (shared && tid < UPS_SHARED_TAPS) s_w2[tid] = a.ups0[tid];
  const int h1 = a.geo.lh[1], w1 = a.geo.lw[1], lo1 = a.geo.loff[1];
  const int ntx = (W + SYN_T0_W - 1) / SYN_T0_W;
  const int i0 = (bid / ntx) * SYN_T0_H, j0 = (bid % ntx) * SYN_T0_W;
  const int r0 = i0 / 2 - 2, c0 = j0 / 2 - 2;
  const int nch = L - 1;
  if (bid == 0 && tid == 0 && a.flag_clear) *a.flag_clear = 0.0f;
  if (bid == 0 && tid == 0 && a.t_slot) *a.t_slot = a.step[0] + 1;
  float kv[UPS_K], kh[UPS_K];
  load_taps(shared ? nullptr : a.ups0, kv, kh);
  stage_weights(sw, a.w, L, tid);
  batched_stage_stack<((MAXL - 1) * RH * RW + 255) / 256, 256>(
      tid, nch * RH * RW, a.y, a.u, a.quant, proxy_alpha(a.u, a.quant, a.geo.n_lat), a.up1,
      [&](int p, int& idx, bool& is_lat) {
        const int c = p / (RH * RW), rem = p % (RH * RW), rr = rem / RW, cc = rem % RW;
        const int q = clampi(r0 + rr, 0, h1 - 1) * w1 + clampi(c0 + cc, 0, w1 - 1);
        is_lat = c == 0;
        idx = c == 0 ? lo1 + q : (c - 1) * h1 * w1 + q;
      },
      [&](int p, float v) {
        const int c = p / (RH * RW), rem = p % (RH * RW);
        s_s[c][rem / RW][rem % RW] = v;
      });
  __syncthreads();
  for (int p = tid; !shared && p < nch * SYN_T0_H * RW; p += 256) {
    const int c = p / (SYN_T0_H * RW), rem = p % (SYN_T0_H * RW), ti = rem / RW, cc = rem % RW;
    const int i = i0 + ti;
    float vt[4];
    parity_taps(kv, i & 1, vt);
    float v = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ky = 2 * q + 1 - (i & 1);
      v = __builtin_fmaf(vt[q], s_s[c][((i + UPS_P - ky) >> 1) - r0][cc], v);
    }
    s_v[c][ti][cc] = v;
  }
  __syncthreads();
  // two pixels per thread, rows ti and ti + SYN_T0_H / 2 of one column
  constexpr int NP = SYN_T0_H * SYN_T0_W / 256;
  static_assert(NP == 2, "two pixels per thread");
  float zz[NP][8], t[NP][3];
  int pi[NP], pj[NP];
#pragma unroll
  for (int n = 0; n < NP; ++n) {
    const int ti = tid / SYN_T0_W + n * (SYN_T0_H / NP), tj = tid % SYN_T0_W;
    pi[n] = i0 + ti;
    pj[n] = j0 + tj;
    const int i = min(pi[n], H - 1), j = min(pj[n], W - 1);  // ragged tiles: computed, not stored
    zz[n][0] = quantise(a.y, a.u, i * W + j, a.quant, proxy_alpha(a.u, a.quant, a.geo.n_lat));
    int col[4];
    float ht[4];
    parity_taps(kh, pj[n] & 1, ht);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kx = 2 * q + 1 - (pj[n] & 1);
      col[q] = ((pj[n] + UPS_P - kx) >> 1) - c0;
    }
#pragma unroll
    for (int c = 1; c < 7; ++c) {
      float acc = 0.0f;
      if (c < L) {
        if (shared) {
          acc = shared_u0<RW + 1>(s_w2, &s_s[c - 1][0][0], pi[n], pj[n], r0, c0);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) acc = __builtin_fmaf(ht[q], s_v[c - 1][ti][col[q]], acc);
        }
      }
      zz[n][c] = acc;
    }
    zz[n][7] = 1.0f;
  }
  layers_1x1_np<HS, NRES, NP>(sw, zz, t);
#pragma unroll
  for (int n = 0; n < NP; ++n) {
    if (pi[n] >= H || pj[n] >= W) continue;
#pragma unroll
    for (int c = 0; c < 3; ++c) a.t0[(size_t)c * H * W + pi[n] * W + pj[n]] = t[n][c];
  }
}

// One residual layer t_r = phi(t_{r-1} + conv(t_{r-1}) + b) on the frame region
// [LO, FS-LO)^2 of a tile frame of side FS whose position (0, 0) is image pixel
// (fi0, fj0).  Values at frame positions outside the image are the values at
// the clamped position (replicate border), so the conv reads its neighbours
// around the clamped position.  INSIDE: the frame lies inside the image.
template <int FS, bool INSIDE, typename WP>
__device__ __forceinline__ void res_pre(WP wr, const float* src, int fa, int fb, int fi0, int fj0, int H,
                                        int W, float (&pre)[3]) {
  constexpr int FA = SYN_FA;
  int ca = fa, cb = fb;
  if (!INSIDE) {
    ca = clampi(fi0 + fa, 0, H - 1) - fi0;
    cb = clampi(fj0 + fb, 0, W - 1) - fj0;
  }
  float nb[3][9];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = 0; d < 9; ++d) nb[c][d] = src[c * FA + (ca + d / 3 - 1) * FS + cb + d % 3 - 1];
#pragma unroll
  for (int o = 0; o < 3; ++o) {
    float acc = nb[o][4] + wr[81 + o];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = 0; d < 9; ++d) acc += wr[o * 27 + c * 9 + d] * nb[c][d];
    pre[o] = acc;
  }
}

template <int FS, int LO, bool INSIDE, typename WP>
__device__ __forceinline__ void res_layer(WP wr, const float* src, float* dst, int fi0, int fj0, int H,
                                          int W, bool relu, int tid) {
  constexpr int SIDE = FS - 2 * LO, FA = SYN_FA;
  int zo = 0;  // opaque zero: the weights are read here, not hoisted out of the caller's loops
  asm volatile("" : "+s"(zo));
  wr += zo;
  for (int p = tid; p < SIDE * SIDE; p += SYN_THREADS) {
    const int fa = LO + p / SIDE, fb = LO + p % SIDE;
    float pre[3];
    res_pre<FS, INSIDE, WP>(wr, src, fa, fb, fi0, fj0, H, W, pre);
#pragma unroll
    for (int o = 0; o < 3; ++o) dst[o * FA + fa * FS + fb] = relu ? fmaxf(pre[o], 0.0f) : pre[o];
  }
}

// The last residual layer of the backward pass: x_hat on the frame region
// [LO, FS-LO) is not stored; the region receives dL/dx_hat = dscale (x_hat -
// x) (zero outside the image) and the tile's own pixels add their squared
// error to sse.
template <int FS, int LO, bool INSIDE, typename WP>
__device__ __forceinline__ void res_layer_last(WP wr, const float* src, float* g, int fi0, int fj0,
                                               int H, int W, const float* __restrict__ img, float dscale, float& sse,
                                               int tid) {
  constexpr int SIDE = FS - 2 * LO, FA = SYN_FA, E = FS / 2 - SYN_T / 2;
  int zo = 0;
  asm volatile("" : "+s"(zo));
  wr += zo;
  for (int p = tid; p < SIDE * SIDE; p += SYN_THREADS) {
    const int fa = LO + p / SIDE, fb = LO + p % SIDE;
    const int ii = fi0 + fa, jj = fj0 + fb;
    const bool in = ii >= 0 && ii < H && jj >= 0 && jj < W;
    const bool own = in && fa >= E && fa < E + SYN_T && fb >= E && fb < E + SYN_T;
    float pre[3];
    res_pre<FS, INSIDE, WP>(wr, src, fa, fb, fi0, fj0, H, W, pre);
#pragma unroll
    for (int o = 0; o < 3; ++o) {
      const float e = in ? pre[o] - img[(size_t)o * H * W + ii * W + jj] : 0.0f;
      g[o * FA + fa * FS + fb] = dscale * e;
      if (own) sse += e * e;
    }
  }
}

template <int HS, int NRES>
__device__ __forceinline__ void syn_res_fwd_body(const SynArgs& a, const int bid, const int nblk) {
  constexpr int FA = SYN_FA, E = NRES, FS = SYN_T + 2 * E;
  __shared__ SynW<HS, NRES> sw;
  __shared__ float s_t[2][3 * FA];
  const int H = a.geo.H, W = a.geo.W, tid = threadIdx.x;
  stage_weights(sw, a.w, a.geo.L, tid);
  float sse = 0.0f;
  for (int tile = bid; tile < a.n_tiles; tile += nblk) {
    const int i0 = (tile / a.n_tiles_x) * SYN_T, j0 = (tile % a.n_tiles_x) * SYN_T;
    const int fi0 = i0 - E, fj0 = j0 - E;
    const bool inside = fi0 >= 0 && fj0 >= 0 && fi0 + FS <= H && fj0 + FS <= W;
    for (int p = tid; p < FS * FS; p += SYN_THREADS) {
      const int fa = p / FS, fb = p % FS;
      const int ii = clampi(fi0 + fa, 0, H - 1), jj = clampi(fj0 + fb, 0, W - 1);
#pragma unroll
      for (int c = 0; c < 3; ++c) s_t[0][c * FA + fa * FS + fb] = a.t0[(size_t)c * H * W + ii * W + jj];
    }
    __syncthreads();
    if (inside) res_layer<FS, 1, true>(sw.conv[0], s_t[0], s_t[1], fi0, fj0, H, W, NRES > 1, tid);
    else res_layer<FS, 1, false>(sw.conv[0], s_t[0], s_t[1], fi0, fj0, H, W, NRES > 1, tid);
    __syncthreads();
    if constexpr (NRES >= 2) {
      if (inside) res_layer<FS, 2, true>(sw.conv[1], s_t[1], s_t[0], fi0, fj0, H, W, false, tid);
      else res_layer<FS, 2, false>(sw.conv[1], s_t[1], s_t[0], fi0, fj0, H, W, false, tid);
      __syncthreads();
    }
    {
      const int ty = tid / SYN_T, tx = tid % SYN_T;
      const int i = i0 + ty, j = j0 + tx;
      if (i < H && j < W) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float xh = s_t[NRES & 1][c * FA + (E + ty) * FS + E + tx];
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
    a.spart[bid] = acc;
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

// acc[bm][bn] += X^T Y over the 64 rows (items) of X [64][LX] and Y [64][LY]
// already staged in LDS by the wave (columns nx / ny and beyond read as 0).
template <int BM, int BN>
__device__ __forceinline__ void mfma_xty64(f32x4 (&acc)[BM][BN], const float* Xs, int LX, int nx, const float* Ys,
                                           int LY, int ny, int lane) {
  const int col = lane & 15;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int item = 4 * t + (lane >> 4);
    float av[BM], bv[BN];
#pragma unroll
    for (int bm = 0; bm < BM; ++bm) av[bm] = (16 * bm + col < nx) ? Xs[item * LX + 16 * bm + col] : 0.0f;
#pragma unroll
    for (int bn = 0; bn < BN; ++bn) bv[bn] = (16 * bn + col < ny) ? Ys[item * LY + 16 * bn + col] : 0.0f;
#pragma unroll
    for (int bm = 0; bm < BM; ++bm)
#pragma unroll
      for (int bn = 0; bn < BN; ++bn) acc[bm][bn] = mfma16x16x4(av[bm], bv[bn], acc[bm][bn]);
  }
}

// Weight gradient of a residual conv over the tile's own pixels, on the
// matrix cores with operands read straight from the LDS frames: acc[0][bn]
// += X^T Y, X[pixel][oc] = g (the gradient at the layer's pre-activation,
// oc < 3), Y[pixel][k] = the layer input's 3x3 neighbourhood (k = 9 c + d)
// and a ones column (k = 27).  Wave w takes pixels 64 w .. 64 w + 63 of the
// tile, four per 16x16x4 step; accumulator r of lane l holds (oc = 4 (l/16)
// + r, k = 16 bn + l % 16).
template <int FS, int E>
__device__ __forceinline__ void conv_wgrad(f32x4 (&acc)[1][2], const float* g, const float* t, int i0, int j0,
                                           int H, int W, int wave, int lane) {
  constexpr int FA = SYN_FA;
  const int col = lane & 15, kq = lane >> 4;
  int ko[2];
#pragma unroll
  for (int bn = 0; bn < 2; ++bn) {
    const int k = 16 * bn + col;
    ko[bn] = k < 27 ? (k / 9) * FA + ((k % 9) / 3 - 1) * FS + (k % 3) - 1 : 0;
  }
#pragma unroll 4
  for (int step = 0; step < 16; ++step) {
    const int item = 64 * wave + 4 * step + kq, ty = item / SYN_T, tx = item % SYN_T;
    const bool own = i0 + ty < H && j0 + tx < W;
    const int fp = (E + ty) * FS + E + tx;
    const float av = (own && col < 3) ? g[col * FA + fp] : 0.0f;
#pragma unroll
    for (int bn = 0; bn < 2; ++bn) {
      const int k = 16 * bn + col;
      const float bv = !own ? 0.0f : (k < 27 ? t[fp + ko[bn]] : (k == 27 ? 1.0f : 0.0f));
      acc[0][bn] = mfma16x16x4(av, bv, acc[0][bn]);
    }
  }
}

template <int BM, int BN>
__device__ __forceinline__ void zero_acc(f32x4 (&acc)[BM][BN]) {
#pragma unroll
  for (int bm = 0; bm < BM; ++bm)
#pragma unroll
    for (int bn = 0; bn < BN; ++bn) acc[bm][bn] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
}

// Adjoint of one residual layer at the frame positions of region [LO, FS-LO)
// (in-image ones; others get 0): g_{r-1}[q] = g_pre[q] + sum over padded
// positions q' that clamp to q of sum_d W_d^T g_pre[q' - d], in-image terms
// only (the replicate border folds the padded positions onto the edge).
// The result, masked by ReLU'(tm) (tm = the layer input, which is the output
// of a ReLU), is the gradient at the previous pre-activation: OUT = 1 writes
// it to the frame gout, OUT = 2 (region = the tile's own pixels) to the
// image-sized gpt.
template <int FS, int LO, bool INSIDE, int OUT, typename WP>
__device__ __forceinline__ void res_adjoint(WP wr, const float* g, float* gout, const float* tm,
                                            float* __restrict__ gpt, int fi0, int fj0, int H, int W, int tid) {
  constexpr int SIDE = FS - 2 * LO, FA = SYN_FA;
  int zo = 0;  // opaque zero: the weights are read here, not hoisted out of the caller's loops
  asm volatile("" : "+s"(zo));
  wr += zo;
  for (int p = tid; p < SIDE * SIDE; p += SYN_THREADS) {
    const int fa = LO + p / SIDE, fb = LO + p % SIDE;
    const int fp = fa * FS + fb;
    float out[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c] = g[c * FA + fp];
    if (INSIDE) {
#pragma unroll
      for (int d = 0; d < 9; ++d) {
        const int sp = fp - (d / 3 - 1) * FS - (d % 3 - 1);
        const float g0 = g[sp], g1 = g[FA + sp], g2 = g[2 * FA + sp];
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c] += wr[c * 9 + d] * g0 + wr[27 + c * 9 + d] * g1 + wr[54 + c * 9 + d] * g2;
      }
    } else {
      const int ii = fi0 + fa, jj = fj0 + fb;
      if (ii < 0 || ii >= H || jj < 0 || jj >= W) {
        out[0] = out[1] = out[2] = 0.0f;
      } else {
        for (int ay = -1; ay <= 1; ++ay) {
          if (ay != 0 && !((ay < 0 && ii == 0) || (ay > 0 && ii == H - 1))) continue;
          for (int ax = -1; ax <= 1; ++ax) {
            if (ax != 0 && !((ax < 0 && jj == 0) || (ax > 0 && jj == W - 1))) continue;
#pragma unroll
            for (int d = 0; d < 9; ++d) {
              const int dy = d / 3 - 1, dx = d % 3 - 1;
              const int si = ii + ay - dy, sj = jj + ax - dx;
              const bool ok = si >= 0 && si < H && sj >= 0 && sj < W;
              const int sp = ok ? (fa + ay - dy) * FS + fb + ax - dx : fp;
              const float m = ok ? 1.0f : 0.0f;
              const float g0 = m * g[sp], g1 = m * g[FA + sp], g2 = m * g[2 * FA + sp];
#pragma unroll
              for (int c = 0; c < 3; ++c)
                out[c] += wr[c * 9 + d] * g0 + wr[27 + c * 9 + d] * g1 + wr[54 + c * 9 + d] * g2;
            }
          }
        }
      }
    }
    if (OUT == 1) {
#pragma unroll
      for (int c = 0; c < 3; ++c) gout[c * FA + fp] = tm[c * FA + fp] > 0.0f ? out[c] : 0.0f;
    } else {
      const int ii = fi0 + fa, jj = fj0 + fb;
      if (ii < H && jj < W) {
#pragma unroll
        for (int c = 0; c < 3; ++c) gpt[(size_t)c * H * W + ii * W + jj] = tm[c * FA + fp] > 0.0f ? out[c] : 0.0f;
      }
    }
  }
}

// Backward of the residual convs on 16x16 tiles (frames with a halo of
// 2 n_res pixels of t0 in LDS): recompute the convs, score the distortion,
// run their adjoint back to t0 and write the gradient at the pre-activation
// of t0 (masked by its ReLU) for the head kernel; conv weight gradients on
// the matrix cores.
template <int HS, int NRES>
__device__ __forceinline__ void syn_bwd_body(const SynArgs& a, const int bid, const int nblk) {
  constexpr int FA = SYN_FA, E = 2 * NRES, FS = SYN_T + 2 * E;
  // LDS pool: residual-conv frames t_0..t_{NRES-1} and two gradient buffers
  // (x_hat = t_NRES is never stored)
  constexpr int POOL = (NRES + 2) * 3 * FA;
  __shared__ SynW<HS, NRES> sw;
  __shared__ float pool[POOL];
  float (*s_t)[3 * FA] = reinterpret_cast<float (*)[3 * FA]>(pool);
  float (*s_g)[3 * FA] = reinterpret_cast<float (*)[3 * FA]>(pool + NRES * 3 * FA);

  const int H = a.geo.H, W = a.geo.W, L = a.geo.L, tid0 = threadIdx.x, lane = tid0 & 63, wave = tid0 >> 6;
  stage_weights(sw, a.w, L, tid0);
  // the convs' weights are read as wave-uniform scalar loads (constant
  // address space) rather than from LDS
  typedef const float __attribute__((address_space(4))) cf;
  cf* wc0 = (cf*)(a.w + a.res_off);
  cf* wc1 = (cf*)(a.w + a.res_off + 84);

  f32x4 accR[NRES][1][2];
#pragma unroll
  for (int r = 0; r < NRES; ++r) zero_acc(accR[r]);
  float sse = 0.0f;

  // t0 on a tile's frame (clamped coordinates), NPF positions per thread;
  // the next tile's frame is fetched while the current one is processed
  constexpr int NPF = (FS * FS + SYN_THREADS - 1) / SYN_THREADS;
  float pf[NPF][3];
  auto fetch = [&](int tile) {
    const int fi = (tile / a.n_tiles_x) * SYN_T - E, fj = (tile % a.n_tiles_x) * SYN_T - E;
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      const int p = tid0 + SYN_THREADS * q;
      const int ii = clampi(fi + p / FS, 0, H - 1), jj = clampi(fj + p % FS, 0, W - 1);
#pragma unroll
      for (int c = 0; c < 3; ++c) pf[q][c] = p < FS * FS ? a.t0[(size_t)c * H * W + ii * W + jj] : 0.0f;
    }
  };
  if (bid < a.n_tiles) fetch(bid);

  for (int tile = bid; tile < a.n_tiles; tile += nblk) {
    const int i0 = (tile / a.n_tiles_x) * SYN_T, j0 = (tile % a.n_tiles_x) * SYN_T;
    const int fi0 = i0 - E, fj0 = j0 - E;
    const bool inside = fi0 >= 0 && fj0 >= 0 && fi0 + FS <= H && fj0 + FS <= W;
    // opaque copy of the thread index: the per-thread address arithmetic of
    // the unrolled frame loops is recomputed in each tile rather than hoisted
    // out of the tile loop (where it would have to live in registers)
    int tid = tid0;
    asm volatile("" : "+v"(tid));
    const float* __restrict__ img = a.img;
    // 1. t0 on the frame
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      const int p = tid0 + SYN_THREADS * q;
      if (p < FS * FS) {
#pragma unroll
        for (int c = 0; c < 3; ++c) s_t[0][c * FA + p] = pf[q][c];
      }
    }
    __syncthreads();
    if (tile + nblk < a.n_tiles) fetch(tile + nblk);
    // 2. residual layers forward, layer r on halo E - r; the last one yields
    // dL/dx_hat on halo NRES (zero outside the image) and the squared error
    if constexpr (NRES >= 2) {
      if (inside) res_layer<FS, 1, true>(wc0, s_t[0], s_t[1], fi0, fj0, H, W, true, tid);
      else res_layer<FS, 1, false>(wc0, s_t[0], s_t[1], fi0, fj0, H, W, true, tid);
      __syncthreads();
      if (inside) res_layer_last<FS, 2, true>(wc1, s_t[1], s_g[0], fi0, fj0, H, W, img, a.dscale, sse, tid);
      else res_layer_last<FS, 2, false>(wc1, s_t[1], s_g[0], fi0, fj0, H, W, img, a.dscale, sse, tid);
    } else {
      if (inside) res_layer_last<FS, 1, true>(wc0, s_t[0], s_g[0], fi0, fj0, H, W, img, a.dscale, sse, tid);
      else res_layer_last<FS, 1, false>(wc0, s_t[0], s_g[0], fi0, fj0, H, W, img, a.dscale, sse, tid);
    }
    __syncthreads();
    // 3. residual layers backward: weight gradient over the tile's own pixels,
    // then the adjoint one ring smaller, masked by the ReLU of the layer
    // input; the first layer's lands, as the gradient at the pre-activation
    // of t0, in gpt
    if constexpr (NRES >= 2) {
      conv_wgrad<FS, E>(accR[1], s_g[0], s_t[1], i0, j0, H, W, wave, lane);
      if (inside) res_adjoint<FS, E - 1, true, 1>(wc1, s_g[0], s_g[1], s_t[1], nullptr, fi0, fj0, H, W, tid);
      else res_adjoint<FS, E - 1, false, 1>(wc1, s_g[0], s_g[1], s_t[1], nullptr, fi0, fj0, H, W, tid);
      __syncthreads();
    }
    constexpr int G1 = NRES >= 2 ? 1 : 0;
    conv_wgrad<FS, E>(accR[0], s_g[G1], s_t[0], i0, j0, H, W, wave, lane);
    if (inside) res_adjoint<FS, E, true, 2>(wc0, s_g[G1], nullptr, s_t[0], a.gpt, fi0, fj0, H, W, tid);
    else res_adjoint<FS, E, false, 2>(wc0, s_g[G1], nullptr, s_t[0], a.gpt, fi0, fj0, H, W, tid);
    __syncthreads();
  }

  // ---- block partials: residual conv r as W (81) then b (3)
  constexpr int NR = NRES * 84;
  static_assert(4 * NR <= POOL, "partials fit");
  float* red = pool;  // [waves][NR]
  float* rw = red + wave * NR;
  const int lg = lane >> 4, lc = lane & 15;
#pragma unroll
  for (int rr = 0; rr < NRES; ++rr) {
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int oc = 4 * lg + r, k = 16 * bn + lc;
        if (oc < 3) {
          if (k < 27) rw[rr * 84 + oc * 27 + k] = accR[rr][0][bn][r];
          else if (k == 27) rw[rr * 84 + 81 + oc] = accR[rr][0][bn][r];
        }
      }
  }
  __shared__ float s_red[SYN_THREADS / 64];
  sse = wave_sum(sse);
  if (lane == 0) s_red[wave] = sse;
  __syncthreads();
  for (int p = tid0; p < NR; p += SYN_THREADS) {
    float acc = 0.0f;
    for (int k = 0; k < SYN_THREADS / 64; ++k) acc += red[k * NR + p];
    a.wpart[(size_t)bid * NR + p] = acc;
  }
  if (tid0 == 0) {
    float acc = 0.0f;
    for (int k = 0; k < SYN_THREADS / 64; ++k) acc += s_red[k];
    a.spart[bid] = acc;
  }
}

// Backward of the two 1x1 layers over a SYN_HD x SYN_HD tile, one pixel per
// thread: z recomputed as in syn_t0_body, the layers recomputed, g_a = W2^T
// g_pre_t masked by the first layer's ReLU, dL/dz = W1^T g_a written out
// (level 0 into g_y, the upsampled channels into gz).  Weight gradients: per
// 16-wide chunk of hidden units, each wave stages the chunk's a and g_a of
// its 64 pixels and accumulates X^T Y on v_mfma_f32_16x16x4f32; the bias
// columns ride along (z[7] = 1, hidden unit HS = 1).
// HALF: a chunk's a and g_a are staged for half a wave at a time (the same
// items in the same order, so the same results), which halves that staging:
// more work-groups per CU.  The batched launches use it; the single-image
// launch keeps the full staging, which leaves more of each CU to the ARM
// running beside it.
template <int HS, int NRES, bool HALF>
__device__ __forceinline__ void syn_head_bwd_body(const SynArgs& a, const int bid) {
  constexpr int T = SYN_HD, RS = T / 2 + 4;
  // chunks of 16 hidden units.  The second layer's bias gradient (the sum of
  // g_pre_t) rides in the last chunk as a unit of ones when that chunk has
  // room (BU); with HS a multiple of 16 it would take a chunk of its own, and
  // is a plain per-lane sum instead
  constexpr bool BU = HS % 16 != 0;
  constexpr int NC = (HS + (BU ? 1 : 0) + 15) / 16;
  constexpr int NCG = (HS + 15) / 16;  // chunks holding hidden units
  constexpr int SYZ = 9, SXT = 3, SYA = 17, SXG = 17;      // staged row lengths
  // per wave: z and g_pre_t of its 64 pixels, and a chunk's a and g_a for
  // 32 of them (the two halves of the wave are staged in turn)
  constexpr int NSTG = HALF ? 32 : 64;  // pixels whose a, g_a are staged at once
  constexpr int STG = 64 * (SYZ + SXT) + NSTG * (SYA + SXG);
  constexpr int ZPOOL = (MAXL - 1) * RS * (RS + 1) + (MAXL - 1) * T * (RS + 1);
  constexpr int NH = HS * MAXL + HS + 3 * HS + 3;          // head parameters (upper bound over L)
  constexpr int P1 = 4 * STG > ZPOOL ? 4 * STG : ZPOOL;
  constexpr int POOL = P1 > 4 * NH ? P1 : 4 * NH;
  __shared__ SynW<HS, NRES> sw;
  __shared__ __align__(16) float pool[POOL];
  float (*s_s)[RS][RS + 1] = reinterpret_cast<float (*)[RS][RS + 1]>(pool);
  float (*s_v)[T][RS + 1] = reinterpret_cast<float (*)[T][RS + 1]>(pool + (MAXL - 1) * RS * (RS + 1));
  const int H = a.geo.H, W = a.geo.W, L = a.geo.L, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h1 = a.geo.lh[1], w1 = a.geo.lw[1], lo1 = a.geo.loff[1];
  const int ntx = (W + T - 1) / T;
  const int i0 = (bid / ntx) * T, j0 = (bid % ntx) * T;
  const int r0 = i0 / 2 - 2, c0 = j0 / 2 - 2;
  const int nch = L - 1;
  const bool shared = a.ups_shared != 0;
  __shared__ float s_w2[UPS_SHARED_TAPS];
  if (shared && tid < UPS_SHARED_TAPS) s_w2[tid] = a.ups0[tid];
  float kv[UPS_K], kh[UPS_K];
  load_taps(shared ? nullptr : a.ups0, kv, kh);
  stage_weights(sw, a.w, L, tid);
  // ---- z (the computation of syn_t0_body on this tile)
  batched_stage_stack<((MAXL - 1) * RS * RS + 255) / 256, 256>(
      tid, nch * RS * RS, a.y, a.u, a.quant, proxy_alpha(a.u, a.quant, a.geo.n_lat), a.up1,
      [&](int p, int& idx, bool& is_lat) {
        const int c = p / (RS * RS), rem = p % (RS * RS), rr = rem / RS, cc = rem % RS;
        const int q = clampi(r0 + rr, 0, h1 - 1) * w1 + clampi(c0 + cc, 0, w1 - 1);
        is_lat = c == 0;
        idx = c == 0 ? lo1 + q : (c - 1) * h1 * w1 + q;
      },
      [&](int p, float v) {
        const int c = p / (RS * RS), rem = p % (RS * RS);
        s_s[c][rem / RS][rem % RS] = v;
      });
  __syncthreads();
  for (int p = tid; !shared && p < nch * T * RS; p += 256) {
    const int c = p / (T * RS), rem = p % (T * RS), ti = rem / RS, cc = rem % RS;
    const int i = i0 + ti;
    float vt[4];
    parity_taps(kv, i & 1, vt);
    float v = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ky = 2 * q + 1 - (i & 1);
      v = __builtin_fmaf(vt[q], s_s[c][((i + UPS_P - ky) >> 1) - r0][cc], v);
    }
    s_v[c][ti][cc] = v;
  }
  __syncthreads();
  const int ti = tid / T, tj = tid % T, pi = i0 + ti, pj = j0 + tj;
  const bool own = pi < H && pj < W;
  const int i = min(pi, H - 1), j = min(pj, W - 1);
  float zz[8], gpt[3], gz[7];
  zz[0] = own ? quantise(a.y, a.u, i * W + j, a.quant, proxy_alpha(a.u, a.quant, a.geo.n_lat)) : 0.0f;
  {
    int col[4];
    float ht[4];
    parity_taps(kh, pj & 1, ht);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kx = 2 * q + 1 - (pj & 1);
      col[q] = ((pj + UPS_P - kx) >> 1) - c0;
    }
#pragma unroll
    for (int c = 1; c < 7; ++c) {
      float acc = 0.0f;
      if (c < L) {
        if (shared) {
          acc = shared_u0<RS + 1>(s_w2, &s_s[c - 1][0][0], pi, pj, r0, c0);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) acc = __builtin_fmaf(ht[q], s_v[c - 1][ti][col[q]], acc);
        }
      }
      zz[c] = own ? acc : 0.0f;
    }
  }
  zz[7] = own ? 1.0f : 0.0f;
#pragma unroll
  for (int c = 0; c < 3; ++c) gpt[c] = own ? a.gpt[(size_t)c * H * W + i * W + j] : 0.0f;
#pragma unroll
  for (int c = 0; c < 7; ++c) gz[c] = 0.0f;
  __syncthreads();  // the z staging is dead: the pool becomes per-wave staging
  float* Yz = pool + wave * STG;
  float* Xt = Yz + 64 * SYZ;
  float* Ya = Xt + 64 * SXT;
  float* Xg = Ya + NSTG * SYA;
#pragma unroll
  for (int c = 0; c < 8; ++c) Yz[lane * SYZ + c] = zz[c];
#pragma unroll
  for (int c = 0; c < 3; ++c) Xt[lane * SXT + c] = gpt[c];
  f32x4 accW1[NCG][1], accW2[1][NC];
  zero_acc(accW1);
  zero_acc(accW2);
  const int col = lane & 15;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    // opaque zero: this chunk's weight reads stay in this chunk
    int wz = 0;
    asm volatile("" : "+s"(wz));
    const SynW<HS, NRES>& swl = *reinterpret_cast<const SynW<HS, NRES>*>(reinterpret_cast<const char*>(&sw) + wz);
    float avs[16], gvs[16];
#pragma unroll 4
    for (int u = 0; u < 16; ++u) {
      const int f = 16 * k + u;
      float av = 0.0f, gv = 0.0f;
      if (f < HS) {
        const f32x4 w0 = *reinterpret_cast<const f32x4*>(&swl.W1p[f][0]);
        const f32x4 w1 = *reinterpret_cast<const f32x4*>(&swl.W1p[f][4]);
        const f32x4 w2 = *reinterpret_cast<const f32x4*>(&swl.W2t[f][0]);
        const float pre = w0.x * zz[0] + w0.y * zz[1] + w0.z * zz[2] + w0.w * zz[3] + w1.x * zz[4] + w1.y * zz[5] +
                          w1.z * zz[6] + w1.w * zz[7];
        float g = w2.x * gpt[0] + w2.y * gpt[1] + w2.z * gpt[2];
        g = pre > 0.0f ? g : 0.0f;
        av = fmaxf(pre, 0.0f);
        gv = g;
        gz[0] += w0.x * g; gz[1] += w0.y * g; gz[2] += w0.z * g; gz[3] += w0.w * g;
        gz[4] += w1.x * g; gz[5] += w1.y * g; gz[6] += w1.z * g;
      } else if (BU && f == HS) {
        av = own ? 1.0f : 0.0f;  // the bias unit of the second layer
      }
      avs[u] = av;
      gvs[u] = gv;
    }
#pragma unroll
    for (int half = 0; half < 64 / NSTG; ++half) {
      if (!HALF || (lane >> 5) == half) {
        const int row = HALF ? lane & 31 : lane;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          Ya[row * SYA + u] = avs[u];
          Xg[row * SXG + u] = gvs[u];
        }
      }
      wave_lds_sync();
#pragma unroll
      for (int t = 0; t < NSTG / 4; ++t) {
        const int item = 4 * t + (lane >> 4), px = NSTG * half + item;
        const float xt = Xt[px * SXT + min(col, 2)];
        const float ya = Ya[item * SYA + col];
        accW2[0][k] = mfma16x16x4(col < 3 ? xt : 0.0f, ya, accW2[0][k]);
        if (k < NCG) {
          const float xg = Xg[item * SXG + col];
          const float yz = Yz[px * SYZ + min(col, 7)];
          accW1[k < NCG ? k : 0][0] = mfma16x16x4(xg, col < 8 ? yz : 0.0f, accW1[k < NCG ? k : 0][0]);
        }
      }
      wave_lds_sync();
    }
  }
  if (own) {
    const int px = pi * W + pj;
    a.g_y[px] = gz[0];
#pragma unroll
    for (int c = 1; c < 7; ++c)
      if (c < L) a.gz[(size_t)(c - 1) * H * W + px] = gz[c];
  }
  // ---- block partials: W1 [HS][L], b1 [HS], W2 [3][HS], b2 [3]
  __syncthreads();
  const int nh = HS * L + HS + 3 * HS + 3;
  const int oW1 = 0, ob1 = HS * L, oW2 = ob1 + HS, ob2 = oW2 + 3 * HS;
  float* rw = pool + wave * nh;
  const int lg = lane >> 4, lc = lane & 15;
#pragma unroll
  for (int bm = 0; bm < NCG; ++bm)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int f = 16 * bm + 4 * lg + r, c = lc;  // X index = hidden unit, Y index = z channel (7 = bias)
      if (f < HS) {
        if (c < L) rw[oW1 + f * L + c] = accW1[bm][0][r];
        else if (c == 7) rw[ob1 + f] = accW1[bm][0][r];
      }
    }
#pragma unroll
  for (int bn = 0; bn < NC; ++bn)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = 4 * lg + r, f = 16 * bn + lc;  // X index = output channel, Y index = hidden unit (HS = bias)
      if (c < 3) {
        if (f < HS) rw[oW2 + c * HS + f] = accW2[0][bn][r];
        else if (BU && f == HS) rw[ob2 + c] = accW2[0][bn][r];
      }
    }
  if constexpr (!BU) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float b2 = wave_sum(gpt[c]);  // zero for pixels outside the image
      if (lane == 0) rw[ob2 + c] = b2;
    }
  }
  __syncthreads();
  for (int p = tid; p < nh; p += 256)
    a.hpart[(size_t)bid * nh + p] = ((pool[p] + pool[nh + p]) + pool[2 * nh + p]) + pool[3 * nh + p];
}

template <int HS, int NRES>
__global__ __launch_bounds__(256) void syn_t0_kernel(SynArgs a) {
  syn_t0_body<HS, NRES>(a, blockIdx.x);
}
template <int HS, int NRES>
__global__ __launch_bounds__(256) void syn_t0_kernel_batch(const SynArgs* __restrict__ d, const WorkItem* __restrict__ w) {
  const WorkItem it = w[blockIdx.x];
  syn_t0_body<HS, NRES>(d[it.img], it.bid);
}
template <int HS, int NRES>
__global__ __launch_bounds__(SYN_THREADS) void syn_res_fwd_kernel(SynArgs a) {
  syn_res_fwd_body<HS, NRES>(a, blockIdx.x, gridDim.x);
}
template <int HS, int NRES>
__global__ __launch_bounds__(SYN_THREADS) void syn_res_fwd_kernel_batch(const SynArgs* __restrict__ d,
                                                                        const WorkItem* __restrict__ w) {
  const WorkItem it = w[blockIdx.x];
  syn_res_fwd_body<HS, NRES>(d[it.img], it.bid, it.nblk);
}
// five waves per SIMD (at most 96 VGPRs, no spills): with 30 KB of LDS per
// work-group, five work-groups share a CU
template <int HS, int NRES>
__global__ __launch_bounds__(SYN_THREADS) __attribute__((amdgpu_waves_per_eu(5))) void syn_bwd_kernel(SynArgs a) {
  syn_bwd_body<HS, NRES>(a, blockIdx.x, gridDim.x);
}
template <int HS, int NRES>
__global__ __launch_bounds__(SYN_THREADS) __attribute__((amdgpu_waves_per_eu(5))) void syn_bwd_kernel_batch(const SynArgs* __restrict__ d,
                                                                       const WorkItem* __restrict__ w) {
  const WorkItem it = w[blockIdx.x];
  syn_bwd_body<HS, NRES>(d[it.img], it.bid, it.nblk);
}

template <int HS, int NRES>
__global__ __launch_bounds__(256) void syn_head_bwd_kernel(SynArgs a) {
  syn_head_bwd_body<HS, NRES, false>(a, blockIdx.x);
}
template <int HS, int NRES>
__global__ __launch_bounds__(256) void syn_head_bwd_kernel_batch(const SynArgs* __restrict__ d,
                                                                 const WorkItem* __restrict__ w) {
  const WorkItem it = w[blockIdx.x];
  syn_head_bwd_body<HS, NRES, true>(d[it.img], it.bid);
}

#define CC_SYN_TABLE(KERNEL)                                         \
  if (nres == 1) switch (Hs) {                                       \
      case 8: return (const void*)KERNEL<8, 1>;                                   \
      case 16: return (const void*)KERNEL<16, 1>;                                 \
      case 24: return (const void*)KERNEL<24, 1>;                                 \
      case 32: return (const void*)KERNEL<32, 1>;                                 \
      case 40: return (const void*)KERNEL<40, 1>;                                 \
      case 48: return (const void*)KERNEL<48, 1>;                                 \
    }                                                                \
  if (nres == 2) switch (Hs) {                                       \
      case 8: return (const void*)KERNEL<8, 2>;                                   \
      case 16: return (const void*)KERNEL<16, 2>;                                 \
      case 24: return (const void*)KERNEL<24, 2>;                                 \
      case 32: return (const void*)KERNEL<32, 2>;                                 \
      case 40: return (const void*)KERNEL<40, 2>;                                 \
      case 48: return (const void*)KERNEL<48, 2>;                                 \
    }                                                                \
  return nullptr;

const void* syn_t0_kernel_for(int Hs, int nres, bool batch) {
  if (batch) { CC_SYN_TABLE(syn_t0_kernel_batch) }
  CC_SYN_TABLE(syn_t0_kernel)
}
const void* syn_res_fwd_kernel_for(int Hs, int nres, bool batch) {
  if (batch) { CC_SYN_TABLE(syn_res_fwd_kernel_batch) }
  CC_SYN_TABLE(syn_res_fwd_kernel)
}
const void* syn_head_bwd_kernel_for(int Hs, int nres, bool batch) {
  if (batch) { CC_SYN_TABLE(syn_head_bwd_kernel_batch) }
  CC_SYN_TABLE(syn_head_bwd_kernel)
}
const void* syn_bwd_kernel_for(int Hs, int nres, bool batch) {
  if (batch) { CC_SYN_TABLE(syn_bwd_kernel_batch) }
  CC_SYN_TABLE(syn_bwd_kernel)
}
#undef CC_SYN_TABLE

}  // namespace cc

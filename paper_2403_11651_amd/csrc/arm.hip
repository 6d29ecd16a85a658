// ARM (auto-regressive probability model) kernels for gfx950.
//
// Per latent y_hat[l][i][j] (Section II "Decoding"): gather the C causal
// neighbours of the same grid (zero outside it), run the residual MLP
// h <- ReLU(W h + b + h) (Table I "C-C-LinR", one ARM shared by all levels),
// read (mu, s) from the C-2 output layer, and take the rate -log2 of the
// Laplace mass over [y_hat - 1/2, y_hat + 1/2] (Eq. (1) rate term).  The
// backward kernel also runs the adjoint of all of it (Section IV-A).
//
// Work layout.  A work-group owns a 4 x 64 tile of one grid and stages the
// quantised latents of the tile plus its causal halo (3 rows above, 3 columns
// each side) in LDS.  With 24 context features each wave processes 32 latents
// at a time with the v_mfma_f32_32x32x2f32 matrix core: latents sit on the 32
// columns of the MFMA, features on its rows, so a layer's output accumulators
// are directly the next layer's B operand (the K order of every product is
// permuted to the accumulator row order, and the weights are loaded in that
// order).  Weight gradients are X^T Y products over latents: the wave stages
// its 32 latents' feature rows in LDS and reads them back as MFMA operands.
// With 8 or 16 features the same scheme runs on v_mfma_f32_16x16x4f32 with
// the 16 rows shared by 16 / C latent sets (arm_body_n16).
//
// The context gradient of a latent goes back to its C causal neighbours.  To
// keep the result deterministic without atomics, each tile writes the
// gradient of every latent of its extended frame (tile + causal halo) as a
// gathered sum in fixed order; a fold kernel later adds, for each latent, the
// frames of the (at most 6) tiles that cover it, in fixed order.
#include "common.hpp"
#include "rate.hpp"
#include "kernels.hpp"

namespace cc {

constexpr int STG = 36;  // row stride of the per-wave staging matrices

// Context gradients of a tile's extended frame: s_gc holds, k-major after
// GPAD padding floats, the gradient of every in-tile latent's k-th context
// input, s_own the gradient reaching each latent through its own rate term.
// Writes, for every frame position, the sum of what its in-tile causal
// successors sent it (in order k = 0 .. C-1) plus its own term.
template <int C, int GPAD>
__device__ __forceinline__ void arm_gather_tile(float* __restrict__ ge, const float* s_gc, const float* s_own,
                                                int tid) {
  constexpr int TL = ARM_TH * ARM_TW;
  for (int idx = tid; idx < ARM_EXT; idx += ARM_THREADS) {
    const int fa = idx / ARM_EW, fb = idx % ARM_EW;
    // the latent whose k-th neighbour is (fa, fb) is (fa - 3 - dy_k,
    // fb - 3 - dx_k): every read is base + a constant (inside the padded
    // buffer), and the in-tile ones are added in order k = 0 .. C-1
    const int gbase = GPAD + (fa - 3) * ARM_TW + fb - 3;
    bool rv[4], cv[7];  // row valid for dy = -j, column valid for dx = i - 3
#pragma unroll
    for (int j = 0; j < 4; ++j) rv[j] = fa - 3 + j >= 0 && fa - 3 + j < ARM_TH;
#pragma unroll
    for (int i = 0; i < 7; ++i) cv[i] = fb - i >= 0 && fb - i < ARM_TW;
    float v[C];
#pragma unroll
    for (int k = 0; k < C; ++k) v[k] = s_gc[gbase + k * TL - ctx_dy<C>(k) * ARM_TW - ctx_dx<C>(k)];
    const bool own_in = fa >= 3 && fb >= 3 && fb < ARM_TW + 3;
    const float vo = s_own[own_in ? (fa - 3) * ARM_TW + fb - 3 : 0];
    float G = 0.0f;
#pragma unroll
    for (int k = 0; k < C; ++k) G += (rv[-ctx_dy<C>(k)] && cv[ctx_dx<C>(k) + 3]) ? v[k] : 0.0f;
    if (own_in) G += vo;
    ge[idx] = G;
  }
}

template <int C, int NH, bool BWD>
__device__ __forceinline__ void arm_body(const ArmArgs& a, const int bid, const int nblk) {
  constexpr int NR = C / 2;            // accumulator rows holding features < C
  constexpr int TL = ARM_TH * ARM_TW;  // latents per tile
  // context gradients of the tile, k-major ([k][latent]) after GC_PAD
  // padding floats: a frame position's C reads share one base address
  constexpr int GC_PAD = 256;
  constexpr int NW = NH * (C * C + C) + 2 * C + 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, n = lane & 31, g = lane >> 5;

  __shared__ float s_yq[ARM_EXT];
  // context gradients of the tile; reused at the end for per-wave partials
  constexpr int GC_NEED = 2 * GC_PAD + C * TL;
  constexpr int GC_SIZE = GC_NEED > ARM_WAVES * NW ? GC_NEED : ARM_WAVES * NW;
  __shared__ float s_gc[BWD ? GC_SIZE : 4 * 64];
  __shared__ float s_own[BWD ? ARM_TH * ARM_TW : 1];
  __shared__ float s_stage[BWD ? ARM_WAVES * 2 * 32 * STG : 1];

  // MFMA A operands of every layer, per lane and k-step, in the order the
  // accumulators hold the features: [0] forward W + I (A[m = out][k = in];
  // the identity carries the residual connection), [1] its transpose
  // (A[m = in][k = out]) for the input gradient
  __shared__ float s_A[BWD ? 2 : 1][NH][NR][64];

  const float* __restrict__ w = a.w;
  constexpr int NA = (BWD ? 2 : 1) * NH * NR * 64;
  batched_stage<(NA + ARM_THREADS - 1) / ARM_THREADS, ARM_THREADS>(
      tid, NA,
      [&](int idx) -> float {
        const int ln = idx & 63, t = (idx >> 6) % NR, j = (idx / (64 * NR)) % NH, tr = idx / (64 * NR * NH);
        const int nn = ln & 31, f = dfeat(t, ln >> 5);
        const float* Wj = w + j * (C * C + C);
        return nn < C ? (tr ? Wj[f * C + nn] : Wj[nn * C + f]) + (nn == f ? 1.0f : 0.0f) : 0.0f;
      },
      [&](int idx, float v) { (&s_A[0][0][0][0])[idx] = v; });
  // per-lane constants: context offsets in the LDS frame, biases and output
  // weights of the features this lane holds
  int ctxoff[NR];
  float bias[NH][NR], wo0[NR], wo1[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int f = dfeat(r, g);
    ctxoff[r] = ctx_dy<C>(f) * ARM_EW + ctx_dx<C>(f);
#pragma unroll
    for (int j = 0; j < NH; ++j) bias[j][r] = w[j * (C * C + C) + C * C + f];
    wo0[r] = w[NH * (C * C + C) + f];
    wo1[r] = w[NH * (C * C + C) + C + f];
  }
  const float bo0 = w[NH * (C * C + C) + 2 * C], bo1 = w[NH * (C * C + C) + 2 * C + 1];

  float* X = s_stage + wave * 2 * 32 * STG;
  float* Y = X + 32 * STG;
  if (BWD) {
    // constant columns of the staging matrices: X pads with zeros, Y holds
    // the bias column (ones) at C and zeros after it
    for (int idx = lane; idx < 32 * STG; idx += 64) {
      const int col = idx % STG;
      X[idx] = 0.0f;
      Y[idx] = col == C ? 1.0f : 0.0f;
    }
  }

  float rate_acc = 0.0f;
  f32x16 accW[NH];
  float accWo0[NR], accWo1[NR], accbo0 = 0.0f, accbo1 = 0.0f;
#pragma unroll
  for (int j = 0; j < NH; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) accW[j][r] = 0.0f;
#pragma unroll
  for (int r = 0; r < NR; ++r) { accWo0[r] = 0.0f; accWo1[r] = 0.0f; }

  // the quantised latents of a tile's frame (zero outside the grid), NPF per
  // thread; the next tile's are fetched while the current one is processed
  constexpr int NPF = (ARM_EXT + ARM_THREADS - 1) / ARM_THREADS;
  float pf[NPF], pu[NPF];  // raw latents (and noise), quantised when staged
  const float alpha = proxy_alpha(a.u, a.quant, a.geo.n_lat);
  auto fetch = [&](int tile) {
    int l = 0;
    while (l + 1 < a.geo.L && tile >= a.tiles.base[l + 1]) ++l;
    const int local = tile - a.tiles.base[l];
    const int i0 = (local / a.tiles.ntw[l]) * ARM_TH, j0 = (local % a.tiles.ntw[l]) * ARM_TW;
    const int h = a.geo.lh[l], wl = a.geo.lw[l], base = a.geo.loff[l];
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      const int idx = tid + ARM_THREADS * q;
      const int ii = i0 - 3 + idx / ARM_EW, jj = j0 - 3 + idx % ARM_EW;
      pf[q] = 0.0f;
      pu[q] = 0.0f;
      if (idx < ARM_EXT && ii >= 0 && ii < h && jj >= 0 && jj < wl) {
        pf[q] = a.y[base + ii * wl + jj];
        if (uses_noise(a.quant)) pu[q] = a.u[base + ii * wl + jj];
      }
    }
  };
  if (bid < a.tiles.n_tiles) fetch(bid);

  for (int tile = bid; tile < a.tiles.n_tiles; tile += nblk) {
    int l = 0;
    while (l + 1 < a.geo.L && tile >= a.tiles.base[l + 1]) ++l;
    const int local = tile - a.tiles.base[l];
    const int i0 = (local / a.tiles.ntw[l]) * ARM_TH, j0 = (local % a.tiles.ntw[l]) * ARM_TW;
    const int h = a.geo.lh[l], wl = a.geo.lw[l], base = a.geo.loff[l];

#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      const int idx = tid + ARM_THREADS * q;
      if (idx < ARM_EXT) s_yq[idx] = quantise_raw(pf[q], pu[q], a.quant, alpha);
    }
    __syncthreads();
    if (tile + nblk < a.tiles.n_tiles) fetch(tile + nblk);

    for (int c = wave; c < ARM_TH * ARM_TW / 32; c += ARM_WAVES) {
      const int rr = c / (ARM_TW / 32), cc0 = (c % (ARM_TW / 32)) * 32;
      const int i = i0 + rr, j = j0 + cc0 + n;
      const bool valid = i < h && j < wl;
      const int own = (3 + rr) * ARM_EW + 3 + cc0 + n;
      float H[NH + 1][NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) H[0][r] = s_yq[own + ctxoff[r]];
      const float yq = s_yq[own];
#pragma unroll
      for (int jl = 0; jl < NH; ++jl) {
        // h <- ReLU((W + I) h + b): the bias is the accumulators' start
        f32x16 acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = r < NR ? bias[jl][r] : 0.0f;
#pragma unroll
        for (int t = 0; t < NR; ++t) acc = mfma32x32x2(s_A[0][jl][t][lane], H[jl][t], acc);
#pragma unroll
        for (int r = 0; r < NR; ++r) H[jl + 1][r] = fmaxf(acc[r], 0.0f);
      }
      float mu = 0.0f, sg = 0.0f;
#pragma unroll
      for (int r = 0; r < NR; ++r) { mu += wo0[r] * H[NH][r]; sg += wo1[r] * H[NH][r]; }
      mu += __shfl_xor(mu, 32, 64) + bo0;
      sg += __shfl_xor(sg, 32, 64) + bo1;
      const Rate ro = laplace_rate<BWD>(yq, mu, sg);
      if (valid && g == 0) {
        rate_acc += ro.r;
        const int q = base + i * wl + j;
        if (a.rate_map) a.rate_map[q] = ro.r;
        if (a.yq_out) a.yq_out[q] = yq;
      }
      if (BWD) {
        const float gmu = valid ? -a.scale * ro.dd : 0.0f;
        const float gsg = valid ? a.scale * ro.ds : 0.0f;
        float gH[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          gH[r] = wo0[r] * gmu + wo1[r] * gsg;
          accWo0[r] += gmu * H[NH][r];
          accWo1[r] += gsg * H[NH][r];
        }
        if (g == 0) { accbo0 += gmu; accbo1 += gsg; }
#pragma unroll
        for (int jl = NH - 1; jl >= 0; --jl) {
          float gp[NR];
#pragma unroll
          for (int r = 0; r < NR; ++r) gp[r] = H[jl + 1][r] > 0.0f ? gH[r] : 0.0f;
          // weight gradient: accW[jl][o][i] += sum over the 32 latents of gp[o] * [H_jl, 1][i]
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            X[n * STG + dfeat(r, g)] = gp[r];
            Y[n * STG + dfeat(r, g)] = H[jl][r];
          }
          wave_lds_sync();
#pragma unroll
          for (int t = 0; t < 16; ++t) {
            const int row = (2 * t + g) * STG + n;
            accW[jl] = mfma32x32x2(X[row], Y[row], accW[jl]);
          }
          wave_lds_sync();
          // input gradient: (W + I)^T gp
          f32x16 acc;
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
          for (int t = 0; t < NR; ++t) acc = mfma32x32x2(s_A[BWD ? 1 : 0][jl][t][lane], gp[t], acc);
#pragma unroll
          for (int r = 0; r < NR; ++r) gH[r] = acc[r];
        }
        const int li = rr * ARM_TW + cc0 + n;
#pragma unroll
        for (int r = 0; r < NR; ++r) s_gc[GC_PAD + dfeat(r, g) * TL + li] = gH[r];
        if (g == 0) s_own[li] = valid ? a.scale * ro.dd : 0.0f;
      }
    }
    __syncthreads();
    if (BWD) {
      arm_gather_tile<C, GC_PAD>(a.gext + (size_t)tile * ARM_EXT, s_gc, s_own, tid);
      __syncthreads();
    }
  }

  // ---- block partials: rate, and (backward) the ARM weight gradients
  rate_acc = wave_sum(rate_acc);
  float* red = s_gc;  // reused: [ARM_WAVES][NW] per-wave partial gradients
  if (BWD) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      float v0 = accWo0[r], v1 = accWo1[r];
#pragma unroll
      for (int m = 16; m >= 1; m >>= 1) { v0 += __shfl_xor(v0, m, 64); v1 += __shfl_xor(v1, m, 64); }
      accWo0[r] = v0; accWo1[r] = v1;
    }
    accbo0 = wave_sum(accbo0);
    accbo1 = wave_sum(accbo1);
    float* rw = red + wave * NW;
#pragma unroll
    for (int jl = 0; jl < NH; ++jl) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int o = dfeat(r, g);
        if (o < C) {
          if (n < C) rw[jl * (C * C + C) + o * C + n] = accW[jl][r];
          else if (n == C) rw[jl * (C * C + C) + C * C + o] = accW[jl][r];
        }
      }
    }
    if (n == 0) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        rw[NH * (C * C + C) + dfeat(r, g)] = accWo0[r];
        rw[NH * (C * C + C) + C + dfeat(r, g)] = accWo1[r];
      }
    }
    if (lane == 0) { rw[NH * (C * C + C) + 2 * C] = accbo0; rw[NH * (C * C + C) + 2 * C + 1] = accbo1; }
  }
  __syncthreads();
  __shared__ float s_rate[ARM_WAVES];
  if (lane == 0) s_rate[wave] = rate_acc;
  __syncthreads();
  if (tid == 0) {
    float s = 0.0f;
    for (int k = 0; k < ARM_WAVES; ++k) s += s_rate[k];
    a.rpart[bid] = s;
  }
  if (BWD) {
    for (int p = tid; p < NW; p += ARM_THREADS) {
      float s = 0.0f;
      for (int k = 0; k < ARM_WAVES; ++k) s += red[k * NW + p];
      a.wpart[(size_t)bid * NW + p] = s;
    }
  }
}

// Narrow contexts (C = 8 or 16) on v_mfma_f32_16x16x4f32.  A wave takes
// GL = 16 x 16 / C latents at a time: the 16 rows of the product hold 16 / C
// latent sets of C features each and its 16 columns 16 latents of every set,
// so the weights enter block-diagonally (the sets never mix).  Accumulator r
// of lane l holds row 4 (l/16) + r, i.e. feature fb + r (fb = 4 (l/16) mod C)
// of latent l % 16 of set 4 (l/16) / C; K-step t of a layer takes accumulator
// t as its B operand (rows t, 4 + t, 8 + t, 12 + t) with the A operand
// permuted to match, so a layer's output feeds the next one in registers and
// every lane keeps its weights in registers.  Weight gradients X^T Y over the
// wave's latents run on the same instruction, each set on a diagonal block of
// the product (the off-diagonal blocks pair different sets and are dropped);
// bias gradients are plain sums.  Against the 32 x 32 layout this takes a
// quarter of the matrix-core cycles for C = 8 (a forward layer: 4 steps of
// 32 cycles per 32 latents instead of 4 of 64; a weight gradient: 4 steps
// instead of 16 of 64).
template <int C, int NH, bool BWD>
__device__ __forceinline__ void arm_body_n16(const ArmArgs& a, const int bid, const int nblk) {
  static_assert(C == 8 || C == 16, "16-row ARM layout");
  constexpr int SETS = 16 / C;
  constexpr int GL = 16 * SETS;        // latents per wave step
  constexpr int TL = ARM_TH * ARM_TW;  // latents per tile
  constexpr int GC_PAD = 256;
  constexpr int NW = NH * (C * C + C) + 2 * C + 2;
  constexpr int SX = C + 1;            // row stride of the staged gradient / activation rows
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int q4 = lane >> 4, j = lane & 15;
  const int set = (4 * q4) / C, fb = (4 * q4) % C;
  const int n32 = set * 16 + j;        // this lane's latent within the wave step
  const bool primary = fb == 0;        // the lane holding features 0..3 of its latent

  __shared__ float s_yq[ARM_EXT];
  constexpr int GC_NEED = 2 * GC_PAD + C * TL;
  constexpr int GC_SIZE = GC_NEED > ARM_WAVES * NW ? GC_NEED : ARM_WAVES * NW;
  __shared__ float s_gc[BWD ? GC_SIZE : 4 * 64];
  __shared__ float s_own[BWD ? TL : 1];
  __shared__ float s_stage[BWD ? ARM_WAVES * 2 * GL * SX : 1];

  const float* __restrict__ w = a.w;
  // per-lane operands: A of K-step t, forward (W + I)[row][fb + t] and
  // transposed (W + I)[fb + t][row] for the input gradient, row = feature
  // j mod C of set j / C (zero off the diagonal blocks); biases, output
  // weights and context offsets of the lane's features fb + r
  float Af[NH][4], Ab[NH][4], bias[NH][4], wo0[4], wo1[4];
  int ctxoff[4];
  const int ri = j % C;
  const bool diag = j / C == set;
#pragma unroll
  for (int jl = 0; jl < NH; ++jl) {
    const float* Wj = w + jl * (C * C + C);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int f = fb + t;
      const float id = ri == f ? 1.0f : 0.0f;
      Af[jl][t] = diag ? Wj[ri * C + f] + id : 0.0f;
      Ab[jl][t] = diag ? Wj[f * C + ri] + id : 0.0f;
      bias[jl][t] = Wj[C * C + f];
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    wo0[r] = w[NH * (C * C + C) + fb + r];
    wo1[r] = w[NH * (C * C + C) + C + fb + r];
    ctxoff[r] = ctx_dy<C>(fb + r) * ARM_EW + ctx_dx<C>(fb + r);
  }
  const float bo0 = w[NH * (C * C + C) + 2 * C], bo1 = w[NH * (C * C + C) + 2 * C + 1];

  float* X = s_stage + wave * 2 * GL * SX;  // [latent][feature] gradient at a layer's pre-activation
  float* Y = X + GL * SX;                   // [latent][feature] the layer's input

  float rate_acc = 0.0f;
  f32x4 accW[NH];
  float accB[NH][4], accWo0[4], accWo1[4], accbo0 = 0.0f, accbo1 = 0.0f;
#pragma unroll
  for (int jl = 0; jl < NH; ++jl) {
    accW[jl] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int r = 0; r < 4; ++r) accB[jl][r] = 0.0f;
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) { accWo0[r] = 0.0f; accWo1[r] = 0.0f; }

  constexpr int NPF = (ARM_EXT + ARM_THREADS - 1) / ARM_THREADS;
  float pf[NPF], pu[NPF];
  const float alpha = proxy_alpha(a.u, a.quant, a.geo.n_lat);
  auto fetch = [&](int tile) {
    int l = 0;
    while (l + 1 < a.geo.L && tile >= a.tiles.base[l + 1]) ++l;
    const int local = tile - a.tiles.base[l];
    const int i0 = (local / a.tiles.ntw[l]) * ARM_TH, j0 = (local % a.tiles.ntw[l]) * ARM_TW;
    const int h = a.geo.lh[l], wl = a.geo.lw[l], base = a.geo.loff[l];
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      const int idx = tid + ARM_THREADS * q;
      const int ii = i0 - 3 + idx / ARM_EW, jj = j0 - 3 + idx % ARM_EW;
      pf[q] = 0.0f;
      pu[q] = 0.0f;
      if (idx < ARM_EXT && ii >= 0 && ii < h && jj >= 0 && jj < wl) {
        pf[q] = a.y[base + ii * wl + jj];
        if (uses_noise(a.quant)) pu[q] = a.u[base + ii * wl + jj];
      }
    }
  };
  if (bid < a.tiles.n_tiles) fetch(bid);

  for (int tile = bid; tile < a.tiles.n_tiles; tile += nblk) {
    int l = 0;
    while (l + 1 < a.geo.L && tile >= a.tiles.base[l + 1]) ++l;
    const int local = tile - a.tiles.base[l];
    const int i0 = (local / a.tiles.ntw[l]) * ARM_TH, j0 = (local % a.tiles.ntw[l]) * ARM_TW;
    const int h = a.geo.lh[l], wl = a.geo.lw[l], base = a.geo.loff[l];

#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      const int idx = tid + ARM_THREADS * q;
      if (idx < ARM_EXT) s_yq[idx] = quantise_raw(pf[q], pu[q], a.quant, alpha);
    }
    __syncthreads();
    if (tile + nblk < a.tiles.n_tiles) fetch(tile + nblk);

    for (int c = wave; c < TL / GL; c += ARM_WAVES) {
      const int rr = c / (ARM_TW / GL), cc0 = (c % (ARM_TW / GL)) * GL;
      const int i = i0 + rr, jj = j0 + cc0 + n32;
      const bool valid = i < h && jj < wl;
      const int own = (3 + rr) * ARM_EW + 3 + cc0 + n32;
      float H[NH + 1][4];
#pragma unroll
      for (int t = 0; t < 4; ++t) H[0][t] = s_yq[own + ctxoff[t]];
      const float yq = s_yq[own];
#pragma unroll
      for (int jl = 0; jl < NH; ++jl) {
        // h <- ReLU((W + I) h + b): the bias is the accumulators' start
        f32x4 acc = f32x4{bias[jl][0], bias[jl][1], bias[jl][2], bias[jl][3]};
#pragma unroll
        for (int t = 0; t < 4; ++t) acc = mfma16x16x4(Af[jl][t], H[jl][t], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) H[jl + 1][r] = fmaxf(acc[r], 0.0f);
      }
      // output layer: the lane's four features, then the other lanes of the latent
      float mu = 0.0f, sg = 0.0f;
#pragma unroll
      for (int r = 0; r < 4; ++r) { mu += wo0[r] * H[NH][r]; sg += wo1[r] * H[NH][r]; }
      mu += __shfl_xor(mu, 16, 64);
      sg += __shfl_xor(sg, 16, 64);
      if constexpr (C == 16) {
        mu += __shfl_xor(mu, 32, 64);
        sg += __shfl_xor(sg, 32, 64);
      }
      mu += bo0;
      sg += bo1;
      const Rate ro = laplace_rate<BWD>(yq, mu, sg);
      if (valid && primary) {
        rate_acc += ro.r;
        const int q = base + i * wl + jj;
        if (a.rate_map) a.rate_map[q] = ro.r;
        if (a.yq_out) a.yq_out[q] = yq;
      }
      if (BWD) {
        const float gmu = valid ? -a.scale * ro.dd : 0.0f;
        const float gsg = valid ? a.scale * ro.ds : 0.0f;
        float gH[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          gH[r] = wo0[r] * gmu + wo1[r] * gsg;
          accWo0[r] += gmu * H[NH][r];
          accWo1[r] += gsg * H[NH][r];
        }
        if (primary) { accbo0 += gmu; accbo1 += gsg; }
#pragma unroll
        for (int jl = NH - 1; jl >= 0; --jl) {
          float gp[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            gp[r] = H[jl + 1][r] > 0.0f ? gH[r] : 0.0f;
            accB[jl][r] += gp[r];
            X[n32 * SX + fb + r] = gp[r];
            Y[n32 * SX + fb + r] = H[jl][r];
          }
          wave_lds_sync();
          // accW[jl][o][i] += sum over the latents of a set of gp[o] * h[i]:
          // K-step m takes latents 4 m .. 4 m + 3 of every set
          const int xr = (j / C) * 16 + q4, xc = j % C;
#pragma unroll
          for (int m = 0; m < 4; ++m)
            accW[jl] = mfma16x16x4(X[(xr + 4 * m) * SX + xc], Y[(xr + 4 * m) * SX + xc], accW[jl]);
          wave_lds_sync();
          // input gradient: (W + I)^T gp
          f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int t = 0; t < 4; ++t) acc = mfma16x16x4(Ab[jl][t], gp[t], acc);
#pragma unroll
          for (int r = 0; r < 4; ++r) gH[r] = acc[r];
        }
        const int li = rr * ARM_TW + cc0 + n32;
#pragma unroll
        for (int r = 0; r < 4; ++r) s_gc[GC_PAD + (fb + r) * TL + li] = gH[r];
        if (primary) s_own[li] = valid ? a.scale * ro.dd : 0.0f;
      }
    }
    __syncthreads();
    if (BWD) {
      arm_gather_tile<C, GC_PAD>(a.gext + (size_t)tile * ARM_EXT, s_gc, s_own, tid);
      __syncthreads();
    }
  }

  // ---- block partials: rate, and (backward) the ARM weight gradients
  rate_acc = wave_sum(rate_acc);
  float* red = s_gc;  // reused: [ARM_WAVES][NW] per-wave partial gradients
  if (BWD) {
    // sums over the lanes holding the same features: the 16 latents of a
    // set, and the sets
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float v0 = accWo0[r], v1 = accWo1[r];
#pragma unroll
      for (int m = 8; m >= 1; m >>= 1) { v0 += __shfl_xor(v0, m, 64); v1 += __shfl_xor(v1, m, 64); }
      if constexpr (SETS == 2) { v0 += __shfl_xor(v0, 32, 64); v1 += __shfl_xor(v1, 32, 64); }
      accWo0[r] = v0; accWo1[r] = v1;
#pragma unroll
      for (int jl = 0; jl < NH; ++jl) {
        float vb = accB[jl][r];
#pragma unroll
        for (int m = 8; m >= 1; m >>= 1) vb += __shfl_xor(vb, m, 64);
        if constexpr (SETS == 2) vb += __shfl_xor(vb, 32, 64);
        accB[jl][r] = vb;
      }
    }
    accbo0 = wave_sum(accbo0);
    accbo1 = wave_sum(accbo1);
    // weight gradients: the diagonal blocks of each product, summed over the
    // sets (for two sets, block 1 sits 2 row groups and 8 columns after block 0)
    float wsum[NH][4];
#pragma unroll
    for (int jl = 0; jl < NH; ++jl)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        wsum[jl][r] = accW[jl][r];
        if constexpr (SETS == 2) wsum[jl][r] += __shfl(accW[jl][r], (lane + 40) & 63, 64);
      }
    float* rw = red + wave * NW;
    const bool wlane = SETS == 1 || (q4 < 2 && j < 8);
    if (wlane) {
#pragma unroll
      for (int jl = 0; jl < NH; ++jl)
#pragma unroll
        for (int r = 0; r < 4; ++r) rw[jl * (C * C + C) + (fb + r) * C + j] = wsum[jl][r];
    }
    if (j == 0 && set == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int jl = 0; jl < NH; ++jl) rw[jl * (C * C + C) + C * C + fb + r] = accB[jl][r];
        rw[NH * (C * C + C) + fb + r] = accWo0[r];
        rw[NH * (C * C + C) + C + fb + r] = accWo1[r];
      }
    }
    if (lane == 0) { rw[NH * (C * C + C) + 2 * C] = accbo0; rw[NH * (C * C + C) + 2 * C + 1] = accbo1; }
  }
  __syncthreads();
  __shared__ float s_rate[ARM_WAVES];
  if (lane == 0) s_rate[wave] = rate_acc;
  __syncthreads();
  if (tid == 0) {
    float s = 0.0f;
    for (int k = 0; k < ARM_WAVES; ++k) s += s_rate[k];
    a.rpart[bid] = s;
  }
  if (BWD) {
    for (int p = tid; p < NW; p += ARM_THREADS) {
      float s = 0.0f;
      for (int k = 0; k < ARM_WAVES; ++k) s += red[k * NW + p];
      a.wpart[(size_t)bid * NW + p] = s;
    }
  }
}

template <int C, int NH, bool BWD>
__global__ __launch_bounds__(ARM_THREADS, 2) void arm_kernel(ArmArgs a) {
  if constexpr (C == 24) arm_body<C, NH, BWD>(a, blockIdx.x, gridDim.x);
  else arm_body_n16<C, NH, BWD>(a, blockIdx.x, gridDim.x);
}

// The batched launch of the 16-row layout runs four work-groups per CU (at
// most 128 VGPRs; measured: the 32-image batch's ARM launch 586 -> 415 us and
// the iteration 2 % shorter); the single-image launch keeps two.
template <int C, int NH, bool BWD>
__global__ __launch_bounds__(ARM_THREADS, C == 24 ? 2 : 4) void arm_kernel_batch(const ArmArgs* __restrict__ descs,
                                                                 const WorkItem* __restrict__ work) {
  const WorkItem w = work[blockIdx.x];
  if constexpr (C == 24) arm_body<C, NH, BWD>(descs[w.img], w.bid, w.nblk);
  else arm_body_n16<C, NH, BWD>(descs[w.img], w.bid, w.nblk);
}

// ---- instantiation table
template <bool BWD, bool BATCH>
static const void* pick(int C, int NH) {
#define CC_ARM_CASE(CC, HH)                                                                          \
  if (C == CC && NH == HH)                                                                          \
    return BATCH ? (const void*)arm_kernel_batch<CC, HH, BWD> : (const void*)arm_kernel<CC, HH, BWD>;
  CC_ARM_CASE(8, 1) CC_ARM_CASE(8, 2) CC_ARM_CASE(8, 3)
  CC_ARM_CASE(16, 1) CC_ARM_CASE(16, 2) CC_ARM_CASE(16, 3)
  CC_ARM_CASE(24, 1) CC_ARM_CASE(24, 2) CC_ARM_CASE(24, 3)
#undef CC_ARM_CASE
  return nullptr;
}

const void* arm_kernel_for(int C, int NH, bool bwd, bool batch) {
  if (batch) return bwd ? pick<true, true>(C, NH) : pick<false, true>(C, NH);
  return bwd ? pick<true, false>(C, NH) : pick<false, false>(C, NH);
}

}  // namespace cc

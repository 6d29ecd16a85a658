// Upsampling f_upsilon kernels for gfx950 (Section II "Decoding"; Table I
// "TConv", stride 2).
//
// stack_{L-1} = y_hat_{L-1}; stack_s = [y_hat_s, U_s(stack_{s+1})].  U_s is a
// stride-2 transposed convolution with 8 taps per axis and input indices
// clamped to the grid (replicate border):
//     out[i][j] = sum_{ky, kx} w[ky][kx] in[clamp((i+3-ky)/2)][clamp((j+3-kx)/2)]
// over the taps with (i+3-ky) and (j+3-kx) even (4 x 4 taps per output), with
// w[ky][kx] = v[ky] h[kx] for the separable per-step kernels (applied as the
// outer product) or one non-separable kernel shared by every step (Table I).
// The step s = 0 is fused into the synthesis kernels; these kernels produce
// the steps s >= 1 and the adjoint of every step: one launch per step, or,
// for one image with separable kernels and L >= 5, step 0, then step 1 beside
// work-groups that compose the inputs of steps 3 .. L-2 from step 1's input
// (the adjoint is linear, so several steps fold into banded 1-D products),
// then steps 2 .. L-2 together.
#include "common.hpp"
#include "kernels.hpp"

namespace cc {

// All steps s = L-2 .. 1 in one launch.  A work-group owns a T x T tile
// of level 1 and works from the coarsest level down: the region of
// stack_{s+1} that U_s needs for the rows / columns [a, b) of level s is
// [a/2 - 2, (b-1)/2 + 3) clipped to the grid (every clamped tap index falls in
// it; at most T/2 + 4 rows / columns for levels >= 2), so each work-group
// recomputes, in LDS, the small coarse regions its tile depends on.  U_1 is
// written for the tile; for s >= 2 the work-group writes the part of U_s that
// lies under its tile, so every output is written exactly once.
constexpr int UF_CH = MAXL - 1;  // channels of stack_2 at most (L - 2 < 6)

template <int T, bool SH>
__device__ __forceinline__ void ups_fwd_body(const UpsFwdArgs& a, const int bid) {
  constexpr int UF_R = T / 2 + 4;  // largest region side at levels >= 2
  // every level s <= L-2 keeps at least one row / column of the tile to write
  static_assert((T >> (MAXL - 3)) >= 1 && T % 2 == 0, "ups_fwd tile too small");
  __shared__ float s_st[2][UF_CH * UF_R * UF_R];
  __shared__ float s_w2[SH ? UPS_SHARED_TAPS : 1];
  constexpr int NQ = (UF_R * UF_R + 255) / 256;  // region values per thread at levels >= 2
  const int L = a.geo.L, tid = threadIdx.x;
  constexpr bool shared = SH;
  if (shared && tid < UPS_SHARED_TAPS) s_w2[tid] = a.ups_w[tid];
  const int h1 = a.geo.lh[1], w1 = a.geo.lw[1];
  const int ntx = (w1 + T - 1) / T;
  const int r0 = (bid / ntx) * T, c0 = (bid % ntx) * T;
  // regions [ra, rb) x [ca, cb) per level
  int ra[MAXL], rb[MAXL], ca[MAXL], cb[MAXL];
  ra[1] = r0; rb[1] = min(r0 + T, h1); ca[1] = c0; cb[1] = min(c0 + T, w1);
  for (int l = 1; l + 1 < L; ++l) {
    ra[l + 1] = max(0, (ra[l] >> 1) - 2); rb[l + 1] = min(a.geo.lh[l + 1], ((rb[l] - 1) >> 1) + 3);
    ca[l + 1] = max(0, (ca[l] >> 1) - 2); cb[l + 1] = min(a.geo.lw[l + 1], ((cb[l] - 1) >> 1) + 3);
  }
  // the latents of every level's region (channel 0 of its stack), all read up
  // front; quantised where they are used
  const float alpha = proxy_alpha(a.u, a.quant, a.geo.n_lat);
  float py[MAXL][NQ], pu[MAXL][NQ];
#pragma unroll
  for (int l = 2; l < MAXL; ++l)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      py[l][q] = 0.0f;
      pu[l][q] = 0.0f;
      const int p = tid + 256 * q;
      if (l < L && p < (rb[l] - ra[l]) * (cb[l] - ca[l])) {
        const int nc = cb[l] - ca[l];
        const int idx = a.geo.loff[l] + (ra[l] + p / nc) * a.geo.lw[l] + ca[l] + p % nc;
        py[l][q] = a.y[idx];
        if (uses_noise(a.quant)) pu[l][q] = a.u[idx];
      }
    }
  // stack_{L-1} = y_hat_{L-1} on its region
#pragma unroll
  for (int l = 2; l < MAXL; ++l)
    if (l == L - 1) {
      const int n = (rb[l] - ra[l]) * (cb[l] - ca[l]);
      float* dst = s_st[l & 1];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int p = tid + 256 * q;
        if (p < n) dst[p] = quantise_raw(py[l][q], pu[l][q], a.quant, alpha);
      }
    }
  __syncthreads();
#pragma unroll
  for (int s = MAXL - 2; s >= 1; --s) {
    if (s > L - 2) continue;
    const float* src = s_st[(s + 1) & 1];
    float* dst = s_st[s & 1];
    const float* taps = shared ? a.ups_w : a.ups_w + (size_t)s * 2 * UPS_K;
    const int nci = L - 1 - s;  // channels of stack_{s+1}
    const int sr = rb[s + 1] - ra[s + 1], sc = cb[s + 1] - ca[s + 1];
    const int nr = rb[s] - ra[s], nc = cb[s] - ca[s];
    const int hi = a.geo.lh[s + 1], wi = a.geo.lw[s + 1], ws = a.geo.lw[s];
    // the part of level s under this tile (written to global for s >= 2)
    const int oa = r0 >> (s - 1), ob = min((r0 + T) >> (s - 1), a.geo.lh[s]);
    const int oc = c0 >> (s - 1), od = min((c0 + T) >> (s - 1), ws);
    float* up = a.up_out[s];
    const size_t plane = (size_t)a.geo.lh[s] * ws;
    for (int p = tid; p < nr * nc; p += 256) {
      const int i = ra[s] + p / nc, j = ca[s] + p % nc;
      int ro[4], co[4];
      float vt[4], ht[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ky = 2 * q + 1 - (i & 1), kx = 2 * q + 1 - (j & 1);
        ro[q] = clampi((i + UPS_P - ky) >> 1, 0, hi - 1) - ra[s + 1];
        co[q] = clampi((j + UPS_P - kx) >> 1, 0, wi - 1) - ca[s + 1];
        vt[q] = shared ? 0.0f : taps[ky];
        ht[q] = shared ? 0.0f : taps[UPS_K + kx];
      }
      const bool owned = s == 1 || (i >= oa && i < ob && j >= oc && j < od);
      const int ky0 = 1 - (i & 1), kx0 = 1 - (j & 1);
      for (int c = 0; c < nci; ++c) {
        const float* in = src + c * sr * sc;
        float acc = 0.0f;
        if constexpr (SH) {
#pragma unroll
          for (int q1 = 0; q1 < 4; ++q1)
#pragma unroll
            for (int q2 = 0; q2 < 4; ++q2)
              acc = __builtin_fmaf(s_w2[(2 * q1 + ky0) * UPS_K + 2 * q2 + kx0], in[ro[q1] * sc + co[q2]], acc);
        } else {
#pragma unroll
          for (int q1 = 0; q1 < 4; ++q1) {
            float rr = 0.0f;
#pragma unroll
            for (int q2 = 0; q2 < 4; ++q2) rr += ht[q2] * in[ro[q1] * sc + co[q2]];
            acc += vt[q1] * rr;
          }
        }
        if (s > 1) dst[(c + 1) * nr * nc + p] = acc;
        if (owned) up[c * plane + i * ws + j] = acc;
      }
    }
    if (s > 1) {  // channel 0 of stack_s = y_hat_s
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int p = tid + 256 * q;
        if (p < nr * nc) dst[p] = quantise_raw(py[s][q], pu[s][q], a.quant, alpha);
      }
    }
    __syncthreads();
  }
}

// Adjoint of step s.  One work-group per UT x UT tile of input positions
// (level s+1) and chunk of channels, one thread per position.  With padded input
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

// A block takes one input tile and the channels [chunk cpb, chunk cpb + cpb)
// of stack_{s+1} in turn (the next channel's output-gradient region is
// fetched into registers while the current one is processed); the tap
// gradients of all its channels go to one partial row.
// (explicit FMAs: every kernel built from this body rounds identically)
template <bool SH>
__device__ __forceinline__ void ups_bwd_body(const UpsBwdArgs& a, const int bid, const int ntiles, const int chunk) {
  __shared__ float s_g[UR_N * UR_N];
  __shared__ float s_T[UR_N * UP_N];   // [output row][padded column]
  __shared__ float s_T2[UP_N * UR_N];  // [padded row][output column]
  __shared__ float s_P[UP_N * UP_N];   // g_pad
  constexpr int NPF = (UR_N * UR_N + 255) / 256;
  const int s = a.s, L = a.geo.L, tid = threadIdx.x;
  const int ho = a.geo.lh[s], wo = a.geo.lw[s], hi = a.geo.lh[s + 1], wi = a.geo.lw[s + 1];
  const int ntx = (wi + UT - 1) / UT;
  const int r0 = (bid / ntx) * UT, c0 = (bid % ntx) * UT;
  const int c_lo = chunk * a.cpb, c_hi = min(L - 1 - s, c_lo + a.cpb);
  constexpr bool shared = SH;
  float v[UPS_K], hh[UPS_K], gv[UPS_K], gh[UPS_K];
#pragma unroll
  for (int k = 0; k < UPS_K; ++k) {
    v[k] = shared ? 0.0f : a.taps[k];
    hh[k] = shared ? 0.0f : a.taps[UPS_K + k];
    gv[k] = 0.0f;
    gh[k] = 0.0f;
  }
  // shared kernel: its taps and their gradients (one accumulator per tap)
  __shared__ float s_w2[SH ? UPS_SHARED_TAPS : 1];
  float gw[SH ? UPS_SHARED_TAPS : 1];
#pragma unroll
  for (int k = 0; k < (SH ? UPS_SHARED_TAPS : 1); ++k) gw[k] = 0.0f;
  if (shared && tid < UPS_SHARED_TAPS) s_w2[tid] = a.taps[tid];
  const int jr0 = 2 * r0 - 7, jc0 = 2 * c0 - 7;
  const int lo = a.geo.loff[s + 1];
  // the thread's input position (one per thread) and, per channel, its
  // forward value (the tap gradients' input): fetched with the channel's
  // output-gradient region, a channel ahead
  const int my_r = r0 + tid / UT, my_c = c0 + tid % UT;
  const bool my_in = my_r < hi && my_c < wi;
  const int my_idx = my_r * wi + my_c;
  const float alpha = proxy_alpha(a.u, a.quant, a.geo.n_lat);
  float pf[NPF], pin = 0.0f;
  auto fetch = [&](int ch) {
    const float* gin = a.g_in + (size_t)ch * ho * wo;
    int t = tid;
    asm volatile("" : "+v"(t));
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      const int p = t + 256 * q;
      const int jr = jr0 + p / UR_N, jc = jc0 + p % UR_N;
      pf[q] = (p < UR_N * UR_N && jr >= 0 && jr < ho && jc >= 0 && jc < wo) ? gin[jr * wo + jc] : 0.0f;
    }
    pin = !my_in ? 0.0f
                 : ch == 0 ? quantise(a.y, a.u, lo + my_idx, a.quant, alpha)
                           : a.up_in[(size_t)(ch - 1) * hi * wi + my_idx];
  };
  fetch(c_lo);
  for (int ch = c_lo; ch < c_hi; ++ch) {
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      const int p = tid + 256 * q;
      if (p < UR_N * UR_N) s_g[p] = pf[q];
    }
    const float inval = pin;
    __syncthreads();
    if (ch + 1 < c_hi) fetch(ch + 1);
    // the thread's indices pass through an empty asm statement so that the
    // LDS addresses below are formed per channel rather than held in
    // registers across the loop
    int t = tid;
    asm volatile("" : "+v"(t));
    const int tr = t / UT, tc = t % UT, r = r0 + tr, c = c0 + tc;
    const bool in_tile = r < hi && c < wi;
    // padded indices (local to the tile frame) that clamp to r / c; -1 = none
    int ca[5], cb[5];
    ca[0] = tr + 2; ca[1] = r == 0 ? 1 : -1; ca[2] = r == 0 ? 0 : -1;
    ca[3] = r == hi - 1 ? tr + 3 : -1; ca[4] = r == hi - 1 ? tr + 4 : -1;
    cb[0] = tc + 2; cb[1] = c == 0 ? 1 : -1; cb[2] = c == 0 ? 0 : -1;
    cb[3] = c == wi - 1 ? tc + 3 : -1; cb[4] = c == wi - 1 ? tc + 4 : -1;
    const int idx = r * wi + c;
    for (int p = t; !shared && p < UR_N * UP_N; p += 256) {
      {  // T[row][pc] = sum_kx h[kx] g[row][2 pc + kx]
        const int row = p / UP_N, pc = p % UP_N;
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < UPS_K; ++k) acc = __builtin_fmaf(hh[k], s_g[row * UR_N + 2 * pc + k], acc);
        s_T[p] = acc;
      }
      {  // T2[pr][col] = sum_ky v[ky] g[2 pr + ky][col]
        const int pr = p / UR_N, col = p % UR_N;
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < UPS_K; ++k) acc = __builtin_fmaf(v[k], s_g[(2 * pr + k) * UR_N + col], acc);
        s_T2[p] = acc;
      }
    }
    __syncthreads();
    for (int p = t; p < UP_N * UP_N; p += 256) {
      const int pr = p / UP_N, pc = p % UP_N;
      float acc = 0.0f;
      if constexpr (SH) {  // g_pad[pr][pc] = sum_{ky, kx} w[ky][kx] g[2 pr + ky][2 pc + kx]
#pragma unroll
        for (int ky = 0; ky < UPS_K; ++ky)
#pragma unroll
          for (int kx = 0; kx < UPS_K; ++kx)
            acc = __builtin_fmaf(s_w2[ky * UPS_K + kx], s_g[(2 * pr + ky) * UR_N + 2 * pc + kx], acc);
      } else {
#pragma unroll
        for (int k = 0; k < UPS_K; ++k) acc = __builtin_fmaf(v[k], s_T[(2 * pr + k) * UP_N + pc], acc);
      }
      s_P[p] = acc;
    }
    __syncthreads();
    if (in_tile) {
      float gsum = 0.0f;
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        if (ca[i] < 0) continue;
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          if (cb[j] < 0) continue;
          gsum += s_P[ca[i] * UP_N + cb[j]];
          if constexpr (SH) {
#pragma unroll
            for (int ky = 0; ky < UPS_K; ++ky)
#pragma unroll
              for (int kx = 0; kx < UPS_K; ++kx)
                gw[ky * UPS_K + kx] =
                    __builtin_fmaf(inval, s_g[(2 * ca[i] + ky) * UR_N + 2 * cb[j] + kx], gw[ky * UPS_K + kx]);
          } else {
#pragma unroll
            for (int k = 0; k < UPS_K; ++k) {
              gv[k] = __builtin_fmaf(inval, s_T[(2 * ca[i] + k) * UP_N + cb[j]], gv[k]);
              gh[k] = __builtin_fmaf(inval, s_T2[ca[i] * UR_N + 2 * cb[j] + k], gh[k]);
            }
          }
        }
      }
      if (ch == 0) a.g_y[idx] = gsum;
      else if (a.g_out) a.g_out[(size_t)(ch - 1) * hi * wi + idx] = gsum;
    }
    __syncthreads();
  }
  constexpr int ncol = SH ? UPS_SHARED_TAPS : 2 * UPS_K;
  __shared__ float s_red[4][ncol];
  const int lane = tid & 63, wave = tid >> 6;
  if constexpr (SH) {
#pragma unroll
    for (int k = 0; k < UPS_SHARED_TAPS; ++k) {
      const float a0 = wave_sum(gw[k]);
      if (lane == 0) s_red[wave][k] = a0;
    }
  } else {
#pragma unroll
    for (int k = 0; k < UPS_K; ++k) {
      const float a0 = wave_sum(gv[k]), a1 = wave_sum(gh[k]);
      if (lane == 0) { s_red[wave][k] = a0; s_red[wave][UPS_K + k] = a1; }
    }
  }
  __syncthreads();
  if (tid < ncol) {
    float acc = 0.0f;
    for (int wv = 0; wv < 4; ++wv) acc += s_red[wv][tid];
    a.part[((size_t)chunk * ntiles + bid) * ncol + tid] = acc;
  }
}

// ---- composed coarse adjoint (separable kernels)
// Column q of the 1-D product P_m of m steps (input length n at the coarse
// end) is nonzero only on rows [2^m q - 3 (2^m - 1), 2^m q + 4 (2^m - 1)]:
// one step maps a window at offset o and width B to offset 2 o - 3 and width
// 2 B + 6 (output x takes tap t of input (x + 3 - t) / 2 for the t with
// x + 3 - t even, clamped to the grid; clamped indices of border outputs fall
// in the same windows).  uc_step applies step j (1-based, after j - 1 steps
// already applied; j = 1 starts from the unit vector) to columns q0 ..
// q0 + nq - 1, reading windows of width B_{j-1} from src and writing width B_j
// to dst; entries on rows outside [0, n_out) are zero.
__device__ __forceinline__ int uc_width(int j) { return 7 * ((1 << j) - 1) + 1; }
__device__ __forceinline__ int uc_offset(int j, int q) { return (1 << j) * q - 3 * ((1 << j) - 1); }
__device__ __forceinline__ void uc_step(const float* tp, int n_in, int n_out, int j, int q0, int nq,
                                        const float* src, float* dst) {
  const int bs = uc_width(j - 1), bd = uc_width(j);
  for (int p = threadIdx.x; p < nq * bd; p += 256) {
    const int c = p / bd, e = p % bd, q = q0 + c;
    const int os = uc_offset(j - 1, q), x = uc_offset(j, q) + e;
    float acc = 0.0f;
    if (x >= 0 && x < n_out) {
      const int par = (x + 3) & 1;
#pragma unroll
      for (int u = 0; u < UPS_K / 2; ++u) {
        const int t = 2 * u + par;
        const float w = tp[t];
        const int i = clampi((x + 3 - t) >> 1, 0, n_in - 1) - os;
        const float v = j == 1 ? (i == 0 ? 1.0f : 0.0f) : ((i >= 0 && i < bs) ? src[c * bs + i] : 0.0f);
        acc = __builtin_fmaf(w, v, acc);
      }
    }
    dst[p] = acc;
  }
}

// Work-group b of the composing part: step s (3 <= s <= L-2), one latent level
// above it and UC_R rows of G_s.  Builds the windows of Cv for its rows, runs
// the vertical pass Vt[r][x] = sum_i Cv[i][r] G_1[i][x] over the union of the
// rows' windows (G_1 read once, four columns per lane, the two halves of a
// wave taking alternate rows), then the horizontal part as the adjoints of
// the steps' horizontal passes one after the other on its UC_R rows (1-D, in
// LDS): an input j takes sum_t h[t] g[2 m' - 3 + t] over the padded indices
// m' that clamp to it (j, and the two beyond the border for border inputs).
__device__ __forceinline__ void ups_compose_body(const UpsComposeArgs& a, const int b) {
  __shared__ __align__(16) float pool[UC_POOL];
  __shared__ float s_tap[MAXL][2 * UPS_K];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int s = 3;
  while (b >= a.first[s + 1]) ++s;
  const int m = s - 1, h1 = a.geo.lh[1], w1 = a.geo.lw[1], hs = a.geo.lh[s];
  const int nrb = (hs + UC_R - 1) / UC_R, local = b - a.first[s];
  const int ch = local / nrb, r0 = (local % nrb) * UC_R, nr = min(UC_R, hs - r0);
  const int bm = uc_width(m), bp = uc_width(m - 1), umax = (UC_R - 1) * (1 << m) + bm;
  float* cv0 = pool;                    // Cv windows [UC_R][bm]
  float* cv1 = cv0 + UC_R * bm;         // [UC_R][bp]
  float* cvu = cv1 + UC_R * bp;         // [UC_R][umax]: Cv over the union of rows
  float* va = pool + ((cvu - pool + UC_R * umax + 3) & ~3);  // [UC_R][w1], 16-byte aligned
  float* vb = va + UC_R * w1;           // [UC_R][w1 / 2]
  if (tid < m * 2 * UPS_K) s_tap[1 + tid / (2 * UPS_K)][tid % (2 * UPS_K)] = a.taps[2 * UPS_K + tid];
  __syncthreads();
  // step j of the recursion is forward step k = s - j; the last (j = m)
  // lands in cv0
  for (int j = 1; j <= m; ++j) {
    const int k = s - j;
    const bool to0 = ((m - j) & 1) == 0;
    uc_step(s_tap[k], a.geo.lh[k + 1], a.geo.lh[k], j, r0, nr, to0 ? cv1 : cv0, to0 ? cv0 : cv1);
    __syncthreads();
  }
  const int ilo = max(0, uc_offset(m, r0)), ihi = min(h1 - 1, uc_offset(m, r0 + nr - 1) + bm - 1);
  for (int p = tid; p < UC_R * umax; p += 256) {
    const int r = p / umax, i = ilo + p % umax, e = i - uc_offset(m, r0 + r);
    cvu[p] = (r < nr && i <= ihi && e >= 0 && e < bm) ? cv0[r * bm + e] : 0.0f;
  }
  __syncthreads();
  const float* g1 = a.g1 + (size_t)(s - 1 + ch) * h1 * w1;
  const int nxg = w1 >> 2, half = lane >> 5;
  for (int base = wave * 32; base < nxg; base += 128) {
    const int xg = base + (lane & 31);
    const bool ok = xg < nxg;
    float4 acc[UC_R];
#pragma unroll
    for (int r = 0; r < UC_R; ++r) acc[r] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (ok) {
#pragma unroll 8
      for (int i = ilo + half; i <= ihi; i += 2) {
        const float4 g = *reinterpret_cast<const float4*>(g1 + (size_t)i * w1 + 4 * xg);
#pragma unroll
        for (int r = 0; r < UC_R; ++r) {
          const float c = cvu[r * umax + i - ilo];
          acc[r].x = __builtin_fmaf(c, g.x, acc[r].x);
          acc[r].y = __builtin_fmaf(c, g.y, acc[r].y);
          acc[r].z = __builtin_fmaf(c, g.z, acc[r].z);
          acc[r].w = __builtin_fmaf(c, g.w, acc[r].w);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < UC_R; ++r) {
      acc[r].x += __shfl_xor(acc[r].x, 32);
      acc[r].y += __shfl_xor(acc[r].y, 32);
      acc[r].z += __shfl_xor(acc[r].z, 32);
      acc[r].w += __shfl_xor(acc[r].w, 32);
      if (ok && half == 0) *reinterpret_cast<float4*>(va + r * w1 + 4 * xg) = acc[r];
    }
  }
  __syncthreads();
  // horizontal: adjoints of steps 1 .. s-1 in turn; the last writes G_s
  float* out = a.gs[s] + (size_t)ch * hs * a.geo.lw[s] + (size_t)r0 * a.geo.lw[s];
  for (int k = 1; k <= m; ++k) {
    const int n_out = a.geo.lw[k], n_in = a.geo.lw[k + 1];
    const float* src = (k & 1) ? va : vb;
    float* dst = k == m ? out : ((k & 1) ? vb : va);
    const float* h = s_tap[k] + UPS_K;
    for (int p = tid; p < nr * n_in; p += 256) {
      const int r = p / n_in, j = p % n_in;
      const float* g = src + r * n_out;
      float acc = 0.0f;
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const int mp = q == 0 ? j : (q == 1 ? -1 : (q == 2 ? -2 : (q == 3 ? n_in : n_in + 1)));
        const bool use = q == 0 || (q <= 2 ? j == 0 : j == n_in - 1);
        if (!use) continue;
#pragma unroll
        for (int t = 0; t < UPS_K; ++t) {
          const int x = 2 * mp - 3 + t;
          if (x >= 0 && x < n_out) acc = __builtin_fmaf(h[t], g[x], acc);
        }
      }
      dst[r * n_in + j] = acc;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void ups_bwd_coarse_kernel(UpsBwdArgs st1, int st1_tiles, int st1_wgs,
                                                             UpsComposeArgs c) {
  const int b = blockIdx.x;
  if (b < st1_wgs) ups_bwd_body<false>(st1, b % st1_tiles, st1_tiles, b / st1_tiles);
  else ups_compose_body(c, b - st1_wgs);
}

__global__ __launch_bounds__(256) void ups_bwd_steps_kernel(UpsBwdSteps m) {
  int k = 0;
  while (k + 1 < m.n && (int)blockIdx.x >= m.first[k + 1]) ++k;
  const int local = blockIdx.x - m.first[k];
  ups_bwd_body<false>(m.st[k], local % m.tiles[k], m.tiles[k], local / m.tiles[k]);
}

__global__ void ups_expand_kernel(const float* __restrict__ src, float* __restrict__ dst, int n_steps, int shared) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (shared) {
    if (t >= UPS_SHARED_TAPS) return;
    const int ky = t / UPS_K - 2, kx = t % UPS_K - 2;
    dst[t] = (ky >= 0 && ky < 4 && kx >= 0 && kx < 4) ? src[ky * 4 + kx] : 0.0f;
  } else {
    if (t >= n_steps * 2 * UPS_K) return;
    const int row = t / UPS_K, k = t % UPS_K - 2;
    dst[t] = (k >= 0 && k < 4) ? src[row * 4 + k] : 0.0f;
  }
}

template <bool SH>
__global__ __launch_bounds__(256) void ups_fwd_kernel_t(UpsFwdArgs a) { ups_fwd_body<UF_T, SH>(a, blockIdx.x); }
template <int T, bool SH>
__global__ __launch_bounds__(256) void ups_fwd_kernel_batch_t(const UpsFwdArgs* __restrict__ d,
                                                              const WorkItem* __restrict__ w) {
  const WorkItem it = w[blockIdx.x];
  ups_fwd_body<T, SH>(d[it.img], it.bid);
}
template <bool SH>
__global__ __launch_bounds__(256) void ups_bwd_kernel_t(UpsBwdArgs a) {
  ups_bwd_body<SH>(a, blockIdx.x, gridDim.x, blockIdx.y);
}
template <bool SH>
__global__ __launch_bounds__(256) void ups_bwd_kernel_batch_t(const UpsBwdArgs* __restrict__ d,
                                                              const WorkItem* __restrict__ w) {
  const WorkItem it = w[blockIdx.x];
  ups_bwd_body<SH>(d[it.img], it.bid, it.nblk, it.aux);
}

const void* ups_fwd_kernel_for(bool shared, bool batch, int tile) {
  if (batch && tile == 16)
    return shared ? (const void*)ups_fwd_kernel_batch_t<16, true> : (const void*)ups_fwd_kernel_batch_t<16, false>;
  if (batch && tile == 32)
    return shared ? (const void*)ups_fwd_kernel_batch_t<32, true> : (const void*)ups_fwd_kernel_batch_t<32, false>;
  if (batch) return nullptr;
  return shared ? (const void*)ups_fwd_kernel_t<true> : (const void*)ups_fwd_kernel_t<false>;
}
const void* ups_bwd_kernel_for(bool shared, bool batch) {
  if (batch) return shared ? (const void*)ups_bwd_kernel_batch_t<true> : (const void*)ups_bwd_kernel_batch_t<false>;
  return shared ? (const void*)ups_bwd_kernel_t<true> : (const void*)ups_bwd_kernel_t<false>;
}

}  // namespace cc

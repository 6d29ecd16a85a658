// Warm-start network on gfx950 (Section IV-B's analysis transform, used as
// Section V suggests to initialise per-image fine-tuning).
//
//   trunk  f_k = bf16(ReLU(conv3x3_s2(f_{k-1}; W_k) + b_k)), k = 1..4, 32 channels
//   heads  y_l = V_l . f_l + beta_l (l = 1..4); y_5, y_6 from f_4 pooled by 2, 4;
//          y_0 = conv3x3(x) + beta_0 + V_0 . f_1 (nearest 2x); theta = P mean(f_4) + pi
//
// The convolutions are implicit GEMMs on the bfloat16 matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation):
//   forward      D[32 pixels][32 out]  = im2col(f_{k-1}) [32][9 C_in] x W^T
//   data adjoint D[32 positions][32 in] = dpre_k gathered over the (at most
//                2 x 2) taps that reach each position x W, one GEMM per
//                parity class of the position so that the taps are fixed
//   weight grad  D[32 out][32 in] per tap = dpre_k^T [32][16 px] x im2col
//                [16 px][32], pixel tiles transposed through LDS
// Heads, pooling and the loss run on the vector ALUs in FP32.  Every
// reduction writes per-block partial rows that a fixed-order column sum
// combines, so results are bit-identical from run to run.
#include "common.hpp"
#include "kernels.hpp"
#include "bf16.hpp"

namespace cc {

// The 32 channels of a bfloat16 feature-map position as FP32.
__device__ __forceinline__ void load_feat(const uint16_t* p, float (&v)[WS_CH]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint4 u = reinterpret_cast<const uint4*>(p)[q];
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      v[q * 8 + 2 * e] = bf16_f(w[e] & 0xffffu);
      v[q * 8 + 2 * e + 1] = bf16_f(w[e] >> 16);
    }
  }
}

// Gradient of the loss w.r.t. latent q (packed index) of image b: given by
// the caller, or that of the regression loss (sy = 2 / (n_lat B)).
__device__ __forceinline__ float dlat(const WarmArgs& a, int b, int q) {
  const size_t i = (size_t)b * a.n_lat + q;
  return a.gy_in ? a.gy_in[i] : (a.y[i] - a.y_t[i]) * a.sy;
}

// ------------------------------------------------------------ parameters

// Rounded copy of the master parameters and the bfloat16 GEMM operands.
__global__ __launch_bounds__(256) void warm_prep_kernel(WarmArgs a) {
  const int n_pad = WS_CH * 5;  // k = 1 operand columns 27..31
  for (int i = blockIdx.x * 256 + threadIdx.x; i < a.n_net + n_pad; i += gridDim.x * 256) {
    if (i >= a.n_net) {
      const int t = i - a.n_net;
      a.wf[1][(t / 5) * 32 + 27 + t % 5] = 0;
      continue;
    }
    const float v = a.net[i];
    float r = v;
    bool done = false;
    for (int k = 1; k <= 4 && !done; ++k) {
      const int cin = k == 1 ? 3 : WS_CH, nw = WS_CH * 9 * cin, o = a.conv_off[k];
      if (i >= o && i < o + nw) {
        const int local = i - o, co = local / (9 * cin), rem = local % (9 * cin);
        const uint16_t h = bf16_bits(v);
        a.wf[k][co * (k == 1 ? 32 : 9 * WS_CH) + rem] = h;
        if (k >= 2 && a.wt[k]) a.wt[k][((rem / WS_CH) * WS_CH + rem % WS_CH) * WS_CH + co] = h;  // backward only
        r = bf16_f(h);
        done = true;
      } else if (i >= o + nw && i < o + nw + WS_CH) {
        done = true;  // bias: kept
      }
    }
    if (!done) {
      if (i >= a.ptheta) {
        if (i < a.ptheta + a.n_theta * WS_CH) r = round_bf16(v);  // P; pi kept
      } else {
        int l = 6;
        while (l > 0 && i < a.head_off[l]) --l;
        const int local = i - a.head_off[l];
        if (local < WS_CH || local > WS_CH) r = round_bf16(v);  // V_l and K_0; beta_l kept
      }
    }
    a.net_r[i] = r;
  }
}

// ------------------------------------------------------------ trunk forward

template <int CIN>
__global__ __launch_bounds__(256) void warm_conv_fwd_kernel(WarmArgs a, int k) {
  constexpr int KP = CIN == 3 ? 32 : 9 * CIN;
  constexpr int NK = KP / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, hi = lane >> 5, m = lane & 31;
  const int ho = a.h[k], wo = a.w[k], hin = a.h[k - 1], win = a.w[k - 1];
  const int tiles_x = (wo + 31) / 32;
  const long n_tiles = (long)a.B * ho * tiles_x;
  bf16x8 bw[NK];
#pragma unroll
  for (int kk = 0; kk < NK; ++kk) bw[kk] = load8(a.wf[k] + m * KP + kk * 16 + hi * 8);
  const float bias = a.net[a.conv_off[k] + WS_CH * 9 * CIN + m];
  const uint16_t* fin = a.f[k - 1];
  uint16_t* fout = a.f[k];
  for (long t = (long)blockIdx.x * 4 + wave; t < n_tiles; t += (long)gridDim.x * 4) {
    const int tx = (int)(t % tiles_x);
    const long r0 = t / tiles_x;
    const int i = (int)(r0 % ho), b = (int)(r0 / ho);
    const int j = tx * 32 + m;
    f32x16 acc = {};
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) {
      bf16x8 av = zero8();
      if constexpr (CIN == 3) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int kp = kk * 16 + hi * 8 + e;
          float v = 0.0f;
          if (kp < 27 && j < wo) {
            const int tap = kp / 3, c = kp % 3;
            const int iy = 2 * i + tap / 3 - 1, ix = 2 * j + tap % 3 - 1;
            if (iy >= 0 && iy < hin && ix >= 0 && ix < win)
              v = a.x[(((size_t)b * 3 + c) * hin + iy) * win + ix];
          }
          av[e] = __builtin_bit_cast(__bf16, bf16_bits(v));
        }
      } else {
        const int kb = kk * 16 + hi * 8, tap = kb / WS_CH, ci0 = kb % WS_CH;
        const int iy = 2 * i + tap / 3 - 1, ix = 2 * j + tap % 3 - 1;
        if (j < wo && iy >= 0 && iy < hin && ix >= 0 && ix < win)
          av = load8(fin + (((size_t)b * hin + iy) * win + ix) * WS_CH + ci0);
      }
      acc = mfma_bf16(av, bw[kk], acc);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int jj = tx * 32 + dfeat(r, hi);
      if (jj < wo) fout[(((size_t)b * ho + i) * wo + jj) * WS_CH + m] = bf16_bits(fmaxf(acc[r] + bias, 0.0f));
    }
  }
}

// ------------------------------------------------------------ heads forward

__global__ __launch_bounds__(256) void warm_heads_fwd_kernel(WarmArgs a, int with_loss) {
  __shared__ float s_red[4];
  const float* nr = a.net_r;
  float lp = 0.0f;
  const long n = (long)a.B * a.n_lat;
  for (long t = (long)blockIdx.x * 256 + threadIdx.x; t < n; t += (long)gridDim.x * 256) {
    const int b = (int)(t / a.n_lat), q = (int)(t % a.n_lat);
    int l = 0;
    while (l < 6 && q >= a.loff[l + 1]) ++l;
    const int wl = a.lw[l], loc = q - a.loff[l], i = loc / wl, j = loc % wl;
    const float* V = nr + a.head_off[l];
    float f[WS_CH];
    float yv = V[WS_CH];  // beta_l
    if (l == 0) {
      const float* K = V + WS_CH + 1;
      float acc = 0.0f;
      for (int ky = 0; ky < 3; ++ky)
        for (int kx = 0; kx < 3; ++kx) {
          const int iy = i + ky - 1, ix = j + kx - 1;
          if (iy < 0 || iy >= a.H || ix < 0 || ix >= a.W) continue;
#pragma unroll
          for (int c = 0; c < 3; ++c)
            acc += K[(ky * 3 + kx) * 3 + c] * round_bf16(a.x[(((size_t)b * 3 + c) * a.H + iy) * a.W + ix]);
        }
      load_feat(a.f[1] + (((size_t)b * a.h[1] + i / 2) * a.w[1] + j / 2) * WS_CH, f);
      float g = 0.0f;
#pragma unroll
      for (int c = 0; c < WS_CH; ++c) g += V[c] * f[c];
      yv += acc + g;
    } else if (l <= 4) {
      load_feat(a.f[l] + (((size_t)b * a.h[l] + i) * a.w[l] + j) * WS_CH, f);
      float acc = 0.0f;
#pragma unroll
      for (int c = 0; c < WS_CH; ++c) acc += V[c] * f[c];
      yv += acc;
    } else {
      const int s = l == 5 ? 2 : 4;
      float sum[WS_CH];
#pragma unroll
      for (int c = 0; c < WS_CH; ++c) sum[c] = 0.0f;
      for (int u = 0; u < s; ++u)
        for (int v = 0; v < s; ++v) {
          load_feat(a.f[4] + (((size_t)b * a.h[4] + i * s + u) * a.w[4] + j * s + v) * WS_CH, f);
#pragma unroll
          for (int c = 0; c < WS_CH; ++c) sum[c] += f[c];
        }
      const float inv = 1.0f / (float)(s * s);
      float acc = 0.0f;
#pragma unroll
      for (int c = 0; c < WS_CH; ++c) acc += V[c] * (sum[c] * inv);
      yv += acc;
    }
    a.y[t] = yv;
    if (with_loss && a.y_t) {
      const float d = yv - a.y_t[t];
      lp += d * d;
    }
  }
  if (with_loss) {
    lp = wave_sum(lp);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = lp;
    __syncthreads();
    if (threadIdx.x == 0) a.lpart_y[blockIdx.x] = (s_red[0] + s_red[1] + s_red[2] + s_red[3]) * (0.5f * a.sy);
  }
}

// One work-group per image: global average pool of f_4, theta = P gap + pi;
// backward: the parameter loss, dtheta, the P / pi gradient row of this
// image and dgap = P^T dtheta.
__global__ __launch_bounds__(256) void warm_theta_kernel(WarmArgs a, int bwd) {
  __shared__ float s_part[8][WS_CH];
  __shared__ float s_gap[WS_CH];
  __shared__ float s_dth[WS_MAX_THETA];
  __shared__ float s_red[4];
  const int b = blockIdx.x, tid = threadIdx.x, c = tid & 31, g8 = tid >> 5;
  const int np = a.h[4] * a.w[4];
  const uint16_t* f4 = a.f[4] + (size_t)b * np * WS_CH;
  float s = 0.0f;
  for (int p = g8; p < np; p += 8) s += bf16_f(f4[(size_t)p * WS_CH + c]);
  s_part[g8][c] = s;
  __syncthreads();
  if (tid < WS_CH) {
    float t = 0.0f;
    for (int q = 0; q < 8; ++q) t += s_part[q][tid];
    t *= 1.0f / (float)np;
    s_gap[tid] = t;
    a.gap[b * WS_CH + tid] = t;
  }
  __syncthreads();
  const float* P = a.net_r + a.ptheta;
  const float* pi = P + (size_t)a.n_theta * WS_CH;
  float lp = 0.0f;
  for (int t = tid; t < a.n_theta; t += 256) {
    float acc = 0.0f;
#pragma unroll
    for (int q = 0; q < WS_CH; ++q) acc += P[(size_t)t * WS_CH + q] * s_gap[q];
    const float th = acc + pi[t];
    a.theta[(size_t)b * a.n_theta + t] = th;
    if (bwd) {
      float dth;
      if (a.gth_in) {
        dth = a.gth_in[(size_t)b * a.n_theta + t];
      } else {
        const float d = th - a.th_t[(size_t)b * a.n_theta + t];
        lp += d * d;
        dth = d * a.sth;
      }
      s_dth[t] = dth;
      float* row = a.part_th + (size_t)b * a.n_theta * (WS_CH + 1);
#pragma unroll
      for (int q = 0; q < WS_CH; ++q) row[(size_t)t * WS_CH + q] = dth * s_gap[q];
      row[(size_t)a.n_theta * WS_CH + t] = dth;
    }
  }
  if (!bwd) return;
  lp = wave_sum(lp);
  if ((tid & 63) == 0) s_red[tid >> 6] = lp;
  __syncthreads();
  if (tid == 0) a.lpart_th[b] = (s_red[0] + s_red[1] + s_red[2] + s_red[3]) * (0.5f * a.sth);
  // dgap[c] = sum_t P[t][c] dtheta[t]: 8 strided partial sums per channel
  float acc = 0.0f;
  for (int t = g8; t < a.n_theta; t += 8) acc += P[(size_t)t * WS_CH + c] * s_dth[t];
  __syncthreads();
  s_part[g8][c] = acc;
  __syncthreads();
  if (tid < WS_CH) {
    float t = 0.0f;
    for (int q = 0; q < 8; ++q) t += s_part[q][tid];
    a.dgap[b * WS_CH + tid] = t;
  }
}

// ------------------------------------------------------------ backward

// Gradient at f_4 from heads 4, 5, 6 and the pooled parameter head, masked
// and rounded into dp_4; partial gradients of heads 4..6.
__global__ __launch_bounds__(256) void warm_df4_kernel(WarmArgs a) {
  __shared__ float s_acc[8][99];
  const int tid = threadIdx.x, c = tid & 31, pg = tid >> 5;
  const int h4 = a.h[4], w4 = a.w[4], np = a.B * h4 * w4;
  const float* nr = a.net_r;
  const float V4 = nr[a.head_off[4] + c], V5 = nr[a.head_off[5] + c], V6 = nr[a.head_off[6] + c];
  const float inv_np = 1.0f / (float)(h4 * w4);
  float pv[3] = {0.0f, 0.0f, 0.0f}, pb[3] = {0.0f, 0.0f, 0.0f};
  const int p0 = blockIdx.x * WS_DF4_POS;
  for (int p = p0 + pg; p < p0 + WS_DF4_POS && p < np; p += 8) {
    const int b = p / (h4 * w4), r = p % (h4 * w4), i = r / w4, j = r % w4;
    const float dy4 = dlat(a, b, a.loff[4] + i * w4 + j);
    const float dy5 = 0.25f * dlat(a, b, a.loff[5] + (i >> 1) * a.lw[5] + (j >> 1));
    const float dy6 = 0.0625f * dlat(a, b, a.loff[6] + (i >> 2) * a.lw[6] + (j >> 2));
    const float fv = bf16_f(a.f[4][(size_t)p * WS_CH + c]);
    const float df = dy4 * V4 + dy5 * V5 + dy6 * V6 + a.dgap[b * WS_CH + c] * inv_np;
    a.dp[4][(size_t)p * WS_CH + c] = bf16_bits(fv > 0.0f ? df : 0.0f);
    pv[0] += dy4 * fv; pv[1] += dy5 * fv; pv[2] += dy6 * fv;
    pb[0] += dy4; pb[1] += dy5; pb[2] += dy6;
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) s_acc[pg][33 * q + c] = pv[q];
  if (c == 0) {
#pragma unroll
    for (int q = 0; q < 3; ++q) s_acc[pg][33 * q + 32] = pb[q];
  }
  __syncthreads();
  if (tid < 99) {
    float t = 0.0f;
    for (int q = 0; q < 8; ++q) t += s_acc[q][tid];
    a.part_h456[(size_t)blockIdx.x * 99 + tid] = t;
  }
}

// Per wave: data adjoint of conv k for one tile of 32 positions of f_{k-1}
// in row i with column parity PX (j = 2 m + PX), row parity PY = i % 2.
// Taps reaching (i, j): rows ky = 1 (even i) or ky = 0, 2 (odd i); the
// same for columns.
template <int PY, int PX>
__device__ __forceinline__ f32x16 adjoint_tile(const WarmArgs& a, int k, int b, int i, int m0, int lane,
                                               const bf16x8 (&wt)[9][2]) {
  const int hi = lane >> 5, mm = m0 + (lane & 31);
  const int hk = a.h[k], wk = a.w[k], wl = a.w[k - 1];
  const bool colok = mm < (wl >> 1);
  const uint16_t* dpk = a.dp[k];
  f32x16 acc = {};
#pragma unroll
  for (int sy = 0; sy < (PY ? 2 : 1); ++sy) {
    const int ky = PY ? (sy == 0 ? 0 : 2) : 1;
    const int oy = PY ? (sy == 0 ? (i + 1) >> 1 : (i - 1) >> 1) : i >> 1;
    const bool rowok = oy < hk;
#pragma unroll
    for (int sx = 0; sx < (PX ? 2 : 1); ++sx) {
      const int kx = PX ? (sx == 0 ? 0 : 2) : 1;
      const int ox = PX ? (sx == 0 ? mm + 1 : mm) : mm;
      const bool ok = rowok && colok && ox < wk;
#pragma unroll
      for (int ch = 0; ch < 2; ++ch) {
        const bf16x8 av = ok ? load8(dpk + (((size_t)b * hk + oy) * wk + ox) * WS_CH + ch * 16 + hi * 8) : zero8();
        acc = mfma_bf16(av, wt[ky * 3 + kx][ch], acc);
      }
    }
  }
  return acc;
}

// dp_{k-1} from dp_k (k = 4, 3, 2) plus the head of level k-1 (and, for
// level 1, the level-0 path through f_1); partial gradients of that head.
__global__ __launch_bounds__(256) void warm_bwd_data_kernel(WarmArgs a, int k) {
  __shared__ float s_acc[4][65];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, hi = lane >> 5, ci = lane & 31;
  const int lv = k - 1, h = a.h[lv], w = a.w[lv];
  const int half = w >> 1, tiles_m = (half + 31) / 32;
  const long n_tiles = (long)a.B * h * 2 * tiles_m;
  bf16x8 wt[9][2];
#pragma unroll
  for (int tap = 0; tap < 9; ++tap)
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) wt[tap][ch] = load8(a.wt[k] + (tap * WS_CH + ci) * WS_CH + ch * 16 + hi * 8);
  const float Vl = a.net_r[a.head_off[lv] + ci];
  const float V0 = a.net_r[a.head_off[0] + ci];
  float pv = 0.0f, pv0 = 0.0f, pb = 0.0f;
  for (long t = (long)blockIdx.x * 4 + wave; t < n_tiles; t += (long)gridDim.x * 4) {
    const int mt = (int)(t % tiles_m);
    long r0 = t / tiles_m;
    const int px = (int)(r0 & 1);
    r0 >>= 1;
    const int i = (int)(r0 % h), b = (int)(r0 / h);
    const int m0 = mt * 32;
    f32x16 acc;
    if ((i & 1) == 0)
      acc = px == 0 ? adjoint_tile<0, 0>(a, k, b, i, m0, lane, wt) : adjoint_tile<0, 1>(a, k, b, i, m0, lane, wt);
    else
      acc = px == 0 ? adjoint_tile<1, 0>(a, k, b, i, m0, lane, wt) : adjoint_tile<1, 1>(a, k, b, i, m0, lane, wt);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int mm = m0 + dfeat(r, hi);
      if (mm >= half) continue;
      const int j = 2 * mm + px;
      const float dyl = dlat(a, b, a.loff[lv] + i * w + j);
      float df = acc[r] + dyl * Vl;
      float dg = 0.0f;
      if (lv == 1) {
        const int W0 = a.lw[0];
        const int q0 = (2 * i) * W0 + 2 * j;
        dg = (dlat(a, b, q0) + dlat(a, b, q0 + 1)) + (dlat(a, b, q0 + W0) + dlat(a, b, q0 + W0 + 1));
        df += dg * V0;
      }
      const size_t idx = (((size_t)b * h + i) * w + j) * WS_CH + ci;
      const float fv = bf16_f(a.f[lv][idx]);
      a.dp[lv][idx] = bf16_bits(fv > 0.0f ? df : 0.0f);
      pv += dyl * fv;
      pv0 += dg * fv;
      if (ci == 0) pb += dyl;
    }
  }
  // lanes ci and ci + 32 hold the two halves of the tile rows
  pv += __shfl_xor(pv, 32, 64);
  pv0 += __shfl_xor(pv0, 32, 64);
  pb += __shfl_xor(pb, 32, 64);
  if (hi == 0) {
    s_acc[wave][ci] = pv;
    s_acc[wave][33 + ci] = pv0;
    if (ci == 0) s_acc[wave][32] = pb;
  }
  __syncthreads();
  const int nv = lv == 1 ? 65 : 33;
  if (threadIdx.x < nv) {
    const float t = ((s_acc[0][threadIdx.x] + s_acc[1][threadIdx.x]) + s_acc[2][threadIdx.x]) + s_acc[3][threadIdx.x];
    if (threadIdx.x < 33)
      a.part_h[lv][(size_t)blockIdx.x * 33 + threadIdx.x] = t;
    else
      a.part_v0[(size_t)blockIdx.x * 32 + threadIdx.x - 33] = t;
  }
}

// beta_0 and the level-0 3x3 kernel: sum over full-resolution positions of
// dy_0 times the rounded image patch.
__global__ __launch_bounds__(256) void warm_head0_grad_kernel(WarmArgs a) {
  __shared__ float s_acc[4][28];
  float acc[28];
#pragma unroll
  for (int q = 0; q < 28; ++q) acc[q] = 0.0f;
  const long n = (long)a.B * a.H * a.W;
  for (long t = (long)blockIdx.x * 256 + threadIdx.x; t < n; t += (long)gridDim.x * 256) {
    const int b = (int)(t / ((long)a.H * a.W)), r = (int)(t % ((long)a.H * a.W)), i = r / a.W, j = r % a.W;
    const float dy = dlat(a, b, r);
    acc[0] += dy;
#pragma unroll
    for (int ky = 0; ky < 3; ++ky)
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        const int iy = i + ky - 1, ix = j + kx - 1;
        const bool in = iy >= 0 && iy < a.H && ix >= 0 && ix < a.W;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float v = in ? round_bf16(a.x[(((size_t)b * 3 + c) * a.H + iy) * a.W + ix]) : 0.0f;
          acc[1 + (ky * 3 + kx) * 3 + c] += dy * v;
        }
      }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 28; ++q) {
    const float s = wave_sum(acc[q]);
    if (lane == 0) s_acc[wave][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < 28) {
    const int q = threadIdx.x;
    a.part_h0[(size_t)blockIdx.x * 28 + q] = ((s_acc[0][q] + s_acc[1][q]) + s_acc[2][q]) + s_acc[3][q];
  }
}

// Weight and bias gradient of conv k: sum over the output pixels p of
// dp_k[p] (x) im2col(f_{k-1})[p], 16 pixels per MFMA step.  Work-group g
// takes pixel chunks [g cpb, (g + 1) cpb), its wave w the chunks w, w + 4, ...
// of that range; the four waves' sums are added in order in LDS.
template <int CIN>
__global__ __launch_bounds__(256) void warm_bwd_weight_kernel(WarmArgs a, int k) {
  constexpr int NT = CIN == 3 ? 1 : 9;          // N tiles of 32 columns
  constexpr int NW = WS_CH * 9 * CIN;           // weight gradients
  __shared__ __align__(16) uint16_t s_a[4][WS_CH][16 + 8];  // dp_k^T per wave (padded rows)
  __shared__ __align__(16) uint16_t s_b[4][WS_CH][16 + 8];  // im2col^T per wave
  __shared__ float s_w[NW + WS_CH];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, hi = lane >> 5, n = lane & 31;
  const int ho = a.h[k], wo = a.w[k], hin = a.h[k - 1], win = a.w[k - 1];
  const long np = (long)a.B * ho * wo;
  const long nchunk = (np + 15) / 16;
  const long cpb = (nchunk + gridDim.x - 1) / gridDim.x;
  const long c_lo = (long)blockIdx.x * cpb, c_hi = c_lo + cpb < nchunk ? c_lo + cpb : nchunk;
  f32x16 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x16{};
  float db = 0.0f;
  const uint16_t* dpk = a.dp[k];
  const uint16_t* fin = a.f[k - 1];
  const int spx = lane >> 2, sc8 = (lane & 3) * 8;  // staging: pixel, first channel
  for (long ch = c_lo + wave; ch < c_hi; ch += 4) {
    const long p0 = ch * 16;
    {  // dp_k rows of 16 pixels, transposed into s_a[channel][pixel]
      const long p = p0 + spx;
      uint4 u = make_uint4(0, 0, 0, 0);
      if (p < np) u = *reinterpret_cast<const uint4*>(dpk + (size_t)p * WS_CH + sc8);
      const uint32_t wv[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        s_a[wave][sc8 + 2 * e][spx] = (uint16_t)(wv[e] & 0xffffu);
        s_a[wave][sc8 + 2 * e + 1][spx] = (uint16_t)(wv[e] >> 16);
      }
    }
    wave_lds_sync();
    const uint4 ua = *reinterpret_cast<const uint4*>(&s_a[wave][n][hi * 8]);
    const bf16x8 av = __builtin_bit_cast(bf16x8, ua);
    {
      const uint32_t wv[4] = {ua.x, ua.y, ua.z, ua.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) db += bf16_f(wv[e] & 0xffffu) + bf16_f(wv[e] >> 16);
    }
    if constexpr (CIN == 3) {
      bf16x8 bv = zero8();
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const long p = p0 + hi * 8 + e;
        float v = 0.0f;
        if (n < 27 && p < np) {
          const int b = (int)(p / ((long)ho * wo)), r = (int)(p % ((long)ho * wo)), i = r / wo, j = r % wo;
          const int tap = n / 3, c = n % 3, iy = 2 * i + tap / 3 - 1, ix = 2 * j + tap % 3 - 1;
          if (iy >= 0 && iy < hin && ix >= 0 && ix < win) v = a.x[(((size_t)b * 3 + c) * hin + iy) * win + ix];
        }
        bv[e] = __builtin_bit_cast(__bf16, bf16_bits(v));
      }
      acc[0] = mfma_bf16(av, bv, acc[0]);
    } else {
      const long p = p0 + spx;
      int b = 0, i = 0, j = 0;
      const bool pin = p < np;
      if (pin) {
        b = (int)(p / ((long)ho * wo));
        const int r = (int)(p % ((long)ho * wo));
        i = r / wo;
        j = r % wo;
      }
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int iy = 2 * i + tap / 3 - 1, ix = 2 * j + tap % 3 - 1;
        uint4 u = make_uint4(0, 0, 0, 0);
        if (pin && iy >= 0 && iy < hin && ix >= 0 && ix < win)
          u = *reinterpret_cast<const uint4*>(fin + (((size_t)b * hin + iy) * win + ix) * WS_CH + sc8);
        wave_lds_sync();  // previous tap's operand reads are complete
        const uint32_t wv[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          s_b[wave][sc8 + 2 * e][spx] = (uint16_t)(wv[e] & 0xffffu);
          s_b[wave][sc8 + 2 * e + 1][spx] = (uint16_t)(wv[e] >> 16);
        }
        wave_lds_sync();
        const bf16x8 bv = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&s_b[wave][n][hi * 8]));
        acc[tap] = mfma_bf16(av, bv, acc[tap]);
      }
    }
    wave_lds_sync();  // s_a is rewritten by the next chunk
  }
  db += __shfl_xor(db, 32, 64);
  // ordered sum of the four waves: acc[t][r] is D[co][col] with
  // co = dfeat(r, hi), col = n (CIN 32: input channel of tap t; CIN 3: k')
  for (int wv = 0; wv < 4; ++wv) {
    if (wave == wv) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int co = dfeat(r, hi);
          int idx = -1;
          if (CIN == 3) {
            if (n < 27) idx = co * 27 + n;
          } else {
            idx = co * 9 * CIN + t * CIN + n;
          }
          if (idx >= 0) s_w[idx] = wv == 0 ? acc[t][r] : s_w[idx] + acc[t][r];
        }
      if (hi == 0) s_w[NW + n] = wv == 0 ? db : s_w[NW + n] + db;
    }
    __syncthreads();
  }
  float* row = a.part_conv[k] + (size_t)blockIdx.x * (NW + WS_CH);
  for (int q = threadIdx.x; q < NW + WS_CH; q += 256) row[q] = s_w[q];
}

const void* warm_conv_fwd_kernel_for(int k) {
  return k == 1 ? (const void*)warm_conv_fwd_kernel<3> : (const void*)warm_conv_fwd_kernel<WS_CH>;
}
const void* warm_bwd_weight_kernel_for(int k) {
  return k == 1 ? (const void*)warm_bwd_weight_kernel<3> : (const void*)warm_bwd_weight_kernel<WS_CH>;
}

}  // namespace cc

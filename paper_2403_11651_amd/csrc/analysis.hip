// Non-overfitted analysis transform on gfx950 (Section IV-B, Eq. (3)):
// y = f_alpha(x), the latent grids of Cool-chic in one forward pass.
//
// 21 ConvNeXt-style blocks (three per latent level, the first of levels
// 1..6 with stride 2), each run as two launches over the positions of its
// output level:
//   ana_dw_kernel   depth-wise 7x7 convolution and the layer normalisation
//                   over channels, FP32; writes the normalised features T in
//                   bfloat16 (position-major, 64 or 16 channels per position)
//   ana_mlp_kernel  the block's 1x1 convolutions on the bfloat16 matrix
//                   cores (v_mfma_f32_32x32x16_bf16, FP32 accumulation),
//                   GELU between them, the identity branch, the bfloat16
//                   block output and, for a level's last block, its latent
//                   head.
// The MLP works transposed: with the weights as the A operand and 32
// positions as the columns, the hidden layer's accumulators (rows = hidden
// units) feed the second product as its B operand without leaving the
// registers: the K order of the second product is permuted to the order the
// accumulators hold the hidden units in, and the second layer's weights are
// read in that order.  A wave takes 32 positions at a time, eight chunks of
// 32 hidden units each; the work-group stages both weight matrices in LDS
// once (rows padded against bank conflicts).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "coolchic.h"
#include "common.hpp"
#include "bf16.hpp"

namespace cc {
namespace {

constexpr int AN_C = 64, AN_HID = 256, AN_K = 7, AN_TAPS = AN_K * AN_K, AN_L = 7, AN_E = 2;
constexpr int AN_BLOCKS = AN_L * (1 + AN_E);
constexpr float AN_LN_EPS = 1e-6f;
constexpr int AN_THREADS = 256;
constexpr int AN_MAX_GRID = 1024;
constexpr int AN_NT = 1;  // 32-position tiles per wave step of the MLP kernel
constexpr int AN_DW_R = 4;  // consecutive positions per lane group of the depth-wise kernel

// Per-block host-side description (offsets in floats into theta, in
// uint16 into the bf16 operand area of the workspace).
struct AnBlock {
  int level, c_in, stride, last, kin, kid;
  long long o_dw_w, o_dw_b, o_ln_g, o_ln_b, o_w1, o_b1, o_w2, o_b2, o_wid, o_bid;
  long long q_w1, q_w2, q_wid;  // bf16 operand offsets
};

struct AnPrepArgs {
  const float* theta;
  uint16_t* q;
  int n_blocks;
  int c_in[AN_BLOCKS], kin[AN_BLOCKS], kid[AN_BLOCKS];
  long long o_w1[AN_BLOCKS], o_w2[AN_BLOCKS], o_wid[AN_BLOCKS];
  long long q_w1[AN_BLOCKS], q_w2[AN_BLOCKS], q_wid[AN_BLOCKS];
  long long n_per[AN_BLOCKS];  // bf16 operand elements of each block
};

struct AnArgs {
  int n, hi, wi, ho, wo;   // images; input and output level sizes
  int c_in, stride, kin, kid;
  const float* x;          // block 0: the image [n][3][hi][wi]
  const uint16_t* fin;     // other blocks: input features [n][hi][wi][64]
  uint16_t* t;             // normalised features [n][ho][wo][kin]
  uint16_t* fout;          // block output [n][ho][wo][64]
  const float *dw_w, *dw_b, *ln_g, *ln_b, *b1, *b2, *bid;
  const uint16_t *w1, *w2, *wid;  // bf16 [256][kin], [64][256], [64][kid]
  const float* head;       // level's last block: head weights [64] then the bias; else null
  float* y;                // [n][n_lat]
  int n_lat, loff;
};

// ------------------------------------------------------------ parameters

// bfloat16 copies of the 1x1 weights, zero-padded to the K the products
// take (16 for the 3 input channels of the first block).
__global__ __launch_bounds__(AN_THREADS) void ana_prep_kernel(AnPrepArgs a) {
  long long i = (long long)blockIdx.x * AN_THREADS + threadIdx.x;
  int b = 0;
  while (b < a.n_blocks && i >= a.n_per[b]) i -= a.n_per[b++];
  if (b >= a.n_blocks) return;
  const int ci = a.c_in[b], kin = a.kin[b], kid = a.kid[b];
  const long long n1 = (long long)AN_HID * kin, n2 = (long long)AN_C * AN_HID;
  float v = 0.0f;
  uint16_t* dst;
  if (i < n1) {
    const int r = (int)(i / kin), k = (int)(i % kin);
    v = k < ci ? a.theta[a.o_w1[b] + (long long)r * ci + k] : 0.0f;
    dst = a.q + a.q_w1[b] + i;
  } else if (i < n1 + n2) {
    i -= n1;
    v = a.theta[a.o_w2[b] + i];
    dst = a.q + a.q_w2[b] + i;
  } else {
    i -= n1 + n2;
    const int r = (int)(i / kid), k = (int)(i % kid);
    v = k < ci ? a.theta[a.o_wid[b] + (long long)r * ci + k] : 0.0f;
    dst = a.q + a.q_wid[b] + i;
  }
  *dst = bf16_bits(v);
}

// ------------------------------------------------- depth-wise conv + norm

// 64 input channels: eight lanes per group of AN_DW_R positions of a row,
// eight channels each; the normalisation's sums run over the eight lanes.  The first block (3 image
// channels): one thread per position, T padded to 16 channels.
template <int S>
__global__ __launch_bounds__(AN_THREADS) void ana_dw_kernel(AnArgs a) {
  __shared__ float s_w[AN_C * AN_TAPS];
  const int tid = threadIdx.x;
  const long long npx = (long long)a.n * a.ho * a.wo;
  if (a.c_in == 3) {
    const long long px = (long long)blockIdx.x * AN_THREADS + tid;
    if (px >= npx) return;
    const int img = (int)(px / ((long long)a.ho * a.wo)), r = (int)(px % ((long long)a.ho * a.wo));
    const int i = r / a.wo, j = r % a.wo;
    float acc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float s = a.dw_b[c];
      const float* xc = a.x + ((size_t)img * 3 + c) * a.hi * a.wi;
      for (int dy = 0; dy < AN_K; ++dy) {
        const int iy = a.stride * i + dy - 3;
        if (iy < 0 || iy >= a.hi) continue;
        for (int dx = 0; dx < AN_K; ++dx) {
          const int ix = a.stride * j + dx - 3;
          if (ix >= 0 && ix < a.wi) s = __builtin_fmaf(a.dw_w[c * AN_TAPS + dy * AN_K + dx], xc[iy * a.wi + ix], s);
        }
      }
      acc[c] = s;
    }
    const float mean = (acc[0] + acc[1] + acc[2]) / 3.0f;
    float var = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) var += (acc[c] - mean) * (acc[c] - mean);
    const float rs = 1.0f / sqrtf(var / 3.0f + AN_LN_EPS);
    uint16_t o[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) o[c] = c < 3 ? bf16_bits((acc[c] - mean) * rs * a.ln_g[c] + a.ln_b[c]) : 0;
    uint4* dst = reinterpret_cast<uint4*>(a.t + px * 16);
    dst[0] = make_uint4(o[0] | (o[1] << 16), o[2] | (o[3] << 16), o[4] | (o[5] << 16), o[6] | (o[7] << 16));
    dst[1] = make_uint4(o[8] | (o[9] << 16), o[10] | (o[11] << 16), o[12] | (o[13] << 16), o[14] | (o[15] << 16));
    return;
  }
  for (int k = tid; k < AN_C * AN_TAPS; k += AN_THREADS) s_w[k] = a.dw_w[k];
  __syncthreads();
  // eight lanes per group of AN_DW_R consecutive positions of a row; each
  // input row's columns are loaded once and used by all the group's taps
  constexpr int R = AN_DW_R;
  const int gpr = (a.wo + R - 1) / R;  // groups per output row
  const long long ngr = (long long)a.n * a.ho * gpr;
  const long long g = (long long)blockIdx.x * AN_THREADS + tid;
  const long long grp = g >> 3;
  const int cg = (int)(g & 7);
  const bool valid = grp < ngr;
  const long long gc = valid ? grp : ngr - 1;
  const int img = (int)(gc / ((long long)a.ho * gpr)), rr = (int)(gc % ((long long)a.ho * gpr));
  const int i = rr / gpr, j0 = (rr % gpr) * R;
  float acc[R][8];
#pragma unroll
  for (int q = 0; q < R; ++q)
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[q][e] = a.dw_b[cg * 8 + e];
  const uint16_t* base = a.fin + (size_t)img * a.hi * a.wi * AN_C + cg * 8;
  for (int dy = 0; dy < AN_K; ++dy) {
    const int iy = S * i + dy - 3;
    if (iy < 0 || iy >= a.hi) continue;
    // input columns s j0 - 3 .. s (j0 + R - 1) + 3
    constexpr int NCOL = S * (R - 1) + AN_K;
    uint4 col[NCOL];
#pragma unroll
    for (int c = 0; c < NCOL; ++c) {
      const int ix = S * j0 - 3 + c;
      col[c] = (ix >= 0 && ix < a.wi)
                   ? *reinterpret_cast<const uint4*>(base + ((size_t)iy * a.wi + ix) * AN_C)
                   : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int dx = 0; dx < AN_K; ++dx) {
      float w[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) w[e] = s_w[(cg * 8 + e) * AN_TAPS + dy * AN_K + dx];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const uint4 u = col[S * q + dx];
        const uint32_t w4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          acc[q][2 * e] = __builtin_fmaf(w[2 * e], bf16_f(w4[e] & 0xffffu), acc[q][2 * e]);
          acc[q][2 * e + 1] = __builtin_fmaf(w[2 * e + 1], bf16_f(w4[e] >> 16), acc[q][2 * e + 1]);
        }
      }
    }
  }
  // normalisation over the 64 channels of each position (its eight lanes)
#pragma unroll
  for (int q = 0; q < R; ++q) {
    float sm = 0.0f;
#pragma unroll
    for (int e = 0; e < 8; ++e) sm += acc[q][e];
    sm += __shfl_xor(sm, 1, 64);
    sm += __shfl_xor(sm, 2, 64);
    sm += __shfl_xor(sm, 4, 64);
    const float mean = sm / 64.0f;
    float sq = 0.0f;
#pragma unroll
    for (int e = 0; e < 8; ++e) sq += (acc[q][e] - mean) * (acc[q][e] - mean);
    sq += __shfl_xor(sq, 1, 64);
    sq += __shfl_xor(sq, 2, 64);
    sq += __shfl_xor(sq, 4, 64);
    const float rs = 1.0f / sqrtf(sq / 64.0f + AN_LN_EPS);
    uint32_t o[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c = cg * 8 + 2 * e;
      const uint32_t lo = bf16_bits((acc[q][2 * e] - mean) * rs * a.ln_g[c] + a.ln_b[c]);
      const uint32_t hi = bf16_bits((acc[q][2 * e + 1] - mean) * rs * a.ln_g[c + 1] + a.ln_b[c + 1]);
      o[e] = lo | (hi << 16);
    }
    const int j = j0 + q;
    if (valid && j < a.wo) {
      const size_t px = ((size_t)img * a.ho + i) * a.wo + j;
      *reinterpret_cast<uint4*>(a.t + px * AN_C + cg * 8) = make_uint4(o[0], o[1], o[2], o[3]);
    }
  }
}

// --------------------------------------------------------- 1x1 MLP block

// erf by Abramowitz & Stegun, Handbook of Mathematical Functions, 7.1.26:
// erf(z) = 1 - (a1 t + a2 t^2 + a3 t^3 + a4 t^4 + a5 t^5) exp(-z^2),
// t = 1 / (1 + p z), z >= 0 (odd extension), absolute error <= 1.5e-7 --
// far below the bfloat16 rounding of the GELU output; a quarter of the
// instructions of the library erff, whose cost made the block VALU bound.
__device__ __forceinline__ float erf_as(float z) {
  const float a = fabsf(z);
  const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(0.3275911f, a, 1.0f));
  float poly = __builtin_fmaf(1.061405429f, t, -1.453152027f);
  poly = __builtin_fmaf(poly, t, 1.421413741f);
  poly = __builtin_fmaf(poly, t, -0.284496736f);
  poly = __builtin_fmaf(poly, t, 0.254829592f);
  poly *= t;
  const float e = __builtin_amdgcn_exp2f(-a * a * 1.4426950408889634f);  // exp(-z^2)
  const float r = __builtin_fmaf(-poly, e, 1.0f);
  return copysignf(r, z);
}
__device__ __forceinline__ float gelu(float v) { return 0.5f * v * (1.0f + erf_as(v * 0.70710678118654752f)); }
// round to the nearest bfloat16 (ties to even) with the hardware conversion
__device__ __forceinline__ uint16_t bf16_rne(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

template <int KIN>
__global__ __launch_bounds__(AN_THREADS, 2) void ana_mlp_kernel(AnArgs a) {
  constexpr int S1 = KIN + 8, S2 = AN_HID + 8;  // padded LDS row strides (bf16)
  constexpr int NT = AN_NT, PW = 32 * NT;       // 32-position tiles per wave step, positions per step
  __shared__ __align__(16) uint16_t s_w1[AN_HID * S1];
  __shared__ __align__(16) uint16_t s_w2[AN_C * S2];
  __shared__ float s_b1[AN_HID], s_b2[AN_C], s_hw[AN_C];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, hi = lane >> 5, col = lane & 31;
  for (int k = tid; k < AN_HID * KIN / 8; k += AN_THREADS) {
    const int r = k / (KIN / 8), c8 = k % (KIN / 8);
    *reinterpret_cast<uint4*>(&s_w1[r * S1 + c8 * 8]) = *reinterpret_cast<const uint4*>(a.w1 + (size_t)r * KIN + c8 * 8);
  }
  for (int k = tid; k < AN_C * AN_HID / 8; k += AN_THREADS) {
    const int r = k / (AN_HID / 8), c8 = k % (AN_HID / 8);
    *reinterpret_cast<uint4*>(&s_w2[r * S2 + c8 * 8]) =
        *reinterpret_cast<const uint4*>(a.w2 + (size_t)r * AN_HID + c8 * 8);
  }
  for (int k = tid; k < AN_HID; k += AN_THREADS) s_b1[k] = a.b1[k];
  for (int k = tid; k < AN_C; k += AN_THREADS) {
    s_b2[k] = a.b2[k] + (a.kid ? a.bid[k] : 0.0f);
    s_hw[k] = a.head ? a.head[k] : 0.0f;
  }
  __syncthreads();
  const int hw = a.ho * a.wo;
  const long long npx = (long long)a.n * hw;
  const float head_b = a.head ? a.head[AN_C] : 0.0f;
  for (long long g = (long long)blockIdx.x * 4 + wave; g * PW < npx; g += (long long)gridDim.x * 4) {
    const long long px0 = g * PW;
    long long pxn[NT];
    bool ok[NT];
#pragma unroll
    for (int n2 = 0; n2 < NT; ++n2) {
      pxn[n2] = px0 + 32 * n2 + col;
      ok[n2] = pxn[n2] < npx;
    }
    // B operands of the first product: the position's normalised features
    bf16x8 tb[NT][KIN / 16];
#pragma unroll
    for (int n2 = 0; n2 < NT; ++n2)
#pragma unroll
      for (int kk = 0; kk < KIN / 16; ++kk)
        tb[n2][kk] = ok[n2] ? load8(a.t + pxn[n2] * KIN + kk * 16 + hi * 8) : zero8();
    f32x16 acc2[2][NT];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int n2 = 0; n2 < NT; ++n2)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc2[mt][n2][r] = 0.0f;
#pragma unroll 1
    for (int c = 0; c < AN_HID / 32; ++c) {
      // hidden units c*32 + 8 (r / 4) + 4 hi + r % 4 of the 64 positions
      f32x16 acc1[NT];
#pragma unroll
      for (int n2 = 0; n2 < NT; ++n2)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc1[n2][r] = s_b1[c * 32 + 8 * (r >> 2) + 4 * hi + (r & 3)];
#pragma unroll
      for (int kk = 0; kk < KIN / 16; ++kk) {
        const bf16x8 aw = load8(&s_w1[(c * 32 + col) * S1 + kk * 16 + hi * 8]);
#pragma unroll
        for (int n2 = 0; n2 < NT; ++n2) acc1[n2] = mfma_bf16(aw, tb[n2][kk], acc1[n2]);
      }
      // GELU, rounded: K-step t of the second product takes accumulators
      // 8 t .. 8 t + 7, i.e. hidden units c*32 + 16 t + 8 (e / 4) + 4 hi + e % 4
      bf16x8 hb[NT][2];
#pragma unroll
      for (int n2 = 0; n2 < NT; ++n2)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int e = 0; e < 8; ++e)
            hb[n2][t][e] = (__bf16)gelu(acc1[n2][8 * t + e]);
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const uint16_t* w = &s_w2[(mt * 32 + col) * S2 + c * 32 + 16 * t + 4 * hi];
          const uint2 u0 = *reinterpret_cast<const uint2*>(w), u1 = *reinterpret_cast<const uint2*>(w + 8);
          const bf16x8 aw = __builtin_bit_cast(bf16x8, make_uint4(u0.x, u0.y, u1.x, u1.y));
#pragma unroll
          for (int n2 = 0; n2 < NT; ++n2) acc2[mt][n2] = mfma_bf16(aw, hb[n2][t], acc2[mt][n2]);
        }
    }
    // identity branch through a 1x1 convolution: the image (first block) or
    // the 2x2-average-pooled input (downsampling blocks), rounded
    if (a.kid) {
#pragma unroll 1
      for (int kk = 0; kk < a.kid / 16; ++kk) {
        bf16x8 sb[NT];
#pragma unroll
        for (int n2 = 0; n2 < NT; ++n2) {
          const long long pc = ok[n2] ? pxn[n2] : 0;
          const int img = (int)(pc / hw), r = (int)(pc % hw), i = r / a.wo, j = r % a.wo;
          if (a.c_in == 3) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int ch = kk * 16 + hi * 8 + e;
              const float v = ok[n2] && ch < 3 ? a.x[(((size_t)img * 3 + ch) * a.hi + i) * a.wi + j] : 0.0f;
              sb[n2][e] = (__bf16)v;
            }
          } else {
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = 0.0f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const size_t pin = ((size_t)img * a.hi + 2 * i + (q >> 1)) * a.wi + 2 * j + (q & 1);
              const uint4 u = ok[n2] ? *reinterpret_cast<const uint4*>(a.fin + pin * AN_C + kk * 16 + hi * 8)
                                     : make_uint4(0, 0, 0, 0);
              const uint32_t w4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                v[2 * e] += bf16_f(w4[e] & 0xffffu);
                v[2 * e + 1] += bf16_f(w4[e] >> 16);
              }
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) sb[n2][e] = (__bf16)(v[e] * 0.25f);
          }
        }
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
          const bf16x8 aw = load8(a.wid + (size_t)(mt * 32 + col) * a.kid + kk * 16 + hi * 8);
#pragma unroll
          for (int n2 = 0; n2 < NT; ++n2) acc2[mt][n2] = mfma_bf16(aw, sb[n2], acc2[mt][n2]);
        }
      }
    }
    // output: + biases (+ the input itself), rounded to bfloat16; the head
#pragma unroll
    for (int n2 = 0; n2 < NT; ++n2) {
      const long long pc = ok[n2] ? pxn[n2] : 0;
      float hsum = 0.0f;
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int qd = 0; qd < 4; ++qd) {
          const int ch0 = mt * 32 + 8 * qd + 4 * hi;
          float v[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = acc2[mt][n2][4 * qd + e] + s_b2[ch0 + e];
          if (!a.kid && ok[n2]) {
            const uint2 u = *reinterpret_cast<const uint2*>(a.fin + pc * AN_C + ch0);
            v[0] += bf16_f(u.x & 0xffffu);
            v[1] += bf16_f(u.x >> 16);
            v[2] += bf16_f(u.y & 0xffffu);
            v[3] += bf16_f(u.y >> 16);
          }
          uint32_t h[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            h[e] = bf16_rne(v[e]);
            hsum = __builtin_fmaf(s_hw[ch0 + e], bf16_f(h[e]), hsum);
          }
          if (ok[n2]) *reinterpret_cast<uint2*>(a.fout + pc * AN_C + ch0) = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
        }
      if (a.head) {
        hsum += __shfl_xor(hsum, 32, 64);
        if (hi == 0 && ok[n2]) {
          const int img = (int)(pc / hw), r = (int)(pc % hw);
          a.y[(size_t)img * a.n_lat + a.loff + r] = hsum + head_b;
        }
      }
    }
  }
}

// ------------------------------------------------------------------ host

bool an_sizes_ok(int H, int W, int n) { return n >= 1 && H >= 64 && W >= 64 && H % 64 == 0 && W % 64 == 0; }

// The blocks' parameter offsets; returns the packed parameter count.
long long an_layout(AnBlock* bl) {
  long long o = 0, q = 0;
  for (int b = 0; b < AN_BLOCKS; ++b) {
    AnBlock& B = bl[b];
    B.level = b / (1 + AN_E);
    const bool first = b % (1 + AN_E) == 0;
    B.c_in = b == 0 ? 3 : AN_C;
    B.stride = first && B.level > 0 ? 2 : 1;
    B.last = b % (1 + AN_E) == AN_E;
    B.kin = B.c_in == 3 ? 16 : AN_C;
    B.kid = first ? B.kin : 0;
    const int ci = B.c_in;
    B.o_dw_w = o; o += (long long)ci * AN_TAPS;
    B.o_dw_b = o; o += ci;
    B.o_ln_g = o; o += ci;
    B.o_ln_b = o; o += ci;
    B.o_w1 = o; o += (long long)AN_HID * ci;
    B.o_b1 = o; o += AN_HID;
    B.o_w2 = o; o += (long long)AN_C * AN_HID;
    B.o_b2 = o; o += AN_C;
    B.o_wid = o; o += first ? (long long)AN_C * ci : 0;
    B.o_bid = o; o += first ? AN_C : 0;
    B.q_w1 = q; q += (long long)AN_HID * B.kin;
    B.q_w2 = q; q += (long long)AN_C * AN_HID;
    B.q_wid = q; q += (long long)AN_C * B.kid;
  }
  return o + (long long)AN_L * (AN_C + 1);
}

long long an_q_elems(const AnBlock* bl) {
  const AnBlock& B = bl[AN_BLOCKS - 1];
  return B.q_wid + (long long)AN_C * B.kid;
}

struct AnWs {
  size_t q, f0, f1, t, total;  // byte offsets
};

AnWs an_ws(int H, int W, int n, const AnBlock* bl) {
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  AnWs w;
  const size_t feat = (size_t)n * H * W * AN_C * sizeof(uint16_t);
  w.q = 0;
  w.f0 = up(an_q_elems(bl) * sizeof(uint16_t));
  w.f1 = w.f0 + up(feat);
  w.t = w.f1 + up(feat);
  w.total = w.t + up(feat);
  return w;
}

}  // namespace
}  // namespace cc

using namespace cc;

extern "C" {

int64_t coolchic_analysis_param_count(void) {
  AnBlock bl[AN_BLOCKS];
  return an_layout(bl);
}

size_t coolchic_analysis_workspace_bytes(int32_t H, int32_t W, int32_t n) {
  if (!an_sizes_ok(H, W, n)) return 0;
  AnBlock bl[AN_BLOCKS];
  an_layout(bl);
  return an_ws(H, W, n, bl).total;
}

int coolchic_analysis_forward(int32_t H, int32_t W, int32_t n, const float* x, const float* theta, float* y,
                              void* ws, size_t ws_bytes, void* stream) {
  if (!an_sizes_ok(H, W, n) || !x || !theta || !y || !ws) return CC_EINVAL;
  AnBlock bl[AN_BLOCKS];
  const long long n_par = an_layout(bl);
  const AnWs L = an_ws(H, W, n, bl);
  if (ws_bytes < L.total) return CC_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  uint16_t* q = (uint16_t*)(base + L.q);
  uint16_t* feat[2] = {(uint16_t*)(base + L.f0), (uint16_t*)(base + L.f1)};
  uint16_t* tbuf = (uint16_t*)(base + L.t);
  (void)hipGetLastError();
  {
    AnPrepArgs pa;
    pa.theta = theta;
    pa.q = q;
    pa.n_blocks = AN_BLOCKS;
    for (int b = 0; b < AN_BLOCKS; ++b) {
      pa.c_in[b] = bl[b].c_in; pa.kin[b] = bl[b].kin; pa.kid[b] = bl[b].kid;
      pa.o_w1[b] = bl[b].o_w1; pa.o_w2[b] = bl[b].o_w2; pa.o_wid[b] = bl[b].o_wid;
      pa.q_w1[b] = bl[b].q_w1; pa.q_w2[b] = bl[b].q_w2; pa.q_wid[b] = bl[b].q_wid;
      pa.n_per[b] = (long long)AN_HID * bl[b].kin + (long long)AN_C * AN_HID + (long long)AN_C * bl[b].kid;
    }
    const long long nq = an_q_elems(bl);
    void* argv[] = {&pa};
    if (hipLaunchKernel((const void*)ana_prep_kernel, dim3((unsigned)((nq + AN_THREADS - 1) / AN_THREADS)),
                        dim3(AN_THREADS), argv, 0, st) != hipSuccess)
      return CC_EHIP;
  }
  int n_lat = 0, loff[AN_L];
  for (int l = 0; l < AN_L; ++l) {
    loff[l] = n_lat;
    n_lat += (H >> l) * (W >> l);
  }
  const long long head0 = n_par - (long long)AN_L * (AN_C + 1);
  int hin = H, win = W;
  for (int b = 0; b < AN_BLOCKS; ++b) {
    const AnBlock& B = bl[b];
    AnArgs a;
    a.n = n; a.hi = hin; a.wi = win;
    a.ho = hin / B.stride; a.wo = win / B.stride;
    a.c_in = B.c_in; a.stride = B.stride; a.kin = B.kin; a.kid = B.kid;
    a.x = x;
    a.fin = b == 0 ? nullptr : feat[(b + 1) & 1];
    a.t = tbuf;
    a.fout = feat[b & 1];
    a.dw_w = theta + B.o_dw_w; a.dw_b = theta + B.o_dw_b; a.ln_g = theta + B.o_ln_g; a.ln_b = theta + B.o_ln_b;
    a.b1 = theta + B.o_b1; a.b2 = theta + B.o_b2; a.bid = B.kid ? theta + B.o_bid : nullptr;
    a.w1 = q + B.q_w1; a.w2 = q + B.q_w2; a.wid = B.kid ? q + B.q_wid : nullptr;
    a.head = B.last ? theta + head0 + (long long)B.level * (AN_C + 1) : nullptr;
    a.y = y; a.n_lat = n_lat; a.loff = loff[B.level];
    const long long npx = (long long)n * a.ho * a.wo;
    void* argv[] = {&a};
    const long long dw_threads = B.c_in == 3 ? npx : (long long)n * a.ho * ((a.wo + AN_DW_R - 1) / AN_DW_R) * 8;
    if (hipLaunchKernel(B.stride == 2 ? (const void*)ana_dw_kernel<2> : (const void*)ana_dw_kernel<1>, dim3((unsigned)((dw_threads + AN_THREADS - 1) / AN_THREADS)),
                        dim3(AN_THREADS), argv, 0, st) != hipSuccess)
      return CC_EHIP;
    const long long groups = (npx + 32 * AN_NT - 1) / (32 * AN_NT);
    const unsigned grid = (unsigned)std::min<long long>((groups + 3) / 4, AN_MAX_GRID);
    const void* mlp = B.kin == 16 ? (const void*)ana_mlp_kernel<16> : (const void*)ana_mlp_kernel<AN_C>;
    if (hipLaunchKernel(mlp, dim3(grid), dim3(AN_THREADS), argv, 0, st) != hipSuccess) return CC_EHIP;
    hin = a.ho;
    win = a.wo;
  }
  return hipGetLastError() == hipSuccess ? CC_OK : CC_EHIP;
}

}  // extern "C"

// Non-overfitted analysis transform on gfx950 (Section IV-B, Eq. (3)):
// y = f_alpha(x), the latent grids of Cool-chic in one forward pass.
//
// 21 ConvNeXt-style blocks (three per latent level, the first of levels
// 1..6 with stride 2).  A block with 64 input channels is one launch,
// ana_block_kernel: per wave and 32 output positions, the depth-wise 7x7
// convolution and the layer normalisation over channels in FP32, the
// normalised features T (bfloat16) handed to the MLP through LDS, then the
// block's 1x1 convolutions on the bfloat16 matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation), GELU between them, the
// identity branch, the bfloat16 block output and, for a level's last block,
// its latent head.  Blocks of at most AN_TEAM_MAX_POSITIONS positions per
// image (the coarse levels) run as ana_block_team_kernel instead, a whole
// work-group on one 32-position tile.  The first block (3 image channels)
// runs as ana_dw3_kernel (depth-wise conv + norm, T with 16 channels in
// global memory) and ana_mlp16_kernel.
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
#include <type_traits>

#include "coolchic.h"
#include "common.hpp"
#include "bf16.hpp"

namespace cc {
namespace {

constexpr int AN_C = 64, AN_HID = 256, AN_K = 7, AN_TAPS = AN_K * AN_K, AN_L = 7, AN_E = 2;
constexpr int AN_BLOCKS = AN_L * (1 + AN_E);
constexpr float AN_LN_EPS = 1e-6f;
constexpr int AN_THREADS = 256;
constexpr int AN_MAX_GRID = 1024;  // work-groups of the first block's MLP launch at most
constexpr int AN_BW = 8, AN_BT = 64 * AN_BW;  // waves, threads per work-group of the fused block kernel
constexpr int AN_BLOCK_GRID = 256;  // fused block kernels: one work-group per CU (their LDS holds one)
constexpr int AN_TEAM_MAX_POSITIONS = 6144;  // blocks of at most this many output positions per image: team kernel

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

// The first block (3 image channels): one thread per position, FP32 planar
// image, T padded to 16 channels (the K step of the matrix cores).
__global__ __launch_bounds__(AN_THREADS) void ana_dw3_kernel(AnArgs a) {
  const long long npx = (long long)a.n * a.ho * a.wo;
  // work-group b runs on XCD b mod 8: with a grid that is a multiple of 8,
  // XCD x takes the x-th eighth of the positions, so that the rows the 7x7
  // window reads again are fetched through one L2
  const unsigned G = gridDim.x, b = G % 8 == 0 ? (blockIdx.x % 8) * (G / 8) + blockIdx.x / 8 : blockIdx.x;
  const long long px = (long long)b * AN_THREADS + threadIdx.x;
  if (px >= npx) return;
  const int img = (int)(px / ((long long)a.ho * a.wo)), r = (int)(px % ((long long)a.ho * a.wo));
  const int i = r / a.wo, j = r % a.wo;
  float acc[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float s = a.dw_b[c];
    const float* xc = a.x + ((size_t)img * 3 + c) * a.hi * a.wi;
    for (int dy = 0; dy < AN_K; ++dy) {
      const int iy = i + dy - 3;
      if (iy < 0 || iy >= a.hi) continue;
      for (int dx = 0; dx < AN_K; ++dx) {
        const int ix = j + dx - 3;
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
}

// --------------------------------------------------------- 1x1 MLP block

// GELU(v) = v Phi(v) = max(v, 0) - |v| Phi(-|v|), with
// Phi(-|v|) = erfc(|v| / sqrt 2) / 2 by Abramowitz & Stegun, Handbook of
// Mathematical Functions, 7.1.26: erfc(z) = (a1 t + a2 t^2 + a3 t^3 + a4 t^4
// + a5 t^5) exp(-z^2), t = 1 / (1 + p z), z >= 0, absolute error <= 1.5e-7
// -- far below the bfloat16 rounding of the GELU output.  The 1/2 and the
// 1/sqrt 2 are folded into the constants: 13 instructions (two of them
// transcendental) against about 60 for the library erff, whose cost made
// the block VALU bound.
__device__ __forceinline__ float gelu(float v) {
  const float u = fabsf(v);
  const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(0.23164189f, u, 1.0f));  // p / sqrt 2
  float q = __builtin_fmaf(0.5307027145f, t, -0.7265760135f);                     // a5 / 2, a4 / 2
  q = __builtin_fmaf(q, t, 0.7107068705f);                                        // a3 / 2
  q = __builtin_fmaf(q, t, -0.142248368f);                                        // a2 / 2
  q = __builtin_fmaf(q, t, 0.127414796f);                                         // a1 / 2
  q *= t;
  const float e = __builtin_amdgcn_exp2f(v * v * -0.7213475204f);  // exp(-v^2 / 2)
  return __builtin_fmaf(-u, q * e, fmaxf(v, 0.0f));
}
// round to the nearest bfloat16 (ties to even) with the hardware conversion
__device__ __forceinline__ uint16_t bf16_rne(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// LDS copies of a block's 1x1 weights (rows padded against bank conflicts),
// biases and head weights, by nthr threads.
template <int KIN>
struct AnMlpLds {
  static constexpr int S1 = KIN + 8, S2 = AN_HID + 8;
  __align__(16) uint16_t w1[AN_HID * S1];
  __align__(16) uint16_t w2[AN_C * S2];
  float b1[AN_HID], b2[AN_C], hw[AN_C];
};

// Every thread's elements are read into registers first and written to LDS
// afterwards: a loop of load-store pairs waits for each load in turn.
template <int KIN, int NTHR>
__device__ __forceinline__ void an_stage_mlp(const AnArgs& a, AnMlpLds<KIN>& s, int tid) {
  constexpr int S1 = AnMlpLds<KIN>::S1, S2 = AnMlpLds<KIN>::S2;
  constexpr int N1 = AN_HID * KIN / 8, N2 = AN_C * AN_HID / 8;  // 16-byte units
  constexpr int R1 = (N1 + NTHR - 1) / NTHR, R2 = (N2 + NTHR - 1) / NTHR;
  static_assert(NTHR >= AN_HID, "one bias per thread");
  uint4 v1[R1], v2[R2];  // (a thread past the end re-reads the last unit and stores nothing)
#pragma unroll
  for (int q = 0; q < R1; ++q) v1[q] = *reinterpret_cast<const uint4*>(a.w1 + (size_t)min(tid + q * NTHR, N1 - 1) * 8);
#pragma unroll
  for (int q = 0; q < R2; ++q) v2[q] = *reinterpret_cast<const uint4*>(a.w2 + (size_t)min(tid + q * NTHR, N2 - 1) * 8);
  const float b1 = tid < AN_HID ? a.b1[tid] : 0.0f;
  const float b2 = tid < AN_C ? a.b2[tid] + (a.kid ? a.bid[tid] : 0.0f) : 0.0f;
  const float hw = tid < AN_C && a.head ? a.head[tid] : 0.0f;
#pragma unroll
  for (int q = 0; q < R1; ++q) {
    const int k = tid + q * NTHR;
    if (N1 % NTHR == 0 || k < N1) *reinterpret_cast<uint4*>(&s.w1[(k / (KIN / 8)) * S1 + (k % (KIN / 8)) * 8]) = v1[q];
  }
#pragma unroll
  for (int q = 0; q < R2; ++q) {
    const int k = tid + q * NTHR;
    if (N2 % NTHR == 0 || k < N2) *reinterpret_cast<uint4*>(&s.w2[(k / (AN_HID / 8)) * S2 + (k % (AN_HID / 8)) * 8]) = v2[q];
  }
  if (tid < AN_HID) s.b1[tid] = b1;
  if (tid < AN_C) {
    s.b2[tid] = b2;
    s.hw[tid] = hw;
  }
}

// Output position of a lane in a block's level: image, row, column (a
// position beyond the last one has ok = false and the coordinates of the
// first).  Positions are counted in 32 bits (the host bounds n h w).
struct AnPos {
  int img, i, j;
  bool ok;
};
__device__ __forceinline__ AnPos an_pos(const AnArgs& a, int p) {
  const int hw = a.ho * a.wo;
  AnPos q;
  q.ok = p < a.n * hw;
  const int pc = q.ok ? p : 0;
  q.img = pc / hw;
  const int r = pc - q.img * hw;
  q.i = r / a.wo;
  q.j = r - q.i * a.wo;
  return q;
}

// One hidden chunk c (32 units) of a wave's 32 positions: the first product
// from tb, GELU, rounded, and the second product added to acc2.
template <int KIN>
__device__ __forceinline__ void an_mlp_chunk(const AnMlpLds<KIN>& s, const bf16x8 (&tb)[KIN / 16], int c, int lane,
                                             f32x16 (&acc2)[2]) {
  constexpr int S1 = AnMlpLds<KIN>::S1, S2 = AnMlpLds<KIN>::S2;
  const int hi = lane >> 5, col = lane & 31;
  // hidden units c*32 + 8 (r / 4) + 4 hi + r % 4 of the 32 positions
  f32x16 acc1;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc1[r] = s.b1[c * 32 + 8 * (r >> 2) + 4 * hi + (r & 3)];
#pragma unroll
  for (int kk = 0; kk < KIN / 16; ++kk) acc1 = mfma_bf16(load8(&s.w1[(c * 32 + col) * S1 + kk * 16 + hi * 8]), tb[kk], acc1);
  // GELU, rounded: K-step t of the second product takes accumulators
  // 8 t .. 8 t + 7, i.e. hidden units c*32 + 16 t + 8 (e / 4) + 4 hi + e % 4
  bf16x8 hb[2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 8; ++e) hb[t][e] = (__bf16)gelu(acc1[8 * t + e]);
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const uint16_t* w = &s.w2[(mt * 32 + col) * S2 + c * 32 + 16 * t + 4 * hi];
      const uint2 u0 = *reinterpret_cast<const uint2*>(w), u1 = *reinterpret_cast<const uint2*>(w + 8);
      acc2[mt] = mfma_bf16(__builtin_bit_cast(bf16x8, make_uint4(u0.x, u0.y, u1.x, u1.y)), hb[t], acc2[mt]);
    }
}

// identity branch through a 1x1 convolution, added to acc2: the image (first
// block) or the 2x2-average-pooled input (downsampling blocks), rounded
__device__ __forceinline__ void an_identity(const AnArgs& a, const AnPos& pos, int lane, f32x16 (&acc2)[2]) {
  const int hi = lane >> 5, col = lane & 31;
  const bool ok = pos.ok;
  const int img = pos.img, i = pos.i, j = pos.j;
#pragma unroll 1
  for (int kk = 0; kk < a.kid / 16; ++kk) {
    bf16x8 sb;
    if (a.c_in == 3) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int ch = kk * 16 + hi * 8 + e;
        const float v = ok && ch < 3 ? a.x[(((size_t)img * 3 + ch) * a.hi + i) * a.wi + j] : 0.0f;
        sb[e] = (__bf16)v;
      }
    } else {
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = 0.0f;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const size_t pin = ((size_t)img * a.hi + 2 * i + (q >> 1)) * a.wi + 2 * j + (q & 1);
        const uint4 u = ok ? *reinterpret_cast<const uint4*>(a.fin + pin * AN_C + kk * 16 + hi * 8) : make_uint4(0, 0, 0, 0);
        const uint32_t w4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          v[2 * e] += bf16_f(w4[e] & 0xffffu);
          v[2 * e + 1] += bf16_f(w4[e] >> 16);
        }
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) sb[e] = (__bf16)(v[e] * 0.25f);
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
      acc2[mt] = mfma_bf16(load8(a.wid + (size_t)(mt * 32 + col) * a.kid + kk * 16 + hi * 8), sb, acc2[mt]);
  }
}

// One wave, 32 positions: both 1x1 layers, GELU, the identity branch, the
// bfloat16 block output and the head.  tb holds the B operands of the first
// product (the lane's position pos, column lane % 32 of the products,
// channels kk * 16 + 8 (lane / 32) .. + 7 of k-step kk).
template <int KIN>
__device__ __forceinline__ void an_mlp_tile(const AnArgs& a, const AnMlpLds<KIN>& s, const bf16x8 (&tb)[KIN / 16],
                                            const AnPos& pos, int lane) {
  const int hi = lane >> 5;
  const bool ok = pos.ok;
  f32x16 acc2[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc2[mt][r] = 0.0f;
#pragma unroll 1
  for (int c = 0; c < AN_HID / 32; ++c) an_mlp_chunk<KIN>(s, tb, c, lane, acc2);
  const int img = pos.img, i = pos.i, j = pos.j, rr = i * a.wo + j;
  const size_t pc = ((size_t)img * a.ho + i) * a.wo + j;
  if (a.kid) an_identity(a, pos, lane, acc2);
  // output: + biases (+ the input itself), rounded to bfloat16; the head
  float hsum = 0.0f;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int qd = 0; qd < 4; ++qd) {
      const int ch0 = mt * 32 + 8 * qd + 4 * hi;
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = acc2[mt][4 * qd + e] + s.b2[ch0 + e];
      if (!a.kid && ok) {
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
        hsum = __builtin_fmaf(s.hw[ch0 + e], bf16_f(h[e]), hsum);
      }
      if (ok) *reinterpret_cast<uint2*>(a.fout + pc * AN_C + ch0) = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
    }
  if (a.head) {
    hsum += __shfl_xor(hsum, 32, 64);
    if (hi == 0 && ok) a.y[(size_t)img * a.n_lat + a.loff + rr] = hsum + a.head[AN_C];
  }
}

// The first block's MLP: T (16 channels, the image's 3 and zeros) from the
// depth-wise kernel.
__global__ __launch_bounds__(AN_THREADS, 2) void ana_mlp16_kernel(AnArgs a) {
  __shared__ AnMlpLds<16> s;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, hi = lane >> 5, col = lane & 31;
  an_stage_mlp<16, AN_THREADS>(a, s, tid);
  __syncthreads();
  const int npx = a.n * a.ho * a.wo;
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  for (int g = blockIdx.x * 4 + wave_u; g * 32 < npx; g += gridDim.x * 4) {
    const int px = g * 32 + col;
    const AnPos pos = an_pos(a, px);
    bf16x8 tb[1];
    tb[0] = pos.ok ? load8(a.t + (size_t)px * 16 + hi * 8) : zero8();
    an_mlp_tile<16>(a, s, tb, pos, lane);
  }
}

// Blocks with 64 input channels, one launch each: per wave and 32 output
// positions, the depth-wise 7x7 convolution (stride S) and the layer norm
// in FP32, the normalised features through the wave's LDS slot (bfloat16)
// into the MLP's operand layout, then the MLP (an_mlp_tile).  Depth-wise
// lanes: eight lanes per group of four positions, eight channels each; with
// ROWSEG (output rows a multiple of 32 wide) a tile is one row segment and a
// group's positions are consecutive, so each input row is loaded once per
// group as S * 3 + 7 columns and converted to FP32 once; otherwise (the small
// coarse levels) each position loads its own 7 x 7 window.
template <int S, bool ROWSEG>
__global__ __launch_bounds__(AN_BT) void ana_block_kernel(AnArgs a) {
  constexpr int ST = AN_C + 8;  // LDS row stride of the normalised features (bf16)
  __shared__ AnMlpLds<AN_C> s;
  __shared__ __align__(16) float s_dw[AN_TAPS * AN_C];  // [tap][channel]
  __shared__ __align__(16) uint16_t s_t[AN_BW * 32 * ST];
  __shared__ __align__(16) float s_dwb[AN_C], s_lg[AN_C], s_lb[AN_C];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, hi = lane >> 5, col = lane & 31;
  {
    // depth-wise weights transposed to [tap][channel] (loads first, as in an_stage_mlp)
    constexpr int RD = (AN_TAPS * AN_C + AN_BT - 1) / AN_BT;
    float v[RD];
#pragma unroll
    for (int q = 0; q < RD; ++q) {
      const int k = min(tid + q * AN_BT, AN_TAPS * AN_C - 1);
      v[q] = a.dw_w[(k % AN_C) * AN_TAPS + k / AN_C];
    }
    float vb = 0.0f, vg = 0.0f, vl = 0.0f;
    if (tid < AN_C) {
      vb = a.dw_b[tid];
      vg = a.ln_g[tid];
      vl = a.ln_b[tid];
    }
    an_stage_mlp<AN_C, AN_BT>(a, s, tid);
#pragma unroll
    for (int q = 0; q < RD; ++q) {
      const int k = tid + q * AN_BT;
      if (k < AN_TAPS * AN_C) s_dw[k] = v[q];
    }
    if (tid < AN_C) {
      s_dwb[tid] = vb;
      s_lg[tid] = vg;
      s_lb[tid] = vl;
    }
  }
  __syncthreads();
  const int cg = lane & 7, pg = lane >> 3;
  const int hw = a.ho * a.wo, npx = a.n * hw;
  uint16_t* st = s_t + wave * 32 * ST;
  const uint16_t* fin = a.fin + cg * 8;
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  // Tiles are walked in row-major order.  Work-groups are dispatched to the
  // eight XCDs in turn (work-group b on XCD b mod 8), each XCD with its own
  // L2: with a grid that is a multiple of 8, XCD x takes the x-th eighth of
  // the tiles, so that the rows above and below a tile, which the 7x7 window
  // reads again, are fetched by work-groups sharing its L2.
  const int tiles = (npx + 31) / 32, G = gridDim.x;
  int g0, gstep, gend;
  if (G % 8 == 0) {
    const int tx = (tiles + 7) / 8, x = blockIdx.x % 8;
    g0 = x * tx + (blockIdx.x / 8) * AN_BW + wave_u;
    gstep = (G / 8) * AN_BW;
    gend = min(tiles, (x + 1) * tx);
  } else {
    g0 = blockIdx.x * AN_BW + wave_u;
    gstep = G * AN_BW;
    gend = tiles;
  }
  for (int g = g0; g < gend; g += gstep) {
    const int px0 = g * 32;
    // the lane's position for the products; with ROWSEG a tile is one row
    // segment, its image and row the same for the whole wave
    AnPos pos;
    int jw = 0;
    if constexpr (ROWSEG) {
      pos.img = px0 / hw;
      const int r = px0 - pos.img * hw;
      pos.i = r / a.wo;
      jw = r - pos.i * a.wo;
      pos.j = jw + col;
      pos.ok = true;  // npx is a multiple of 32
    } else {
      pos = an_pos(a, px0 + col);
    }
    float acc[4][8];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[q][e] = s_dwb[cg * 8 + e];
    if constexpr (ROWSEG) {
      const int img = pos.img, i = pos.i, j0 = jw + 4 * pg;
      const uint16_t* base = fin + (size_t)img * a.hi * a.wi * AN_C;
      constexpr int NCOL = S * 3 + AN_K;
      // input row S i + dy - 3, columns S j0 - 3 .. S j0 - 3 + NCOL - 1
      // rows outside the image add nothing and are skipped (the row is the
      // same for the whole wave); columns of a group away from the image's
      // left and right borders need no checks
      const bool inside = S * j0 - 3 >= 0 && S * j0 - 3 + NCOL <= a.wi;
      auto rows = [&](auto checked) {
#pragma unroll 1
        for (int dy = 0; dy < AN_K; ++dy) {
          const int iy = S * i + dy - 3;
          if (iy < 0 || iy >= a.hi) continue;
          const uint16_t* rowp = base + (size_t)iy * a.wi * AN_C;
          uint4 u[NCOL];
#pragma unroll
          for (int c = 0; c < NCOL; ++c) {
            const int ix = S * j0 - 3 + c;
            if constexpr (decltype(checked)::value)
              u[c] = (ix >= 0 && ix < a.wi) ? *reinterpret_cast<const uint4*>(rowp + (size_t)ix * AN_C) : make_uint4(0, 0, 0, 0);
            else
              u[c] = *reinterpret_cast<const uint4*>(rowp + (size_t)(S * j0 - 3) * AN_C + c * AN_C);
          }
          // each column converted to FP32 once (stride 1) or where it is used
          // (stride 2: 13 columns, whose FP32 copies would not fit the registers)
          if constexpr (S == 1) {
            float f[NCOL][8];
#pragma unroll
            for (int c = 0; c < NCOL; ++c) {
              const uint32_t w4[4] = {u[c].x, u[c].y, u[c].z, u[c].w};
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                f[c][2 * e] = bf16_f(w4[e] & 0xffffu);
                f[c][2 * e + 1] = bf16_f(w4[e] >> 16);
              }
            }
#pragma unroll
            for (int dx = 0; dx < AN_K; ++dx) {
              const float4 w0 = *reinterpret_cast<const float4*>(&s_dw[(dy * AN_K + dx) * AN_C + cg * 8]);
              const float4 w1 = *reinterpret_cast<const float4*>(&s_dw[(dy * AN_K + dx) * AN_C + cg * 8 + 4]);
              const float w[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
#pragma unroll
              for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int e = 0; e < 8; ++e) acc[q][e] = __builtin_fmaf(w[e], f[q + dx][e], acc[q][e]);
            }
          } else {
#pragma unroll
            for (int dx = 0; dx < AN_K; ++dx) {
              const float4 w0 = *reinterpret_cast<const float4*>(&s_dw[(dy * AN_K + dx) * AN_C + cg * 8]);
              const float4 w1 = *reinterpret_cast<const float4*>(&s_dw[(dy * AN_K + dx) * AN_C + cg * 8 + 4]);
              const float w[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const uint4 x = u[S * q + dx];
                const uint32_t w4[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                  acc[q][2 * e] = __builtin_fmaf(w[2 * e], bf16_f(w4[e] & 0xffffu), acc[q][2 * e]);
                  acc[q][2 * e + 1] = __builtin_fmaf(w[2 * e + 1], bf16_f(w4[e] >> 16), acc[q][2 * e + 1]);
                }
              }
            }
          }
        }
      };
      if (inside)
        rows(std::false_type{});
      else
        rows(std::true_type{});
    } else {
      // per input row, the seven columns of two positions in flight
      int img[4], pi[4], pj[4];
      bool pok[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const AnPos pq = an_pos(a, px0 + 4 * pg + q);  // features beyond the last position are never used
        pok[q] = pq.ok;
        img[q] = pq.img;
        pi[q] = pq.i;
        pj[q] = pq.j;
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll 1
        for (int dy = 0; dy < AN_K; ++dy) {
          uint4 u[2][AN_K];
#pragma unroll
          for (int q2 = 0; q2 < 2; ++q2) {
            const int q = 2 * h + q2;
            const int iy = S * pi[q] + dy - 3;
            const bool row_ok = pok[q] && iy >= 0 && iy < a.hi;
            const uint16_t* base = fin + ((size_t)img[q] * a.hi + (row_ok ? iy : 0)) * a.wi * AN_C;
#pragma unroll
            for (int dx = 0; dx < AN_K; ++dx) {
              const int ix = S * pj[q] + dx - 3;
              u[q2][dx] = (row_ok && ix >= 0 && ix < a.wi) ? *reinterpret_cast<const uint4*>(base + (size_t)ix * AN_C)
                                                           : make_uint4(0, 0, 0, 0);
            }
          }
#pragma unroll
          for (int dx = 0; dx < AN_K; ++dx) {
            const float4 w0 = *reinterpret_cast<const float4*>(&s_dw[(dy * AN_K + dx) * AN_C + cg * 8]);
            const float4 w1 = *reinterpret_cast<const float4*>(&s_dw[(dy * AN_K + dx) * AN_C + cg * 8 + 4]);
            const float w[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
#pragma unroll
            for (int q2 = 0; q2 < 2; ++q2) {
              const uint32_t w4[4] = {u[q2][dx].x, u[q2][dx].y, u[q2][dx].z, u[q2][dx].w};
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                acc[2 * h + q2][2 * e] = __builtin_fmaf(w[2 * e], bf16_f(w4[e] & 0xffffu), acc[2 * h + q2][2 * e]);
                acc[2 * h + q2][2 * e + 1] = __builtin_fmaf(w[2 * e + 1], bf16_f(w4[e] >> 16), acc[2 * h + q2][2 * e + 1]);
              }
            }
          }
        }
      }
    }
    // normalisation over the 64 channels of each position (its eight lanes),
    // rounded into the wave's LDS slot
#pragma unroll
    for (int q = 0; q < 4; ++q) {
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
        const uint32_t lo = bf16_bits((acc[q][2 * e] - mean) * rs * s_lg[c] + s_lb[c]);
        const uint32_t hb = bf16_bits((acc[q][2 * e + 1] - mean) * rs * s_lg[c + 1] + s_lb[c + 1]);
        o[e] = lo | (hb << 16);
      }
      *reinterpret_cast<uint4*>(&st[(4 * pg + q) * ST + cg * 8]) = make_uint4(o[0], o[1], o[2], o[3]);
    }
    // the slot is the wave's own: order its writes before the reads of
    // other lanes of the same wave
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    bf16x8 tb[AN_C / 16];
#pragma unroll
    for (int kk = 0; kk < AN_C / 16; ++kk) tb[kk] = pos.ok ? load8(&st[col * ST + kk * 16 + hi * 8]) : zero8();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    an_mlp_tile<AN_C>(a, s, tb, pos, lane);
  }
}

// Blocks of the coarse levels (a few thousand positions per image or fewer),
// where a wave's serial chain -- its rows of loads, eight hidden chunks, the
// epilogue -- sets the time of ana_block_kernel: the whole work-group takes
// one 32-position tile at a time.  Depth-wise: wave w computes positions
// 4w .. 4w + 3 of the tile, eight lanes per position (eight channels each)
// and two lanes per channel group splitting the seven rows (0-3, 4-6), all
// of a lane's loads issued at once.  MLP: wave w computes hidden chunk w (32
// units) and writes its share of the second product to LDS (wave 0 adds the
// identity branch); wave w then sums the eight shares of output channels
// 32 (w / 4) + 8 (w % 4) .. + 7 of the 32 positions for the epilogue.  The
// depth-wise sums run in another order than in ana_block_kernel, so a block
// is run by one kernel or the other according to its size per image only.
template <int S>
__global__ __launch_bounds__(AN_BT) void ana_block_team_kernel(AnArgs a) {
  constexpr int ST = AN_C + 8, SP = 33;  // LDS row strides: features (bf16), second-product shares (floats)
  static_assert(AN_BW == 8, "one hidden chunk per wave");
  __shared__ AnMlpLds<AN_C> s;
  __shared__ __align__(16) float s_dw[AN_TAPS * AN_C];  // [tap][channel]
  __shared__ __align__(16) uint16_t s_t[32 * ST];
  __shared__ float s_part[AN_BW * 64 * SP];             // [wave][lane][32 accumulators]
  __shared__ float s_head[AN_BW * 32];
  __shared__ float s_dwb[AN_C], s_lg[AN_C], s_lb[AN_C];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, hi = lane >> 5, col = lane & 31;
  {
    constexpr int RD = (AN_TAPS * AN_C + AN_BT - 1) / AN_BT;
    float v[RD];
#pragma unroll
    for (int q = 0; q < RD; ++q) {
      const int k = min(tid + q * AN_BT, AN_TAPS * AN_C - 1);
      v[q] = a.dw_w[(k % AN_C) * AN_TAPS + k / AN_C];
    }
    float vb = 0.0f, vg = 0.0f, vl = 0.0f;
    if (tid < AN_C) {
      vb = a.dw_b[tid];
      vg = a.ln_g[tid];
      vl = a.ln_b[tid];
    }
    an_stage_mlp<AN_C, AN_BT>(a, s, tid);
#pragma unroll
    for (int q = 0; q < RD; ++q) {
      const int k = tid + q * AN_BT;
      if (k < AN_TAPS * AN_C) s_dw[k] = v[q];
    }
    if (tid < AN_C) {
      s_dwb[tid] = vb;
      s_lg[tid] = vg;
      s_lb[tid] = vl;
    }
  }
  __syncthreads();
  const int npx = a.n * a.ho * a.wo, tiles = (npx + 31) / 32;
  const int cg = lane & 7, p4 = (lane >> 3) & 3, half = lane >> 5;
  const int mt_e = wave >> 2, qd_e = wave & 3;  // this wave's output channels in the epilogue
  for (int g = blockIdx.x; g < tiles; g += gridDim.x) {  // uniform over the work-group
    const int px0 = g * 32;
    // ---- depth-wise 7x7 and layer norm of position 4 wave + p4
    {
      const AnPos q = an_pos(a, px0 + 4 * wave + p4);
      const uint16_t* base = a.fin + (size_t)q.img * a.hi * a.wi * AN_C + cg * 8;
      uint4 u[4][AN_K];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int dy = 4 * half + r, iy = S * q.i + dy - 3;
        const bool row_ok = q.ok && dy < AN_K && iy >= 0 && iy < a.hi;
#pragma unroll
        for (int dx = 0; dx < AN_K; ++dx) {
          const int ix = S * q.j + dx - 3;
          u[r][dx] = (row_ok && ix >= 0 && ix < a.wi) ? *reinterpret_cast<const uint4*>(base + ((size_t)iy * a.wi + ix) * AN_C)
                                                      : make_uint4(0, 0, 0, 0);
        }
      }
      float acc[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[e] = 0.0f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int dy = min(4 * half + r, AN_K - 1);  // row 7 of the second half: zeros, any weights
#pragma unroll
        for (int dx = 0; dx < AN_K; ++dx) {
          const float4 w0 = *reinterpret_cast<const float4*>(&s_dw[(dy * AN_K + dx) * AN_C + cg * 8]);
          const float4 w1 = *reinterpret_cast<const float4*>(&s_dw[(dy * AN_K + dx) * AN_C + cg * 8 + 4]);
          const float w[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
          const uint32_t w4[4] = {u[r][dx].x, u[r][dx].y, u[r][dx].z, u[r][dx].w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            acc[2 * e] = __builtin_fmaf(w[2 * e], bf16_f(w4[e] & 0xffffu), acc[2 * e]);
            acc[2 * e + 1] = __builtin_fmaf(w[2 * e + 1], bf16_f(w4[e] >> 16), acc[2 * e + 1]);
          }
        }
      }
      // rows 0-3 + rows 4-6, then the bias
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float other = __shfl_xor(acc[e], 32, 64);
        acc[e] = (half == 0 ? acc[e] + other : other + acc[e]) + s_dwb[cg * 8 + e];
      }
      float sm = 0.0f;
#pragma unroll
      for (int e = 0; e < 8; ++e) sm += acc[e];
      sm += __shfl_xor(sm, 1, 64);
      sm += __shfl_xor(sm, 2, 64);
      sm += __shfl_xor(sm, 4, 64);
      const float mean = sm / 64.0f;
      float sq = 0.0f;
#pragma unroll
      for (int e = 0; e < 8; ++e) sq += (acc[e] - mean) * (acc[e] - mean);
      sq += __shfl_xor(sq, 1, 64);
      sq += __shfl_xor(sq, 2, 64);
      sq += __shfl_xor(sq, 4, 64);
      const float rs = 1.0f / sqrtf(sq / 64.0f + AN_LN_EPS);
      if (half == 0) {
        uint32_t o[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int c = cg * 8 + 2 * e;
          const uint32_t lo = bf16_bits((acc[2 * e] - mean) * rs * s_lg[c] + s_lb[c]);
          const uint32_t hb = bf16_bits((acc[2 * e + 1] - mean) * rs * s_lg[c + 1] + s_lb[c + 1]);
          o[e] = lo | (hb << 16);
        }
        *reinterpret_cast<uint4*>(&s_t[(4 * wave + p4) * ST + cg * 8]) = make_uint4(o[0], o[1], o[2], o[3]);
      }
    }
    __syncthreads();
    // ---- hidden chunk `wave` of the tile's 32 positions
    const AnPos pos = an_pos(a, px0 + col);
    {
      bf16x8 tb[AN_C / 16];
#pragma unroll
      for (int kk = 0; kk < AN_C / 16; ++kk) tb[kk] = pos.ok ? load8(&s_t[col * ST + kk * 16 + hi * 8]) : zero8();
      f32x16 acc2[2];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc2[mt][r] = 0.0f;
      an_mlp_chunk<AN_C>(s, tb, wave, lane, acc2);
      if (wave == 0 && a.kid) an_identity(a, pos, lane, acc2);
      float* dst = &s_part[(wave * 64 + lane) * SP];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 16; ++r) dst[mt * 16 + r] = acc2[mt][r];
    }
    __syncthreads();
    // ---- epilogue: output channels ch0 .. ch0 + 3 of the lane's position
    {
      const int ch0 = mt_e * 32 + 8 * qd_e + 4 * hi;
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = 0.0f;
#pragma unroll
      for (int w = 0; w < AN_BW; ++w)
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] += s_part[(w * 64 + lane) * SP + mt_e * 16 + 4 * qd_e + e];
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] += s.b2[ch0 + e];
      const size_t pc = ((size_t)pos.img * a.ho + pos.i) * a.wo + pos.j;
      if (!a.kid && pos.ok) {
        const uint2 u = *reinterpret_cast<const uint2*>(a.fin + pc * AN_C + ch0);
        v[0] += bf16_f(u.x & 0xffffu);
        v[1] += bf16_f(u.x >> 16);
        v[2] += bf16_f(u.y & 0xffffu);
        v[3] += bf16_f(u.y >> 16);
      }
      uint32_t h[4];
      float hsum = 0.0f;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        h[e] = bf16_rne(v[e]);
        hsum = __builtin_fmaf(s.hw[ch0 + e], bf16_f(h[e]), hsum);
      }
      if (pos.ok) *reinterpret_cast<uint2*>(a.fout + pc * AN_C + ch0) = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
      if (a.head) {
        hsum += __shfl_xor(hsum, 32, 64);
        if (hi == 0) s_head[wave * 32 + col] = hsum;
      }
    }
    if (a.head) {  // uniform
      __syncthreads();
      if (wave == 0 && hi == 0 && pos.ok) {
        float y = 0.0f;
#pragma unroll
        for (int w = 0; w < AN_BW; ++w) y += s_head[w * 32 + col];
        a.y[(size_t)pos.img * a.n_lat + a.loff + pos.i * a.wo + pos.j] = y + a.head[AN_C];
      }
    }
  }
}

// ------------------------------------------------------------------ host

// positions are counted in 32 bits on the device: n H W < 2^31
bool an_sizes_ok(int H, int W, int n) {
  return n >= 1 && H >= 64 && W >= 64 && H % 64 == 0 && W % 64 == 0 && (long long)n * H * W <= 0x7fffffffLL;
}

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
  w.t = w.f1 + up(feat);  // the first block's T: 16 channels per position
  w.total = w.t + up((size_t)n * H * W * 16 * sizeof(uint16_t));
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
    const long long tiles = (npx + 31) / 32;  // 32 positions per wave step
    if (B.c_in == 3) {
      if (hipLaunchKernel((const void*)ana_dw3_kernel, dim3((unsigned)((npx + AN_THREADS - 1) / AN_THREADS)),
                          dim3(AN_THREADS), argv, 0, st) != hipSuccess)
        return CC_EHIP;
      const unsigned grid = (unsigned)std::min<long long>((tiles + 3) / 4, AN_MAX_GRID);
      if (hipLaunchKernel((const void*)ana_mlp16_kernel, dim3(grid), dim3(AN_THREADS), argv, 0, st) != hipSuccess)
        return CC_EHIP;
    } else if (a.ho * a.wo <= AN_TEAM_MAX_POSITIONS) {
      // chosen by the size per image only, so a batch of images runs every
      // block with the same kernel as single images
      const void* k = B.stride == 2 ? (const void*)ana_block_team_kernel<2> : (const void*)ana_block_team_kernel<1>;
      const unsigned grid = (unsigned)std::min<long long>(tiles, AN_BLOCK_GRID);
      if (hipLaunchKernel(k, dim3(grid), dim3(AN_BT), argv, 0, st) != hipSuccess) return CC_EHIP;
    } else {
      const bool rowseg = a.wo % 32 == 0;
      const void* k = B.stride == 2 ? (rowseg ? (const void*)ana_block_kernel<2, true> : (const void*)ana_block_kernel<2, false>)
                                    : (rowseg ? (const void*)ana_block_kernel<1, true> : (const void*)ana_block_kernel<1, false>);
      const unsigned grid = (unsigned)std::min<long long>((tiles + AN_BW - 1) / AN_BW, AN_BLOCK_GRID);
      if (hipLaunchKernel(k, dim3(grid), dim3(AN_BT), argv, 0, st) != hipSuccess) return CC_EHIP;
    }
    hin = a.ho;
    win = a.wo;
  }
  return hipGetLastError() == hipSuccess ? CC_OK : CC_EHIP;
}

}  // extern "C"

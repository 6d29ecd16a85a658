// Kernel argument blocks and entry points shared by the kernel sources and
// the host-side C ABI.
#pragma once

#include "common.hpp"

namespace cc {

// ---------------------------------------------------------------- ARM
constexpr int ARM_TH = 4, ARM_TW = 64;               // latents per tile: rows x columns
constexpr int ARM_EH = ARM_TH + 3, ARM_EW = ARM_TW + 6;  // tile + causal halo frame
constexpr int ARM_EXT = ARM_EH * ARM_EW;
constexpr int ARM_THREADS = 256, ARM_WAVES = 4;

struct ArmTiles {
  int n_tiles;
  int base[MAXL + 1];  // first tile of level l
  int nth[MAXL + 1];   // tile rows of level l
  int ntw[MAXL + 1];   // tile columns of level l
};

struct ArmArgs {
  Geo geo;
  ArmTiles tiles;
  const float* y;
  const float* u;
  int quant;
  const float* w;      // packed ARM parameters
  float scale;         // dloss * lambda / (H W): gradient of the loss per bit
  float* rate_map;     // optional [N_lat]
  float* yq_out;       // optional [N_lat]
  float* gext;         // backward: [n_tiles][ARM_EXT] gathered context gradients
  float* wpart;        // backward: [gridDim][n_arm] weight-gradient partials
  float* rpart;        // [gridDim] rate partial sums (bits)
};
// kernel handle (host stub address) for hipLaunchKernel; batch: the variant
// taking (const ArmArgs* descs, const WorkItem* work)
const void* arm_kernel_for(int C, int NH, bool bwd, bool batch);

struct FoldArgs {
  Geo geo;
  ArmTiles tiles;
  const float* gext;
  float* g_y;
  int q0, q1;          // the latents [q0, q1) of the packed pyramid
  float *th, *m, *v;   // fused Adam: the latents and their moments (indexed like g_y)
};


// ---------------------------------------------------------------- upsampling
// level-1 tile side of the upsampling forward (one work-group per tile):
// small tiles fill the device for one image; a batch has work-groups to
// spare and keeps the halo recompute of larger tiles low
constexpr int UF_T = 16, UF_T_BATCH = 32;
struct UpsFwdArgs {
  Geo geo;
  const float* y;
  const float* u;
  int quant;
  const float* ups_w;          // [L-1][2][K] all taps
  float* up_out[MAXL];         // U_s output [(L-1-s)][h_s][w_s] for s = 1..L-2
};
__global__ void ups_fwd_kernel(UpsFwdArgs a);
__global__ void ups_fwd_kernel_batch(const UpsFwdArgs* d, const WorkItem* w);

struct UpsBwdArgs {
  Geo geo;
  int s;               // adjoint of step s: g_stack_s[1..] (level s) -> g_stack_{s+1} (level s+1)
  const float* y;
  const float* u;
  int quant;
  const float* taps;   // [2][K]
  const float* up_in;  // forward U_{s+1} output (channels 1.. of stack_{s+1}); null when s = L-2
  const float* g_in;   // [(L-1-s)][h_s][w_s]: gradient of U_s's output
  float* g_y;          // level s+1 of the packed latent gradient (channel 0 of g_stack_{s+1})
  float* g_out;        // [(L-2-s)][h_{s+1}][w_{s+1}]: channels 1.. of g_stack_{s+1}; null when s = L-2
  float* part;         // [chunks][tiles][2K] tap-gradient partials
  int cpb;             // channels of stack_{s+1} per block: block (tile, chunk) takes [chunk cpb, chunk cpb + cpb)
};
__global__ void ups_bwd_kernel(UpsBwdArgs a);
__global__ void ups_bwd_kernel_batch(const UpsBwdArgs* d, const WorkItem* w);


// ---------------------------------------------------------------- synthesis
constexpr int SYN_T = 16;                  // output tile side (pixels)
constexpr int SYN_T0_H = 16, SYN_T0_W = 32;  // pixel tile of syn_t0_kernel
constexpr int SYN_HD = 16;                 // pixel tile side of syn_head_bwd_kernel (one pixel per thread)
constexpr int SYN_THREADS = 256;
constexpr int SYN_MAXRES = 2;              // residual 3x3 convs supported
constexpr int SYN_FMAX = SYN_T + 4 * SYN_MAXRES;  // largest LDS frame side
// channel stride of an LDS frame: padded off a multiple of the bank count, so
// that the weight-gradient operand reads across channels spread over banks
// (43 % fewer bank-conflict cycles in the residual-conv backward)
constexpr int SYN_FA = SYN_FMAX * SYN_FMAX + 4;

struct SynArgs {
  Geo geo;
  const float* y;
  const float* u;
  int quant;
  const float* ups0;   // [2][K] taps of step 0
  const float* up1;    // U_1 output (channels 1.. of stack_1); null when L = 2
  const float* w;      // packed synthesis parameters
  int n_res;
  int res_off;         // offset of the first residual conv inside w
  const float* img;    // [3][H][W] (may be null for decoding)
  float* t0;           // [3][H][W] output of the two 1x1 layers
  float* xhat;         // optional [3][H][W]
  float dscale;        // backward: dloss * 2 / (3 H W)
  float* g_y;          // backward: level 0 of the packed latent gradient
  float* gz;           // backward: [(L-1)][H][W] gradient of U_0's output
  float* gpt;          // backward: [3][H][W] gradient at the pre-activation of t0
  float* wpart;        // backward: [gridDim][n_res * 84] residual-conv weight-gradient partials
  float* hpart;        // backward: [head tiles][Hs L + 4 Hs + 3] 1x1-layer weight-gradient partials
  float* spart;        // [gridDim] squared-error partial sums
  float* flag_clear;   // optional: block 0 of syn_t0_kernel stores 0 here (the non-finite flag of the pass)
  int n_tiles_x, n_tiles;
};
const void* syn_t0_kernel_for(int Hs, int nres, bool batch);
const void* syn_res_fwd_kernel_for(int Hs, int nres, bool batch);
const void* syn_bwd_kernel_for(int Hs, int nres, bool batch);
const void* syn_head_bwd_kernel_for(int Hs, int nres, bool batch);

// ---------------------------------------------------------------- reductions, optimiser
constexpr int RED_MAXSEG = 12;
struct RedSeg {
  const float* src;    // [rows][ld]
  int rows, cols, ld;
  int cpb;             // columns per block: 16 (16 row groups) or 1 (256 row groups)
  float* dst;          // [cols]
  float *th, *m, *v;   // fused Adam: the parameters of the columns and their moments, or null
};
struct FinalArgs {
  const float* rpart; int nr;    // rate partials (bits)
  const float* spart; int ns;    // squared-error partials
  const float* flags; int nflags;
  float lambda, inv_hw, inv_3hw;
  int have_rate, have_sse;
  int sticky;          // 1: loss4[3] is only ever set to 1 (cleared earlier in the pass), 0: written 0 or 1
  float* loss4;
};

// One launch does up to three independent jobs: blocks [0, n_red) sum
// partial matrices column by column (segments in order), blocks [n_red,
// n_red + fold blocks) fold the ARM context gradients into g_y, and block
// loss_block (when >= 0, in place of a fold block) evaluates the loss from
// fin.
struct CombineArgs {
  RedSeg seg[RED_MAXSEG];
  int nseg;
  int block_start[RED_MAXSEG + 1];
  FoldArgs fold;
  float* flags;        // [gridDim] 1 if any result of the block is not finite; or null, and then
  float* bad;          // a block with a non-finite result stores 1 here (never 0)
  int loss_block;
  FinalArgs fin;
  // Adam fused into the launch (on = 1): each final gradient value is
  // applied to its parameter at once.  The first of the pass's two launches
  // (last = 0) takes t = step[0] + 1 and its block 0 stores t in *t_slot; the
  // last one (last = 1) reads t there and its block 0 stores it in step[0]
  // (none of its blocks reads step[0], so no completion count is needed)
  struct {
    int on, last;
    int32_t* step;
    int32_t* t_slot;
    float lr, beta1, beta2, eps;
  } adam;
};
__global__ void combine_kernel(CombineArgs a);
__global__ void combine_kernel_batch(const CombineArgs* d, const WorkItem* w);
__global__ void finalize_kernel(FinalArgs a);

struct AdamArgs {
  float* theta;
  const float* g;
  float* m;
  float* v;
  int64_t n;
  int32_t* step;
  float lr, beta1, beta2, eps;
};
constexpr int ADAM_U = 4;  // float4 groups per thread and pass (vector form)
template <bool VEC>
__global__ void adam_kernel(AdamArgs a);
__global__ void noise_kernel(float* u, int64_t n, uint32_t k0, uint32_t k1, const int32_t* step, uint32_t stream_id);

// ---------------------------------------------------------------- warm start
constexpr int WS_CH = 32;          // trunk width
constexpr int WS_MAX_THETA = 4096; // decoder parameters the head can predict

// Level k = 0..4 of the trunk: k = 0 is the image (3 planar FP32 channels),
// k >= 1 the bfloat16 feature maps f_k [B][h_k][w_k][32] (channels last).
// The latent pyramid of each image is packed level by level (7 levels).
struct WarmArgs {
  int B, H, W;
  int h[5], w[5];
  int n_lat, n_theta, n_net;
  int loff[8], lh[8], lw[8];
  int conv_off[5];     // offset of W_k in the master vector (k = 1..4); b_k follows W_k
  int head_off[7];     // level l head block: V_l[32], beta_l (level 0: then K_0[27])
  int ptheta;          // P [n_theta][32], then pi [n_theta]
  const float* x;      // [B][3][H][W]
  const float* net;    // master parameters
  float* net_r;        // the same with every weight matrix rounded to bfloat16
  uint16_t* wf[5];     // forward operands [32][K] (K = 32 for k = 1, 288 otherwise)
  uint16_t* wt[5];     // data-adjoint operands [9][32 in][32 out] (k >= 2)
  uint16_t* f[5];      // feature maps (k >= 1)
  uint16_t* dp[5];     // gradient at the pre-activation, rounded (k >= 1)
  float* y;            // [B][n_lat] predicted latents
  float* theta;        // [B][n_theta] predicted decoder parameters
  const float* y_t;    // backward: targets (regression loss), or
  const float* th_t;
  const float* gy_in;  // backward: given gradients of an outer loss w.r.t. y and theta
  const float* gth_in;
  float sy, sth;       // 2 / (n_lat B), 2 / (n_theta B)
  float* gap;          // [B][32]
  float* dgap;         // [B][32]
  float* lpart_y;      // [heads grid] latent-loss partials
  float* lpart_th;     // [B] parameter-loss partials
  float* part_conv[5]; // [grid][32 * 9 * C_in + 32] conv weight / bias gradient partials
  float* part_h456;    // [grid][99] heads 4, 5, 6
  float* part_h[4];    // levels 1..3: [grid][33]
  float* part_v0;      // [grid][32] V_0 (level-0 path through f_1)
  float* part_h0;      // [grid][28] beta_0, K_0
  float* part_th;      // [B][33 n_theta] P, pi
};
__global__ void warm_prep_kernel(WarmArgs a);
__global__ void warm_heads_fwd_kernel(WarmArgs a, int with_loss);
__global__ void warm_theta_kernel(WarmArgs a, int bwd);
__global__ void warm_df4_kernel(WarmArgs a);
__global__ void warm_head0_grad_kernel(WarmArgs a);
__global__ void warm_bwd_data_kernel(WarmArgs a, int k);
const void* warm_conv_fwd_kernel_for(int k);
const void* warm_bwd_weight_kernel_for(int k);
constexpr int WS_DF4_POS = 64;     // f_4 positions per block of warm_df4_kernel

}  // namespace cc

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
  // the soft proxy (quant 3): its derivative multiplies the folded gradient
  const float* y;
  const float* u;
  int quant;
};


// ---------------------------------------------------------------- upsampling
// level-1 tile side of the upsampling forward (one work-group per tile):
// small tiles fill the device for one image; a batch has work-groups to
// spare and keeps the halo recompute of larger tiles low (its default; the
// batch also runs 16)
constexpr int UF_T = 16, UF_T_BATCH = 32;
// Upsampler kernels: separable, [L-1][2][8] (vertical, horizontal taps per
// step), or shared (Table I "1-1-TConv-K"): one non-separable [8][8] kernel
// for every step.  A 4-tap kernel runs as the 8-tap one with two zero taps
// on each side (same operator: p = 1 for K = 4 against p = 3 for K = 8).
struct UpsFwdArgs {
  Geo geo;
  const float* y;
  const float* u;
  int quant;
  int shared;                  // 0: separable taps, 1: one shared [8][8] kernel
  const float* ups_w;          // [L-1][2][8] all taps, or [8][8]
  float* up_out[MAXL];         // U_s output [(L-1-s)][h_s][w_s] for s = 1..L-2
};
// kernel handles (host stub addresses); batch: the variant taking
// (const UpsFwdArgs* descs, const WorkItem* work) with level-1 tiles of side
// tile (16 or 32; nullptr otherwise); the single-image kernel ignores tile
const void* ups_fwd_kernel_for(bool shared, bool batch, int tile = UF_T);

struct UpsBwdArgs {
  Geo geo;
  int s;               // adjoint of step s: g_stack_s[1..] (level s) -> g_stack_{s+1} (level s+1)
  const float* y;
  const float* u;
  int quant;
  int shared;          // 0: taps [2][8] of step s; 1: the shared [8][8] kernel
  const float* taps;   // [2][8] or [8][8]
  const float* up_in;  // forward U_{s+1} output (channels 1.. of stack_{s+1}); null when s = L-2
  const float* g_in;   // [(L-1-s)][h_s][w_s]: gradient of U_s's output
  float* g_y;          // level s+1 of the packed latent gradient (channel 0 of g_stack_{s+1})
  float* g_out;        // [(L-2-s)][h_{s+1}][w_{s+1}]: channels 1.. of g_stack_{s+1}; null when s = L-2
  float* part;         // [chunks][tiles][2K] (separable) or [chunks][tiles][64] (shared) tap-gradient partials
  int cpb;             // channels of stack_{s+1} per block: block (tile, chunk) takes [chunk cpb, chunk cpb + cpb)
};
const void* ups_bwd_kernel_for(bool shared, bool batch);
// Coarse steps of the adjoint of one image without the step-by-step chain
// (separable kernels, L >= 5): the gradient at U_s's output for 3 <= s <= L-2
// is the composed adjoint of steps 1 .. s-1 applied to the gradient at U_1's
// output, G_s = Cv^T G_1 Ch with the 1-D products Cv = V_1 ... V_{s-1} and
// Ch = H_1 ... H_{s-1}.  ups_bwd_coarse_kernel runs step 1 (work-groups
// [0, st1_wgs)) beside the composed G_s (the rest); ups_bwd_steps_kernel then
// runs steps 2 .. L-2 at once, each reading its G_s and writing its g_y level
// and tap partials (g_out null: the next step's input is already there).
constexpr int UC_R = 2;        // rows of G_s per composing work-group
constexpr int UC_POOL = 3072;  // LDS floats of a composing work-group
struct UpsComposeArgs {
  Geo geo;
  const float* taps;    // separable taps [L-1][2][8]
  const float* g1;      // gradient at U_1's output: [(L-2)][h_1][w_1], levels 2 .. L-1
  float* gs[MAXL];      // gs[s], 3 <= s <= L-2: gradient at U_s's output, [(L-1-s)][h_s][w_s]
  int first[MAXL + 1];  // composing work-groups of step s: [first[s], first[s + 1]), first[3] = 0
};
// LDS floats a composing work-group of step s needs (the row windows while
// they are built, the vertical pass and the horizontal steps' rows)
inline int ups_compose_lds(const Geo& g, int s) {
  const int m = s - 1, bm = 7 * ((1 << m) - 1) + 1, bp = 7 * ((1 << (m - 1)) - 1) + 1;
  const int umax = (UC_R - 1) * (1 << m) + bm;
  return ((UC_R * (bm + bp + umax) + 3) & ~3) + UC_R * (g.lw[1] + g.lw[1] / 2);
}
struct UpsBwdSteps {
  UpsBwdArgs st[MAXL];
  int first[MAXL + 1];  // work-groups of st[k]: [first[k], first[k + 1])
  int tiles[MAXL];
  int n;
};
__global__ void ups_bwd_coarse_kernel(UpsBwdArgs st1, int st1_tiles, int st1_wgs, UpsComposeArgs c);
__global__ void ups_bwd_steps_kernel(UpsBwdSteps m);
// 4-tap parameters (separable [L-1][2][4] or shared [4][4]) as 8-tap ones
// with two zero taps on each side; one thread per output tap
__global__ void ups_expand_kernel(const float* src, float* dst, int n_steps, int shared);
constexpr int UPS_SHARED_TAPS = UPS_K * UPS_K;


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
  int ups_shared;      // 0: ups0 = [2][8] taps of step 0; 1: ups0 = the shared [8][8] kernel
  const float* ups0;   // taps of step 0
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
  const int32_t* step; // optional (Adam fused into the combines): block 0 of syn_t0_kernel stores
  int32_t* t_slot;     //   step[0] + 1 in *t_slot, the step number both combine launches use
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
  int cpb;             // columns per block: 16 or, for 1024 rows or more, 4 (16 or 64 row groups)
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
  // applied to its parameter at once, with the step number t = *t_slot that
  // syn_t0_kernel stored at the start of the pass (step[0] + 1).  The launch
  // with store_step = 1 (the side combine) has its block 0 store t in
  // step[0]; no kernel of the pass reads step[0] after syn_t0_kernel, so the
  // two launches may run in either order or together
  struct {
    int on, store_step;
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

// ---------------------------------------------------------------- parameter quantisation
constexpr float PARAM_B_MIN = 0.01f;  // smallest Laplace scale of the parameter model
struct ParamQArgs {
  const float* src[3];   // ARM, upsampling, synthesis parameters
  float* dst[3];         // their quantised values (may alias src)
  int n[3];
  int k[3];              // step 2^-k per module
  float* bits;           // [3] rate of each module, bits
};
__global__ void param_quant_kernel(ParamQArgs a);

// ---------------------------------------------------------------- entropy coding
// Interleaved rANS over the latents with the ARM's Laplace probabilities
// (quantised per latent to a table row) and the wavefront decode order.
constexpr int CD_PREC = 16;                      // frequency total 2^16
constexpr uint32_t CD_TOTAL = 1u << CD_PREC;
constexpr uint32_t CD_RANS_L = 1u << 23;         // coder state in [2^23, 2^31)
constexpr int CD_A = 48;                         // |d| <= 48 has a symbol of its own
constexpr int CD_NSYM = 2 * CD_A + 2;            // 97 symbols and the escape
constexpr int CD_ESC = CD_NSYM - 1;
constexpr int CD_ROW = CD_NSYM + 1;              // cumulative frequencies per table row
constexpr int CD_NMU = 16;                       // mean offsets per integer
constexpr int CD_SCALE_PER_LN = 8;               // scale indices per unit of ln b
constexpr int CD_NSCALE = 75;                    // scale indices 0..74 (b = 0.01 .. 100)
constexpr float CD_LOG_BMIN = -0x1.26bb1cp+2f;   // ln 0.01 rounded to float32
constexpr float CD_LOG_BMAX = 0x1.26bb1cp+2f;    // ln 100
constexpr float CD_MU_LIM = 1048576.0f;          // |mu| clamp, 2^20
constexpr int CD_YQ_LIM = 1 << 20;               // |y_hat| limit of the coder
constexpr int CD_LANES = 64;                     // coder states per set (one wave)
constexpr int CD_RING = 16;                      // decoded columns kept per row
constexpr int CD_MAX_SETS = 2;
constexpr int CD_MAX_ROWS = 1024;                // rows of a set's first level (LDS of the decoder)
constexpr int CD_BYTES_PER_LATENT = 12;          // worst case: 6 symbols of 2 bytes
constexpr uint32_t CD_MAGIC = 0x31524343u;       // "CCR1"
constexpr int CD_ROW16 = 104;                    // uint16 copy of a row: cum[0..97], padding (16-byte rows)
constexpr int CD_SLOTS = 256;                    // table rows the decoder holds in LDS per chunk of a step

struct CodecSet {
  int n_lanes;   // coder states of the set (min(64, rows of its first level))
  int lv0, lv1;  // levels [lv0, lv1)
};

struct CodecArgs {
  Geo geo;
  int C, NH, slope, n_sets, rows_max;
  CodecSet set[CD_MAX_SETS];
  const float* w;                  // packed ARM parameters
  uint32_t* cum;                   // [CD_NSCALE * CD_NMU][CD_ROW]
  uint16_t* cum16;                 // [CD_NSCALE * CD_NMU][CD_ROW16]: cum[0..97] (cum[98] = 2^16 implied)
  // encoder
  const float* yq;                 // [N_lat] integer-valued latents
  uint16_t* tbl;                   // [N_lat] table row of each latent
  int32_t* dsym;                   // [N_lat] y_hat - c
  uint8_t* emit[CD_MAX_SETS];      // bytes in emission order, per set
  int64_t emit_cap[CD_MAX_SETS];
  uint32_t* meta;                  // [set] emitted bytes, [2 + 64 set + lane] final states, [130] bad latent, [131] overflow
  uint8_t* out;
  int64_t out_cap;
  int64_t* out_nbytes;
  // decoder
  const uint8_t* in;
  int64_t in_bytes;
  float* yq_out;
  int32_t* status;                 // [n_sets]
};
constexpr int CD_META_BAD = 2 + CD_MAX_SETS * CD_LANES, CD_META_OVF = CD_META_BAD + 1, CD_META_N = CD_META_OVF + 1;
__global__ void codec_table_kernel(uint32_t* cum, uint16_t* cum16, uint32_t* meta);
__global__ void codec_encode_kernel(CodecArgs a);
__global__ void codec_pack_kernel(CodecArgs a);
const void* codec_params_kernel_for(int C);
const void* codec_decode_kernel_for(int C);
size_t codec_decode_lds_bytes(int rows_max, int n_arm);  // dynamic LDS of the decoder

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

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
};


// ---------------------------------------------------------------- upsampling
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
  float* part;         // [gridDim][2K] tap-gradient partials
};
__global__ void ups_bwd_kernel(UpsBwdArgs a);
__global__ void ups_bwd_kernel_batch(const UpsBwdArgs* d, const WorkItem* w);

// ---------------------------------------------------------------- synthesis
constexpr int SYN_T = 16;                  // output tile side (pixels)
constexpr int SYN_THREADS = 256;
constexpr int SYN_MAXRES = 2;              // residual 3x3 convs supported
constexpr int SYN_FMAX = SYN_T + 4 * SYN_MAXRES;  // largest LDS frame side

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
  float* wpart;        // backward: [gridDim][n_syn]
  float* spart;        // [gridDim] squared-error partial sums
  int n_tiles_x, n_tiles;
};
const void* syn_t0_kernel_for(int Hs, int nres, bool batch);
const void* syn_res_fwd_kernel_for(int Hs, int nres, bool batch);
const void* syn_bwd_kernel_for(int Hs, int nres, bool batch);

// ---------------------------------------------------------------- reductions, optimiser
constexpr int RED_MAXSEG = 12;
struct RedSeg {
  const float* src;    // [rows][ld]
  int rows, cols, ld;
  int cpb;             // columns per block: 16 (16 row groups) or 1 (256 row groups)
  float* dst;          // [cols]
};
// One launch does two independent jobs: blocks [0, n_red) sum partial
// matrices column by column (segments in order), blocks [n_red, n_red +
// fold blocks) fold the ARM context gradients into g_y.
struct CombineArgs {
  RedSeg seg[RED_MAXSEG];
  int nseg;
  int block_start[RED_MAXSEG + 1];
  FoldArgs fold;
  float* flags;        // [gridDim] 1 if any result of the block is not finite
};
__global__ void combine_kernel(CombineArgs a);
__global__ void combine_kernel_batch(const CombineArgs* d, const WorkItem* w);

struct FinalArgs {
  const float* rpart; int nr;    // rate partials (bits)
  const float* spart; int ns;    // squared-error partials
  const float* flags; int nflags;
  float lambda, inv_hw, inv_3hw;
  int have_rate, have_sse;
  float* loss4;
};
__global__ void finalize_kernel(FinalArgs a);
__global__ void finalize_kernel_batch(const FinalArgs* d);

struct AdamArgs {
  float* theta;
  const float* g;
  float* m;
  float* v;
  int64_t n;
  int32_t* step;
  float lr, beta1, beta2, eps;
};
__global__ void adam_kernel(AdamArgs a);

}  // namespace cc

// Host side of the C ABI declared in include/coolchic.h: argument checks,
// workspace layout, and the launch sequence of each entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "coolchic.h"
#include "kernels.hpp"

namespace cc {
namespace {

constexpr size_t ALIGN_FLOATS = 64;  // 256-byte alignment of workspace blocks
constexpr int MAX_GRID = 512;

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

struct Plan {
  Geo geo;
  ArmTiles tiles;
  int C, NH, K, Hs, nres;
  int64_t n_arm, n_ups, n_syn;
  int arm_grid, syn_grid, syn_tiles_x, syn_tiles, fold_grid, red_grid;
  int red_blocks_arm, red_blocks_ups[MAXL], red_blocks_syn;
  int ups_grid[MAXL];
  // workspace offsets, in floats
  size_t up[MAXL];       // U_s output, s = 1..L-2
  size_t gb[MAXL];       // adjoint buffers, s = 1..L-2
  size_t t0, gz, gext, wpart_arm, wpart_syn, rpart, spart, upart[MAXL], flags, total;
};

bool arch_ok(const cc_arch* a) {
  if (!a) return false;
  if (a->n_levels < 2 || a->n_levels > MAXL) return false;
  if (a->arm_ctx != 8 && a->arm_ctx != 16 && a->arm_ctx != 24) return false;
  if (a->arm_layers < 1 || a->arm_layers > 3) return false;
  if (a->ups_taps != UPS_K) return false;
  if (a->syn_hidden < 8 || a->syn_hidden > 48 || a->syn_hidden % 8) return false;
  if (a->syn_res < 1 || a->syn_res > SYN_MAXRES) return false;
  return true;
}

void counts(const cc_arch* a, int64_t* n_arm, int64_t* n_ups, int64_t* n_syn) {
  const int64_t C = a->arm_ctx, L = a->n_levels, Hs = a->syn_hidden;
  *n_arm = a->arm_layers * (C * C + C) + 2 * C + 2;
  *n_ups = (L - 1) * 2 * a->ups_taps;
  *n_syn = Hs * L + Hs + 3 * Hs + 3 + a->syn_res * 84;
}

// Shape checks only; CC_EUNSUPPORTED for a well-formed but not compiled arch.
int check_problem(const cc_problem* p) {
  if (!p) return CC_EINVAL;
  const cc_arch* a = &p->arch;
  if (a->n_levels < 1 || a->n_levels > 16) return CC_EINVAL;
  if (p->H <= 0 || p->W <= 0 || p->H > 16384 || p->W > 16384) return CC_EINVAL;
  const int m = 1 << (a->n_levels - 1);
  if (p->H % m || p->W % m) return CC_EINVAL;
  if (p->quant != CC_QUANT_ROUND && p->quant != CC_QUANT_NOISE) return CC_EINVAL;
  if (!arch_ok(a)) return CC_EUNSUPPORTED;
  return CC_OK;
}

size_t take(size_t& cur, size_t n) {
  const size_t at = cur;
  cur += (n + ALIGN_FLOATS - 1) / ALIGN_FLOATS * ALIGN_FLOATS;
  return at;
}

int make_plan(const cc_problem* p, int which, Plan* P) {
  int rc = check_problem(p);
  if (rc) return rc;
  std::memset(P, 0, sizeof(*P));
  const cc_arch* a = &p->arch;
  const int L = a->n_levels;
  P->C = a->arm_ctx; P->NH = a->arm_layers; P->K = a->ups_taps; P->Hs = a->syn_hidden; P->nres = a->syn_res;
  counts(a, &P->n_arm, &P->n_ups, &P->n_syn);
  Geo& g = P->geo;
  g.H = p->H; g.W = p->W; g.L = L;
  int off = 0;
  for (int l = 0; l < L; ++l) {
    g.lh[l] = p->H >> l; g.lw[l] = p->W >> l; g.loff[l] = off;
    off += g.lh[l] * g.lw[l];
  }
  g.loff[L] = off;
  g.n_lat = off;
  ArmTiles& t = P->tiles;
  int nt = 0;
  for (int l = 0; l < L; ++l) {
    t.base[l] = nt;
    t.nth[l] = cdiv(g.lh[l], ARM_TH);
    t.ntw[l] = cdiv(g.lw[l], ARM_TW);
    nt += t.nth[l] * t.ntw[l];
  }
  t.base[L] = nt;
  t.n_tiles = nt;
  P->arm_grid = std::min(nt, MAX_GRID);
  P->syn_tiles_x = cdiv(p->W, SYN_T);
  P->syn_tiles = P->syn_tiles_x * cdiv(p->H, SYN_T);
  P->syn_grid = std::min(P->syn_tiles, MAX_GRID);
  for (int s = 0; s + 1 < L; ++s) P->ups_grid[s] = cdiv(g.lh[s + 1], 16) * cdiv(g.lw[s + 1], 16);  // tiles
  P->fold_grid = cdiv(g.n_lat, 256);
  // column reductions: 16 columns per block for the wide ARM / synthesis
  // partials (at most MAX_GRID rows), one column per block for the tall
  // upsampling partials (tiles x channels rows)
  P->red_blocks_arm = cdiv((int)P->n_arm, 16);
  P->red_blocks_syn = cdiv((int)P->n_syn, 16);
  P->red_grid = P->red_blocks_arm + P->red_blocks_syn;
  for (int s = 0; s + 1 < L; ++s) {
    P->red_blocks_ups[s] = 2 * UPS_K;
    P->red_grid += P->red_blocks_ups[s];
  }

  size_t cur = 0;
  for (int s = 1; s + 1 < L; ++s) P->up[s] = take(cur, (size_t)(L - 1 - s) * g.lh[s] * g.lw[s]);
  P->t0 = take(cur, (size_t)3 * p->H * p->W);
  P->rpart = take(cur, P->arm_grid);
  P->spart = take(cur, P->syn_grid);
  if (which == CC_WS_BACKWARD) {
    P->gz = take(cur, (size_t)(L - 1) * p->H * p->W);
    for (int s = 1; s + 1 < L; ++s) P->gb[s] = take(cur, (size_t)(L - 1 - s) * g.lh[s] * g.lw[s]);
    P->gext = take(cur, (size_t)nt * ARM_EXT);
    P->wpart_arm = take(cur, (size_t)P->arm_grid * P->n_arm);
    P->wpart_syn = take(cur, (size_t)P->syn_grid * P->n_syn);
    for (int s = 0; s + 1 < L; ++s) P->upart[s] = take(cur, (size_t)P->ups_grid[s] * (L - 1 - s) * 2 * UPS_K);
    P->flags = take(cur, (size_t)P->red_grid + P->fold_grid);
  }
  P->total = cur;
  return CC_OK;
}

int launch(const void* fn, int grid, int block, void* args, hipStream_t st) {
  void* argv[] = {args};
  return hipLaunchKernel(fn, dim3(grid), dim3(block), argv, 0, st) == hipSuccess ? CC_OK : CC_EHIP;
}

// measurement hook: events recorded around one stage's launch
int g_stage = CC_STAGE_NONE;
hipEvent_t g_ev_begin = nullptr, g_ev_end = nullptr;

int launch_stage(int stage, const void* fn, int grid, int block, void* args, hipStream_t st) {
  const bool timed = stage == g_stage && g_ev_begin && g_ev_end;
  if (timed && hipEventRecord(g_ev_begin, st) != hipSuccess) return CC_EHIP;
  int rc = launch(fn, grid, block, args, st);
  if (rc) return rc;
  if (timed && hipEventRecord(g_ev_end, st) != hipSuccess) return CC_EHIP;
  return CC_OK;
}

// Side stream per device for the ARM kernel, which is independent of the
// upsampling / synthesis chain until the final reductions: the call forks it
// off the caller's stream with an event and joins it back with another.
// Created once per device on first use (default priority, non-blocking).
struct Side {
  hipStream_t stream = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
constexpr int MAX_DEVICES = 64;
Side g_side[MAX_DEVICES];
std::mutex g_side_mu;  // also serialises the fork/join enqueue of concurrent calls

int side_for_current_device(Side** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return CC_EHIP;
  Side& sd = g_side[dev];
  if (!sd.stream) {
    if (hipStreamCreateWithFlags(&sd.stream, hipStreamNonBlocking) != hipSuccess) return CC_EHIP;
    if (hipEventCreateWithFlags(&sd.fork, hipEventDisableTiming) != hipSuccess) return CC_EHIP;
    if (hipEventCreateWithFlags(&sd.join, hipEventDisableTiming) != hipSuccess) return CC_EHIP;
  }
  *out = &sd;
  return CC_OK;
}

int fork_to(Side* sd, hipStream_t main) {
  if (hipEventRecord(sd->fork, main) != hipSuccess) return CC_EHIP;
  return hipStreamWaitEvent(sd->stream, sd->fork, 0) == hipSuccess ? CC_OK : CC_EHIP;
}

int join_from(Side* sd, hipStream_t main) {
  if (hipEventRecord(sd->join, sd->stream) != hipSuccess) return CC_EHIP;
  return hipStreamWaitEvent(main, sd->join, 0) == hipSuccess ? CC_OK : CC_EHIP;
}

// U_s for s = L-2 .. 1 in one launch (stack_1 is then complete for the
// step s = 0 fused into the synthesis kernels).
int launch_ups_fwd(const Plan& P, float* ws, const float* y, const float* u, int quant, const float* ups_w,
                   hipStream_t st) {
  const int L = P.geo.L;
  if (L < 3) return CC_OK;
  UpsFwdArgs a;
  std::memset(&a, 0, sizeof(a));
  a.geo = P.geo; a.y = y; a.u = u; a.quant = quant; a.ups_w = ups_w;
  for (int s = 1; s + 1 < L; ++s) a.up_out[s] = ws + P.up[s];
  const int grid = cdiv(P.geo.lh[1], 32) * cdiv(P.geo.lw[1], 32);
  return launch((const void*)ups_fwd_kernel, grid, 256, &a, st);
}

SynArgs syn_args(const Plan& P, float* ws, const float* y, const float* u, int quant, const float* ups_w,
                 const float* syn_w) {
  SynArgs a;
  std::memset(&a, 0, sizeof(a));
  a.geo = P.geo; a.y = y; a.u = u; a.quant = quant;
  a.ups0 = ups_w;
  a.up1 = P.geo.L > 2 ? ws + P.up[1] : nullptr;
  a.w = syn_w;
  a.n_res = P.nres;
  a.res_off = P.Hs * P.geo.L + 4 * P.Hs + 3;
  a.t0 = ws + P.t0;
  a.n_tiles_x = P.syn_tiles_x;
  a.n_tiles = P.syn_tiles;
  return a;
}

}  // namespace
}  // namespace cc

using namespace cc;

extern "C" {

int64_t coolchic_param_count(const cc_arch* arch, int64_t* n_arm, int64_t* n_ups, int64_t* n_syn) {
  if (!arch || !arch_ok(arch)) return -1;
  int64_t a, u, s;
  counts(arch, &a, &u, &s);
  if (n_arm) *n_arm = a;
  if (n_ups) *n_ups = u;
  if (n_syn) *n_syn = s;
  return a + u + s;
}

int64_t coolchic_latent_count(const cc_problem* p) {
  Plan P;
  if (make_plan(p, CC_WS_FORWARD, &P)) return -1;
  return P.geo.n_lat;
}

size_t coolchic_workspace_bytes(const cc_problem* p, int which) {
  Plan P;
  if (which < CC_WS_FORWARD || which > CC_WS_DECODE) return 0;
  if (make_plan(p, which, &P)) return 0;
  return P.total * sizeof(float);
}

int coolchic_forward(const cc_problem* p, const float* img, const float* y, const float* u, const float* arm_w,
                     const float* ups_w, const float* syn_w, float* loss4, float* rate_map, float* yq_out,
                     float* xhat_out, void* ws, size_t ws_bytes, void* stream) {
  Plan P;
  int rc = make_plan(p, CC_WS_FORWARD, &P);
  if (rc) return rc;
  if (!img || !y || !arm_w || !ups_w || !syn_w || !loss4 || !ws) return CC_EINVAL;
  if (p->quant == CC_QUANT_NOISE && !u) return CC_EINVAL;
  if (ws_bytes < P.total * sizeof(float)) return CC_EWORKSPACE;
  ArmKernelFn armk = arm_kernel_for(P.C, P.NH, false);
  SynKernelFn t0k = syn_t0_kernel_for(P.Hs, P.nres), resk = syn_res_fwd_kernel_for(P.Hs, P.nres);
  if (!armk || !t0k || !resk) return CC_EUNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  float* W = (float*)ws;
  std::lock_guard<std::mutex> lock(g_side_mu);
  Side* sd = nullptr;
  if ((rc = side_for_current_device(&sd))) return rc;
  (void)hipGetLastError();
  ArmArgs aa;
  std::memset(&aa, 0, sizeof(aa));
  aa.geo = P.geo; aa.tiles = P.tiles; aa.y = y; aa.u = u; aa.quant = p->quant; aa.w = arm_w;
  aa.rate_map = rate_map; aa.yq_out = yq_out; aa.rpart = W + P.rpart;
  if ((rc = fork_to(sd, st))) return rc;
  if ((rc = launch_stage(CC_STAGE_ARM, (const void*)armk, P.arm_grid, ARM_THREADS, &aa, sd->stream))) return rc;
  if ((rc = launch_ups_fwd(P, W, y, u, p->quant, ups_w, st))) return rc;
  SynArgs sa = syn_args(P, W, y, u, p->quant, ups_w, syn_w);
  sa.img = img;
  sa.xhat = xhat_out;
  sa.spart = W + P.spart;
  if ((rc = launch((const void*)t0k, cdiv(p->H * p->W, 256), 256, &sa, st))) return rc;
  if ((rc = launch_stage(CC_STAGE_SYNTHESIS, (const void*)resk, P.syn_grid, SYN_THREADS, &sa, st))) return rc;
  if ((rc = join_from(sd, st))) return rc;
  FinalArgs fa;
  std::memset(&fa, 0, sizeof(fa));
  fa.rpart = W + P.rpart; fa.nr = P.arm_grid; fa.spart = W + P.spart; fa.ns = P.syn_grid;
  fa.lambda = p->lambda; fa.inv_hw = 1.0f / ((float)p->H * p->W); fa.inv_3hw = 1.0f / (3.0f * p->H * p->W);
  fa.have_rate = 1; fa.have_sse = 1; fa.loss4 = loss4;
  if ((rc = launch((const void*)finalize_kernel, 1, 256, &fa, st))) return rc;
  return hipGetLastError() == hipSuccess ? CC_OK : CC_EHIP;
}

int coolchic_backward(const cc_problem* p, const float* img, const float* y, const float* u, const float* arm_w,
                      const float* ups_w, const float* syn_w, float dloss, float* loss4, float* g_y, float* g_arm,
                      float* g_ups, float* g_syn, void* ws, size_t ws_bytes, void* stream) {
  Plan P;
  int rc = make_plan(p, CC_WS_BACKWARD, &P);
  if (rc) return rc;
  if (!img || !y || !arm_w || !ups_w || !syn_w || !loss4 || !g_y || !g_arm || !g_ups || !g_syn || !ws)
    return CC_EINVAL;
  if (p->quant == CC_QUANT_NOISE && !u) return CC_EINVAL;
  if (ws_bytes < P.total * sizeof(float)) return CC_EWORKSPACE;
  ArmKernelFn armk = arm_kernel_for(P.C, P.NH, true);
  SynKernelFn t0k = syn_t0_kernel_for(P.Hs, P.nres), bwk = syn_bwd_kernel_for(P.Hs, P.nres);
  if (!armk || !t0k || !bwk) return CC_EUNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  float* W = (float*)ws;
  const int L = P.geo.L;
  const float HW = (float)p->H * p->W;
  std::lock_guard<std::mutex> lock(g_side_mu);
  Side* sd = nullptr;
  if ((rc = side_for_current_device(&sd))) return rc;
  (void)hipGetLastError();
  ArmArgs aa;
  std::memset(&aa, 0, sizeof(aa));
  aa.geo = P.geo; aa.tiles = P.tiles; aa.y = y; aa.u = u; aa.quant = p->quant; aa.w = arm_w;
  aa.scale = dloss * p->lambda / HW;
  aa.gext = W + P.gext; aa.wpart = W + P.wpart_arm; aa.rpart = W + P.rpart;
  if ((rc = fork_to(sd, st))) return rc;
  if ((rc = launch_stage(CC_STAGE_ARM, (const void*)armk, P.arm_grid, ARM_THREADS, &aa, sd->stream))) return rc;
  if ((rc = launch_ups_fwd(P, W, y, u, p->quant, ups_w, st))) return rc;
  SynArgs sa = syn_args(P, W, y, u, p->quant, ups_w, syn_w);
  sa.img = img;
  sa.dscale = dloss * 2.0f / (3.0f * HW);
  sa.g_y = g_y;
  sa.gz = W + P.gz;
  sa.wpart = W + P.wpart_syn;
  sa.spart = W + P.spart;
  if ((rc = launch((const void*)t0k, cdiv(p->H * p->W, 256), 256, &sa, st))) return rc;
  if ((rc = launch_stage(CC_STAGE_SYNTHESIS, (const void*)bwk, P.syn_grid, SYN_THREADS, &sa, st))) return rc;
  for (int s = 0; s + 1 < L; ++s) {
    UpsBwdArgs ua;
    ua.geo = P.geo; ua.s = s; ua.y = y; ua.u = u; ua.quant = p->quant;
    ua.taps = ups_w + (size_t)s * 2 * UPS_K;
    ua.up_in = (s + 1 <= L - 2) ? W + P.up[s + 1] : nullptr;
    ua.g_in = s == 0 ? W + P.gz : W + P.gb[s];
    ua.g_y = g_y + P.geo.loff[s + 1];
    ua.g_out = (s + 1 <= L - 2) ? W + P.gb[s + 1] : nullptr;
    ua.part = W + P.upart[s];
    {
      void* argv[] = {&ua};
      if (hipLaunchKernel((const void*)ups_bwd_kernel, dim3(P.ups_grid[s], L - 1 - s), dim3(256), argv, 0, st) !=
          hipSuccess)
        return CC_EHIP;
    }
  }
  if ((rc = join_from(sd, st))) return rc;
  CombineArgs ca;
  std::memset(&ca, 0, sizeof(ca));
  int ns = 0, blk = 0;
  auto add = [&](const float* src, int rows, int cols, int cpb, float* dst) {
    ca.seg[ns] = RedSeg{src, rows, cols, cols, cpb, dst};
    ca.block_start[ns] = blk;
    blk += cdiv(cols, cpb);
    ++ns;
  };
  add(W + P.wpart_arm, P.arm_grid, (int)P.n_arm, 16, g_arm);
  for (int s = 0; s + 1 < L; ++s)
    add(W + P.upart[s], P.ups_grid[s] * (L - 1 - s), 2 * UPS_K, 1, g_ups + (size_t)s * 2 * UPS_K);
  add(W + P.wpart_syn, P.syn_grid, (int)P.n_syn, 16, g_syn);
  ca.nseg = ns;
  ca.block_start[ns] = blk;
  ca.fold.geo = P.geo; ca.fold.tiles = P.tiles; ca.fold.gext = W + P.gext; ca.fold.g_y = g_y;
  ca.flags = W + P.flags;
  if ((rc = launch((const void*)combine_kernel, blk + P.fold_grid, 256, &ca, st))) return rc;
  FinalArgs fa;
  std::memset(&fa, 0, sizeof(fa));
  fa.rpart = W + P.rpart; fa.nr = P.arm_grid; fa.spart = W + P.spart; fa.ns = P.syn_grid;
  fa.flags = W + P.flags; fa.nflags = P.red_grid + P.fold_grid;
  fa.lambda = p->lambda; fa.inv_hw = 1.0f / HW; fa.inv_3hw = 1.0f / (3.0f * HW);
  fa.have_rate = 1; fa.have_sse = 1; fa.loss4 = loss4;
  if ((rc = launch((const void*)finalize_kernel, 1, 256, &fa, st))) return rc;
  return hipGetLastError() == hipSuccess ? CC_OK : CC_EHIP;
}

int coolchic_decode_synth(const cc_problem* p, const float* yq, const float* ups_w, const float* syn_w, float* xhat,
                          void* ws, size_t ws_bytes, void* stream) {
  if (!p) return CC_EINVAL;
  cc_problem q = *p;
  q.quant = CC_QUANT_ROUND;  // shape checks only; latents are used as given
  Plan P;
  int rc = make_plan(&q, CC_WS_DECODE, &P);
  if (rc) return rc;
  if (!yq || !ups_w || !syn_w || !xhat || !ws) return CC_EINVAL;
  if (ws_bytes < P.total * sizeof(float)) return CC_EWORKSPACE;
  SynKernelFn t0k = syn_t0_kernel_for(P.Hs, P.nres), resk = syn_res_fwd_kernel_for(P.Hs, P.nres);
  if (!t0k || !resk) return CC_EUNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  float* W = (float*)ws;
  (void)hipGetLastError();
  if ((rc = launch_ups_fwd(P, W, yq, nullptr, 2, ups_w, st))) return rc;
  SynArgs sa = syn_args(P, W, yq, nullptr, 2, ups_w, syn_w);
  sa.xhat = xhat;
  if ((rc = launch((const void*)t0k, cdiv(p->H * p->W, 256), 256, &sa, st))) return rc;
  if ((rc = launch((const void*)resk, P.syn_grid, SYN_THREADS, &sa, st))) return rc;
  return hipGetLastError() == hipSuccess ? CC_OK : CC_EHIP;
}

int coolchic_adam_step(float* theta, const float* grad, float* m, float* v, int64_t n, int32_t* step, float lr,
                       float beta1, float beta2, float eps, void* stream) {
  if (!theta || !grad || !m || !v || !step || n <= 0) return CC_EINVAL;
  if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return CC_EINVAL;
  AdamArgs a{theta, grad, m, v, n, step, lr, beta1, beta2, eps};
  const int64_t blocks = (n + 255) / 256;
  const int grid = (int)std::min<int64_t>(blocks, 256);
  (void)hipGetLastError();
  int rc = launch((const void*)adam_kernel, grid, 256, &a, (hipStream_t)stream);
  if (rc) return rc;

  return hipGetLastError() == hipSuccess ? CC_OK : CC_EHIP;
}

int coolchic_set_stage_events(int stage, void* ev_begin, void* ev_end) {
  if (stage == CC_STAGE_NONE) {
    g_stage = CC_STAGE_NONE;
    g_ev_begin = g_ev_end = nullptr;
    return CC_OK;
  }
  if ((stage != CC_STAGE_ARM && stage != CC_STAGE_SYNTHESIS) || !ev_begin || !ev_end) return CC_EINVAL;
  g_stage = stage;
  g_ev_begin = (hipEvent_t)ev_begin;
  g_ev_end = (hipEvent_t)ev_end;
  return CC_OK;
}

const char* coolchic_strerror(int code) {
  switch (code) {
    case CC_OK: return "ok";
    case CC_EINVAL: return "invalid argument (null pointer, size, or H/W not a multiple of 2^(L-1))";
    case CC_EUNSUPPORTED: return "architecture not supported by the compiled kernels";
    case CC_EWORKSPACE: return "workspace smaller than coolchic_workspace_bytes()";
    case CC_EHIP: return "HIP kernel launch failed";
  }
  return "unknown error code";
}

}  // extern "C"

// Host side of the C ABI declared in include/coolchic.h: argument checks,
// workspace layout, and the launch sequence of each entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "coolchic.h"
#include "kernels.hpp"

namespace cc {
namespace {

constexpr size_t ALIGN_FLOATS = 64;  // 256-byte alignment of workspace blocks
constexpr int MAX_GRID = 1280;
constexpr int RED_CPB = 16;  // gradient columns per combine work-group (16 row groups each)
// columns per combine work-group for a segment of `rows` partial rows: tall
// segments (the synthesis partials of every pixel tile) take four columns
// and 64 row groups, so that each thread sums a few dozen rows
inline int red_cpb(long long rows) { return rows >= 1024 ? 4 : RED_CPB; }
// a batch's side combine starts after the level-0 upsampling adjoint and also
// folds level 1 (one image: after the head backward, level 0 only)
constexpr int BATCH_SIDE_LEVELS = 2;
static_assert(BATCH_SIDE_LEVELS == 1 || BATCH_SIDE_LEVELS == 2, "side combine after the head or step 0");
// Default ARM grid: the ARM launch runs beside the head backward and the
// upsampling-adjoint launches, and each of its work-groups holds ~78 KB of
// LDS; 384 work-groups (1.5 per CU of the 256-CU MI355X) leave part of the
// CUs to the other stream (measured: 296.9 us per 768x512 iteration against
// 318.1 us with 512 and 321.0 us with 768).
constexpr int ARM_DEFAULT_GRID = 384;

inline int cdiv(int a, int b) { return (a + b - 1) / b; }
// quantiser mode of the kernels: the public modes, with the soft proxy as 3
// (2 is the kernels' "latents used as given" of the decode path)
inline int kmode(int quant) { return quant == CC_QUANT_SOFT ? QMODE_SOFT : quant; }
inline bool needs_noise(int quant) { return quant == CC_QUANT_NOISE || quant == CC_QUANT_SOFT; }
inline int t0_tiles(int H, int W) { return cdiv(H, SYN_T0_H) * cdiv(W, SYN_T0_W); }

struct Plan {
  Geo geo;
  ArmTiles tiles;
  int C, NH, K, Hs, nres;
  int64_t n_arm, n_ups, n_syn;
  int shared;             // upsampler: one shared K x K kernel (Table I) instead of separable ones; K = 4 or 8
  int arm_grid, syn_grid, syn_tiles_x, syn_tiles, fold_split, fold_grid0, fold_grid1, red_grid;
  int red_blocks_arm, red_blocks_ups[MAXL], red_blocks_syn;
  int ups_grid[MAXL];
  int ups_cpb[MAXL], ups_chunks[MAXL];  // channels per upsampling-adjoint block, blocks per tile
  // one image's coarse adjoint steps composed (separable, L >= 5, LDS fits):
  // work-groups of each composed step s (prefix sums from s = 3)
  int coarse, comp_first[MAXL + 1];
  // workspace offsets, in floats
  size_t up[MAXL];       // U_s output, s = 1..L-2
  size_t gb[MAXL];       // adjoint buffers, s = 1..L-2
  size_t t0, gz, gpt, gext, wpart_arm, wpart_syn, hpart, rpart, spart, upart[MAXL], tslot, tapx, total;
  int up_rows[MAXL];      // tap-gradient partial rows of each upsampling step
  int head_grid;  // tiles of the 1x1-layer backward
  int n_head;     // 1x1-layer parameters (W1, b1, W2, b2)
};

bool arch_ok(const cc_arch* a) {
  if (!a) return false;
  if (a->n_levels < 1 || a->n_levels > MAXL) return false;
  if (a->arm_ctx != 8 && a->arm_ctx != 16 && a->arm_ctx != 24) return false;
  if (a->arm_layers < 1 || a->arm_layers > 3) return false;
  if (a->ups_taps != 4 && a->ups_taps != 8) return false;
  if (a->ups_shared != 0 && a->ups_shared != 1) return false;
  if (a->syn_hidden < 8 || a->syn_hidden > 48 || a->syn_hidden % 8) return false;
  if (a->syn_res < 1 || a->syn_res > SYN_MAXRES) return false;
  return true;
}

void counts(const cc_arch* a, int64_t* n_arm, int64_t* n_ups, int64_t* n_syn) {
  const int64_t C = a->arm_ctx, L = a->n_levels, Hs = a->syn_hidden;
  *n_arm = a->arm_layers * (C * C + C) + 2 * C + 2;
  *n_ups = L < 2 ? 0 : (a->ups_shared ? (int64_t)a->ups_taps * a->ups_taps : (L - 1) * 2 * a->ups_taps);
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
  if (p->quant != CC_QUANT_ROUND && p->quant != CC_QUANT_NOISE && p->quant != CC_QUANT_SOFT) return CC_EINVAL;
  if (!arch_ok(a)) return CC_EUNSUPPORTED;
  return CC_OK;
}

size_t take(size_t& cur, size_t n) {
  const size_t at = cur;
  cur += (n + ALIGN_FLOATS - 1) / ALIGN_FLOATS * ALIGN_FLOATS;
  return at;
}

int make_plan(const cc_problem* p, int which, Plan* P, int arm_grid = 0, int syn_grid = 0, int side_levels = 1) {
  int rc = check_problem(p);
  if (rc) return rc;
  std::memset(P, 0, sizeof(*P));
  const cc_arch* a = &p->arch;
  const int L = a->n_levels;
  P->C = a->arm_ctx; P->NH = a->arm_layers; P->K = a->ups_taps; P->Hs = a->syn_hidden; P->nres = a->syn_res;
  counts(a, &P->n_arm, &P->n_ups, &P->n_syn);
  P->shared = a->ups_shared;
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
  P->arm_grid = arm_grid > 0 ? std::min(arm_grid, nt) : std::min(nt, ARM_DEFAULT_GRID);
  P->syn_tiles_x = cdiv(p->W, SYN_T);
  P->syn_tiles = P->syn_tiles_x * cdiv(p->H, SYN_T);
  P->syn_grid = syn_grid > 0 ? std::min(syn_grid, P->syn_tiles) : std::min(P->syn_tiles, MAX_GRID);
  for (int s = 0; s + 1 < L; ++s) {
    P->ups_grid[s] = cdiv(g.lh[s + 1], 16) * cdiv(g.lw[s + 1], 16);  // tiles
    // a level with enough tiles to fill the device takes every channel of a
    // tile in one block; the small levels keep one channel per block
    P->ups_cpb[s] = P->ups_grid[s] >= 256 ? L - 1 - s : 1;
    P->ups_chunks[s] = cdiv(L - 1 - s, P->ups_cpb[s]);
  }
  P->coarse = !P->shared && L >= 5;
  for (int s = 3; s + 1 < L; ++s) P->coarse = P->coarse && ups_compose_lds(g, s) <= UC_POOL;
  if (P->coarse) {
    P->comp_first[3] = 0;
    for (int s = 3; s + 1 < L; ++s) P->comp_first[s + 1] = P->comp_first[s] + (L - 1 - s) * cdiv(g.lh[s], UC_R);
  }
  // the ARM context fold of the side combine takes the first side_levels
  // levels (level 0 is final once the head backward has run, level 1 after
  // the level-0 upsampling adjoint); the final combine folds the others
  P->fold_split = L > side_levels ? g.loff[side_levels] : g.n_lat;
  P->fold_grid0 = cdiv(P->fold_split, 256);
  P->fold_grid1 = cdiv(g.n_lat - P->fold_split, 256);
  // column reductions, one column per block (256 row groups: every column
  // has hundreds to thousands of partial rows)
  P->red_blocks_arm = cdiv((int)P->n_arm, red_cpb(P->arm_grid));
  P->n_head = P->Hs * L + 4 * P->Hs + 3;
  P->head_grid = cdiv(p->H, SYN_HD) * cdiv(p->W, SYN_HD);
  P->red_blocks_syn = cdiv(P->nres * 84, red_cpb(P->syn_grid)) + cdiv(P->n_head, red_cpb(P->head_grid));
  P->red_grid = P->red_blocks_arm + P->red_blocks_syn;
  // tap-gradient reduction blocks (segments as build_backward lays them out)
  long long ups_rows_all = 0;
  for (int s = 0; s + 1 < L; ++s) ups_rows_all += (long long)P->ups_grid[s] * P->ups_chunks[s];
  for (int s = 0; s + 1 < L; ++s) {
    const int c = red_cpb((long long)P->ups_grid[s] * P->ups_chunks[s]), ca = red_cpb(ups_rows_all);
    if (P->shared) P->red_blocks_ups[s] = s == 0 ? (P->K == 8 ? cdiv(UPS_SHARED_TAPS, ca) : 4 * cdiv(4, ca)) : 0;
    else P->red_blocks_ups[s] = P->K == 8 ? cdiv(2 * UPS_K, c) : 2 * cdiv(4, c);
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
    P->gpt = take(cur, (size_t)3 * p->H * p->W);
    P->wpart_syn = take(cur, (size_t)P->syn_grid * P->nres * 84);
    P->hpart = take(cur, (size_t)P->head_grid * P->n_head);
    for (int s = 0; s + 1 < L; ++s) P->up_rows[s] = P->ups_grid[s] * P->ups_chunks[s];
    if (P->shared) {
      // one matrix of [all steps' rows][64]: the shared kernel's gradient is
      // the column sums over every step
      size_t rows = 0;
      for (int s = 0; s + 1 < L; ++s) rows += P->up_rows[s];
      const size_t base = take(cur, rows * UPS_SHARED_TAPS);
      size_t r = 0;
      for (int s = 0; s + 1 < L; ++s) {
        P->upart[s] = base + r * UPS_SHARED_TAPS;
        r += P->up_rows[s];
      }
    } else {
      for (int s = 0; s + 1 < L; ++s) P->upart[s] = take(cur, (size_t)P->up_rows[s] * 2 * UPS_K);
    }
    P->tslot = take(cur, 1);  // the fused Adam's step number, stored by syn_t0_kernel for both combines
  }
  // 4-tap kernels run as 8-tap ones with zero taps on each side
  P->tapx = take(cur, P->K == 4 && L > 1 ? (P->shared ? UPS_SHARED_TAPS : (size_t)(L - 1) * 2 * UPS_K) : 0);
  P->total = cur;
  return CC_OK;
}

// The 8-tap form of the upsampling parameters the kernels use: ups_w itself
// for K = 8, else its zero-padded copy in the workspace (written by
// launch_expand).
const float* taps8(const Plan& P, float* ws, const float* ups_w) {
  return P.K == 8 || P.geo.L < 2 ? ups_w : ws + P.tapx;
}

int launch_expand(const Plan& P, float* ws, const float* ups_w, hipStream_t st) {
  if (P.K == 8 || P.geo.L < 2) return CC_OK;
  const float* src = ups_w;
  float* dst = ws + P.tapx;
  int steps = P.geo.L - 1, shared = P.shared;
  void* argv[] = {&src, &dst, &steps, &shared};
  const int n = shared ? UPS_SHARED_TAPS : steps * 2 * UPS_K;
  return hipLaunchKernel((const void*)ups_expand_kernel, dim3(cdiv(n, 64)), dim3(64), argv, 0, st) == hipSuccess
             ? CC_OK
             : CC_EHIP;
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

// Side stream for the ARM kernel, which is independent of the upsampling /
// synthesis chain until the final reductions: the call forks it off the
// caller's stream with an event and joins it back with another.  One side
// stream and event set per (device, caller stream), created on first use
// (default priority, non-blocking) or by coolchic_stream_prepare: calls on
// different streams do not share them and run concurrently; calls on one
// stream take its set's lock while they enqueue.
struct Side {
  int dev = -1;
  hipStream_t main = nullptr;  // the caller's stream this set serves
  hipStream_t stream = nullptr;
  hipEvent_t fork = nullptr, join = nullptr, head = nullptr, armdone = nullptr;
  std::mutex mu;
};
constexpr int MAX_DEVICES = 64;  // devices with a static-scratch address (coolchic_train_step_noalloc)
constexpr int MAX_SIDES = 256;
Side g_side[MAX_SIDES];
int g_n_side = 0;
std::mutex g_side_mu;  // guards the table

int side_for(hipStream_t main, Side** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CC_EHIP;
  std::lock_guard<std::mutex> lock(g_side_mu);
  for (int i = 0; i < g_n_side; ++i)
    if (g_side[i].dev == dev && g_side[i].main == main) {
      *out = &g_side[i];
      return CC_OK;
    }
  // a stream being captured into a graph without a set of its own uses one
  // the device already has (no stream or event is created during capture)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(main, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive)
    for (int i = 0; i < g_n_side; ++i)
      if (g_side[i].dev == dev) {
        *out = &g_side[i];
        return CC_OK;
      }
  if (g_n_side == MAX_SIDES) return CC_EUNSUPPORTED;
  Side& sd = g_side[g_n_side];
  if (hipStreamCreateWithFlags(&sd.stream, hipStreamNonBlocking) != hipSuccess) return CC_EHIP;
  // the events only order the two streams of one device: no system-scope
  // cache fence when they are recorded (1-2 % of the training iteration)
  const unsigned fl = hipEventDisableTiming | hipEventDisableSystemFence;
  if (hipEventCreateWithFlags(&sd.fork, fl) != hipSuccess || hipEventCreateWithFlags(&sd.join, fl) != hipSuccess ||
      hipEventCreateWithFlags(&sd.head, fl) != hipSuccess || hipEventCreateWithFlags(&sd.armdone, fl) != hipSuccess)
    return CC_EHIP;
  sd.dev = dev;
  sd.main = main;
  ++g_n_side;  // published only once complete
  *out = &sd;
  return CC_OK;
}

int fork_to(Side* sd, hipStream_t main) {
  if (hipEventRecord(sd->fork, main) != hipSuccess) return CC_EHIP;
  return hipStreamWaitEvent(sd->stream, sd->fork, 0) == hipSuccess ? CC_OK : CC_EHIP;
}

// the side stream waits for the work enqueued on main so far
int side_waits(Side* sd, hipStream_t main) {
  if (hipEventRecord(sd->head, main) != hipSuccess) return CC_EHIP;
  return hipStreamWaitEvent(sd->stream, sd->head, 0) == hipSuccess ? CC_OK : CC_EHIP;
}

int join_from(Side* sd, hipStream_t main) {
  if (hipEventRecord(sd->join, sd->stream) != hipSuccess) return CC_EHIP;
  return hipStreamWaitEvent(main, sd->join, 0) == hipSuccess ? CC_OK : CC_EHIP;
}

// U_s for s = L-2 .. 1 in one launch (stack_1 is then complete for the
// step s = 0 fused into the synthesis kernels); grid 0 when L < 3.
UpsFwdArgs ups_fwd_args(const Plan& P, float* ws, const float* y, const float* u, int quant, const float* ups_w,
                        int* grid) {
  const int L = P.geo.L;
  UpsFwdArgs a;
  std::memset(&a, 0, sizeof(a));
  a.geo = P.geo; a.y = y; a.u = u; a.quant = quant; a.ups_w = taps8(P, ws, ups_w); a.shared = P.shared;
  for (int s = 1; s + 1 < L; ++s) a.up_out[s] = ws + P.up[s];
  *grid = L < 3 ? 0 : cdiv(P.geo.lh[1], UF_T) * cdiv(P.geo.lw[1], UF_T);
  return a;
}

int launch_ups_fwd(const Plan& P, float* ws, const float* y, const float* u, int quant, const float* ups_w,
                   hipStream_t st) {
  int grid = 0;
  UpsFwdArgs a = ups_fwd_args(P, ws, y, u, quant, ups_w, &grid);
  if (!grid) return CC_OK;
  return launch(ups_fwd_kernel_for(P.shared, false), grid, 256, &a, st);
}

SynArgs syn_args(const Plan& P, float* ws, const float* y, const float* u, int quant, const float* ups_w,
                 const float* syn_w) {
  SynArgs a;
  std::memset(&a, 0, sizeof(a));
  a.geo = P.geo; a.y = y; a.u = u; a.quant = quant;
  a.ups0 = taps8(P, ws, ups_w);
  a.ups_shared = P.shared;
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
  if (!img || !y || !arm_w || (!ups_w && P.n_ups) || !syn_w || !loss4 || !ws) return CC_EINVAL;
  if (needs_noise(p->quant) && !u) return CC_EINVAL;
  if (ws_bytes < P.total * sizeof(float)) return CC_EWORKSPACE;
  const void* armk = arm_kernel_for(P.C, P.NH, false, false);
  const void *t0k = syn_t0_kernel_for(P.Hs, P.nres, false), *resk = syn_res_fwd_kernel_for(P.Hs, P.nres, false);
  if (!armk || !t0k || !resk) return CC_EUNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  float* W = (float*)ws;
  Side* sd = nullptr;
  if ((rc = side_for(st, &sd))) return rc;
  std::lock_guard<std::mutex> lock(sd->mu);
  (void)hipGetLastError();
  ArmArgs aa;
  std::memset(&aa, 0, sizeof(aa));
  aa.geo = P.geo; aa.tiles = P.tiles; aa.y = y; aa.u = u; aa.quant = kmode(p->quant); aa.w = arm_w;
  aa.rate_map = rate_map; aa.yq_out = yq_out; aa.rpart = W + P.rpart;
  if ((rc = fork_to(sd, st))) return rc;
  if ((rc = launch_stage(CC_STAGE_ARM, armk, P.arm_grid, ARM_THREADS, &aa, sd->stream))) return rc;
  if ((rc = launch_expand(P, W, ups_w, st))) return rc;
  if ((rc = launch_ups_fwd(P, W, y, u, kmode(p->quant), ups_w, st))) return rc;
  SynArgs sa = syn_args(P, W, y, u, kmode(p->quant), ups_w, syn_w);
  sa.img = img;
  sa.xhat = xhat_out;
  sa.spart = W + P.spart;
  if ((rc = launch(t0k, t0_tiles(p->H, p->W), 256, &sa, st))) return rc;
  if ((rc = launch_stage(CC_STAGE_SYNTHESIS, resk, P.syn_grid, SYN_THREADS, &sa, st))) return rc;
  if ((rc = join_from(sd, st))) return rc;
  FinalArgs fa;
  std::memset(&fa, 0, sizeof(fa));
  fa.rpart = W + P.rpart; fa.nr = P.arm_grid; fa.spart = W + P.spart; fa.ns = P.syn_grid;
  fa.lambda = p->lambda; fa.inv_hw = 1.0f / ((float)p->H * p->W); fa.inv_3hw = 1.0f / (3.0f * p->H * p->W);
  fa.have_rate = 1; fa.have_sse = 1; fa.loss4 = loss4;
  if ((rc = launch((const void*)finalize_kernel, 1, 256, &fa, st))) return rc;
  return hipGetLastError() == hipSuccess ? CC_OK : CC_EHIP;
}

// Every argument block of one image's backward pass, and the grids.
struct BwdSet {
  ArmArgs arm;
  UpsFwdArgs upf;
  SynArgs syn;
  UpsBwdArgs upb[MAXL];
  CombineArgs comb_side, comb_main;
  FinalArgs fin;
  int upf_grid, t0_grid, comb_side_grid, comb_main_grid;
};

void build_backward(const cc_problem* p, const Plan& P, float* W, const float* img, const float* y, const float* u,
                    const float* arm_w, const float* ups_w, const float* syn_w, float dloss, float* loss4, float* g_y,
                    float* g_arm, float* g_ups, float* g_syn, BwdSet* b) {
  std::memset(b, 0, sizeof(*b));
  const int L = P.geo.L;
  const float HW = (float)p->H * p->W;
  ArmArgs& aa = b->arm;
  aa.geo = P.geo; aa.tiles = P.tiles; aa.y = y; aa.u = u; aa.quant = kmode(p->quant); aa.w = arm_w;
  aa.scale = dloss * p->lambda / HW;
  aa.gext = W + P.gext; aa.wpart = W + P.wpart_arm; aa.rpart = W + P.rpart;
  b->upf = ups_fwd_args(P, W, y, u, kmode(p->quant), ups_w, &b->upf_grid);
  SynArgs& sa = b->syn;
  sa = syn_args(P, W, y, u, kmode(p->quant), ups_w, syn_w);
  sa.img = img;
  sa.dscale = dloss * 2.0f / (3.0f * HW);
  sa.g_y = g_y;
  sa.gz = W + P.gz;
  sa.gpt = W + P.gpt;
  sa.hpart = W + P.hpart;
  sa.wpart = W + P.wpart_syn;
  sa.spart = W + P.spart;
  sa.flag_clear = loss4 + 3;
  b->t0_grid = t0_tiles(p->H, p->W);
  for (int s = 0; s + 1 < L; ++s) {
    UpsBwdArgs& ua = b->upb[s];
    ua.geo = P.geo; ua.s = s; ua.y = y; ua.u = u; ua.quant = kmode(p->quant);
    ua.shared = P.shared;
    ua.taps = P.shared ? taps8(P, W, ups_w) : taps8(P, W, ups_w) + (size_t)s * 2 * UPS_K;
    ua.up_in = (s + 1 <= L - 2) ? W + P.up[s + 1] : nullptr;
    ua.g_in = s == 0 ? W + P.gz : W + P.gb[s];
    ua.g_y = g_y + P.geo.loff[s + 1];
    ua.g_out = (s + 1 <= L - 2) ? W + P.gb[s + 1] : nullptr;
    ua.part = W + P.upart[s];
    ua.cpb = P.ups_cpb[s];
  }
  // the loss of Eq. (1) from the rate and squared-error partials (complete
  // once the ARM and the residual-conv backward have run); the non-finite
  // flag loss4[3] is cleared by syn_t0_kernel and set by any combine block
  // or the loss block that meets a non-finite value
  FinalArgs& fa = b->fin;
  fa.rpart = W + P.rpart; fa.nr = P.arm_grid; fa.spart = W + P.spart; fa.ns = P.syn_grid;
  fa.flags = nullptr; fa.nflags = 0;
  fa.lambda = p->lambda; fa.inv_hw = 1.0f / HW; fa.inv_3hw = 1.0f / (3.0f * HW);
  fa.have_rate = 1; fa.have_sse = 1; fa.sticky = 1; fa.loss4 = loss4;
  // two combine launches: the side one (after the ARM and the head backward,
  // or for a batch the level-0 upsampling adjoint, beside the rest of the
  // adjoint) sums the ARM and synthesis weight-gradient partials, folds the
  // ARM context gradients of the first levels into g_y and evaluates the
  // loss in one more block; the final one sums the upsampling tap partials
  // and folds the context gradients of the other levels
  auto build = [&](CombineArgs& ca, int* grid, bool final_part) {
    int ns = 0, blk = 0;
    auto add = [&](const float* src, int rows, int cols, float* dst, int ld = 0) {
      const int cpb = red_cpb(rows);
      ca.seg[ns] = RedSeg{src, rows, cols, ld ? ld : cols, cpb, dst};
      ca.block_start[ns] = blk;
      blk += cdiv(cols, cpb);
      ++ns;
    };
    if (!final_part) {
      add(W + P.wpart_arm, P.arm_grid, (int)P.n_arm, g_arm);
      add(W + P.hpart, P.head_grid, P.n_head, g_syn);                                 // W1, b1, W2, b2
      add(W + P.wpart_syn, P.syn_grid, P.nres * 84, g_syn + (P.n_syn - P.nres * 84));  // residual convs
    } else {
      if (P.shared && L > 1) {
        // every step's rows of the shared kernel's partials, summed at once
        int rows = 0;
        for (int s = 0; s + 1 < L; ++s) rows += P.up_rows[s];
        if (P.K == 8) {
          add(W + P.upart[0], rows, UPS_SHARED_TAPS, g_ups);
        } else {  // the inner 4 x 4 taps of the 8 x 8 gradient
          for (int r = 0; r < 4; ++r) add(W + P.upart[0] + (r + 2) * UPS_K + 2, rows, 4, g_ups + 4 * r, UPS_SHARED_TAPS);
        }
      } else {
        for (int s = 0; s + 1 < L; ++s) {
          if (P.K == 8) {
            add(W + P.upart[s], P.up_rows[s], 2 * UPS_K, g_ups + (size_t)s * 2 * UPS_K);
          } else {  // the inner 4 taps of each direction
            add(W + P.upart[s] + 2, P.up_rows[s], 4, g_ups + (size_t)s * 8, 2 * UPS_K);
            add(W + P.upart[s] + UPS_K + 2, P.up_rows[s], 4, g_ups + (size_t)s * 8 + 4, 2 * UPS_K);
          }
        }
      }
    }
    ca.nseg = ns;
    ca.block_start[ns] = blk;
    ca.flags = nullptr;
    ca.bad = loss4 + 3;
    ca.loss_block = -1;
    ca.fold.geo = P.geo; ca.fold.tiles = P.tiles; ca.fold.gext = W + P.gext; ca.fold.g_y = g_y;
    ca.fold.y = y; ca.fold.u = u; ca.fold.quant = kmode(p->quant);
    if (final_part) {
      ca.fold.q0 = P.fold_split; ca.fold.q1 = P.geo.n_lat;
      // at least one block (a launch needs one): with a single level there
      // are no taps and every latent is folded by the side combine
      blk += std::max(P.fold_grid1, blk == 0 ? 1 : 0);
    } else {
      ca.fold.q0 = 0; ca.fold.q1 = P.fold_split;
      blk += P.fold_grid0;
      ca.loss_block = blk++;
      ca.fin = fa;
    }
    *grid = blk;
  };
  build(b->comb_side, &b->comb_side_grid, false);
  build(b->comb_main, &b->comb_main_grid, true);
}

}  // extern "C"

namespace cc {
namespace {
// Adam fused into the two combine launches of a backward pass, for the
// packed vectors theta = [y | arm_w | ups_w | syn_w] with grad, m, v laid out
// alike: every gradient the combines finalise is applied to its parameter
// there (level 0 of y and the ARM and synthesis weights in the side combine,
// once nothing of the pass reads them any more; levels 1.. of y and the taps
// in the final one, which advances the step counter).
struct FusedAdam {
  float *theta, *grad, *m, *v;
  int32_t* step;
  float lr, beta1, beta2, eps;
};

void fuse_adam(const FusedAdam& f, CombineArgs& ca, bool store_step, int32_t* t_slot) {
  ca.adam.on = 1;
  ca.adam.store_step = store_step ? 1 : 0;
  ca.adam.step = f.step;
  ca.adam.t_slot = t_slot;
  ca.adam.lr = f.lr; ca.adam.beta1 = f.beta1; ca.adam.beta2 = f.beta2; ca.adam.eps = f.eps;
  for (int k = 0; k < ca.nseg; ++k) {
    RedSeg& S = ca.seg[k];
    const ptrdiff_t o = S.dst - f.grad;
    S.th = f.theta + o; S.m = f.m + o; S.v = f.v + o;
  }
  const ptrdiff_t o = ca.fold.g_y - f.grad;
  ca.fold.th = f.theta + o; ca.fold.m = f.m + o; ca.fold.v = f.v + o;
}

// one_stream: every kernel on the caller's stream in dependency order (no
// side stream, so no stream or event is ever created); otherwise the ARM and
// the side combine run on the device's side stream beside the synthesis
// adjoint.  Both orders give bit-identical results.
int backward_impl(const cc_problem* p, const float* img, const float* y, const float* u, const float* arm_w,
                  const float* ups_w, const float* syn_w, float dloss, float* loss4, float* g_y, float* g_arm,
                  float* g_ups, float* g_syn, void* ws, size_t ws_bytes, void* stream, const FusedAdam* fused,
                  bool one_stream = false) {
  Plan P;
  int rc = make_plan(p, CC_WS_BACKWARD, &P);
  if (rc) return rc;
  if (!img || !y || !arm_w || (!ups_w && P.n_ups) || !syn_w || !loss4 || !g_y || !g_arm || (!g_ups && P.n_ups) ||
      !g_syn || !ws)
    return CC_EINVAL;
  if (needs_noise(p->quant) && !u) return CC_EINVAL;
  if (ws_bytes < P.total * sizeof(float)) return CC_EWORKSPACE;
  const void* armk = arm_kernel_for(P.C, P.NH, true, false);
  const void *t0k = syn_t0_kernel_for(P.Hs, P.nres, false), *bwk = syn_bwd_kernel_for(P.Hs, P.nres, false);
  const void* hdk = syn_head_bwd_kernel_for(P.Hs, P.nres, false);
  if (!armk || !t0k || !bwk || !hdk) return CC_EUNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  const int L = P.geo.L;
  static thread_local BwdSet b;
  build_backward(p, P, (float*)ws, img, y, u, arm_w, ups_w, syn_w, dloss, loss4, g_y, g_arm, g_ups, g_syn, &b);
  if (fused) {
    int32_t* t_slot = (int32_t*)((float*)ws + P.tslot);
    fuse_adam(*fused, b.comb_side, true, t_slot);
    fuse_adam(*fused, b.comb_main, false, t_slot);
    b.syn.step = fused->step;
    b.syn.t_slot = t_slot;
  }
  Side* sd = nullptr;
  if (!one_stream && (rc = side_for(st, &sd))) return rc;
  std::unique_lock<std::mutex> lock;
  if (sd) lock = std::unique_lock<std::mutex>(sd->mu);
  hipStream_t side = one_stream ? st : sd->stream;
  (void)hipGetLastError();
  if ((rc = launch_expand(P, (float*)ws, ups_w, st))) return rc;
  if (b.upf_grid && (rc = launch(ups_fwd_kernel_for(P.shared, false), b.upf_grid, 256, &b.upf, st))) return rc;
  if ((rc = launch(t0k, b.t0_grid, 256, &b.syn, st))) return rc;
  if ((rc = launch_stage(CC_STAGE_SYNTHESIS, bwk, P.syn_grid, SYN_THREADS, &b.syn, st))) return rc;
  // the ARM (independent of the synthesis chain) on the side stream, beside
  // the head backward and the latency-bound upsampling adjoint launches.
  // Eagerly enqueued, the head backward reaches the CUs first when the ARM is
  // forked just before it; a graph replay starts the forked ARM first and the
  // head backward then waits for CUs, so under stream capture the ARM is
  // forked after the head backward instead (measured at 768x512: eager 4337
  // against 3566 iterations/s with the late fork, graph-replayed 3681 against
  // 4327).
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess) return CC_EHIP;
  const bool late_fork = cap == hipStreamCaptureStatusActive;
  if (!late_fork) {
    if (!one_stream && (rc = fork_to(sd, st))) return rc;
    if ((rc = launch_stage(CC_STAGE_ARM, armk, P.arm_grid, ARM_THREADS, &b.arm, side))) return rc;
  }
  if ((rc = launch(hdk, P.head_grid, 256, &b.syn, st))) return rc;
  if (late_fork) {
    if (!one_stream && (rc = fork_to(sd, st))) return rc;
    if ((rc = launch_stage(CC_STAGE_ARM, armk, P.arm_grid, ARM_THREADS, &b.arm, side))) return rc;
  }
  // The final combine needs the ARM's context gradients but nothing of the
  // side combine.  Where the ARM and the side combine are the longer stream
  // (the 24-wide ARM, enqueued eagerly), it waits for the ARM alone so that
  // the two combines overlap, and the side combine is joined at the end of
  // the call (768x512: 4621 against 4504 iterations/s); otherwise it waits
  // for both (low decoder: 6330 against 6249 eager; graph replays, which fork
  // the ARM late: 4557 against 4487 and 6397 against 6162).
  const bool overlap = !one_stream && !late_fork && P.C == 24;
  if (overlap && hipEventRecord(sd->armdone, side) != hipSuccess) return CC_EHIP;
  // level 0 of g_y is final: the side combine may start
  if (!one_stream && (rc = side_waits(sd, st))) return rc;
  if ((rc = launch((const void*)combine_kernel, b.comb_side_grid, 256, &b.comb_side, side))) return rc;
  // the upsampling adjoint: step by step, or for L >= 5 step 0, then step 1
  // beside the composed inputs of steps 3 .. L-2, then steps 2 .. L-2 at once
  // (three launches instead of L - 1 latency-bound ones)
  for (int s = 0; s + 1 < L && (s == 0 || !P.coarse); ++s) {
    void* argv[] = {&b.upb[s]};
    if (hipLaunchKernel(ups_bwd_kernel_for(P.shared, false), dim3(P.ups_grid[s], P.ups_chunks[s]), dim3(256), argv, 0,
                        st) !=
        hipSuccess)
      return CC_EHIP;
  }
  if (P.coarse) {
    UpsComposeArgs ca;
    std::memset(&ca, 0, sizeof(ca));
    ca.geo = P.geo;
    ca.taps = b.upb[0].taps;  // the separable taps from step 0 on
    ca.g1 = b.upb[1].g_in;
    for (int s = 3; s + 1 < L; ++s) ca.gs[s] = b.upb[s - 1].g_out;
    std::memcpy(ca.first, P.comp_first, sizeof(ca.first));
    int st1_tiles = P.ups_grid[1], st1_wgs = P.ups_grid[1] * P.ups_chunks[1];
    void* argc[] = {&b.upb[1], &st1_tiles, &st1_wgs, &ca};
    if (hipLaunchKernel((const void*)ups_bwd_coarse_kernel, dim3(st1_wgs + P.comp_first[L - 1]), dim3(256), argc, 0,
                        st) != hipSuccess)
      return CC_EHIP;
    static thread_local UpsBwdSteps ms;
    std::memset(&ms, 0, sizeof(ms));
    ms.n = L - 3;
    for (int k = 0; k < ms.n; ++k) {
      const int s = k + 2;
      ms.st[k] = b.upb[s];
      ms.st[k].g_out = nullptr;
      ms.tiles[k] = P.ups_grid[s];
      ms.first[k + 1] = ms.first[k] + P.ups_grid[s] * P.ups_chunks[s];
    }
    void* argm[] = {&ms};
    if (hipLaunchKernel((const void*)ups_bwd_steps_kernel, dim3(ms.first[ms.n]), dim3(256), argm, 0, st) !=
        hipSuccess)
      return CC_EHIP;
  }
  if (overlap && hipStreamWaitEvent(st, sd->armdone, 0) != hipSuccess) return CC_EHIP;
  if (!overlap && !one_stream && (rc = join_from(sd, st))) return rc;
  if ((rc = launch((const void*)combine_kernel, b.comb_main_grid, 256, &b.comb_main, st))) return rc;
  if (overlap && (rc = join_from(sd, st))) return rc;
  return hipGetLastError() == hipSuccess ? CC_OK : CC_EHIP;
}

}  // namespace
}  // namespace cc

extern "C" {

int coolchic_backward(const cc_problem* p, const float* img, const float* y, const float* u, const float* arm_w,
                      const float* ups_w, const float* syn_w, float dloss, float* loss4, float* g_y, float* g_arm,
                      float* g_ups, float* g_syn, void* ws, size_t ws_bytes, void* stream) {
  return backward_impl(p, img, y, u, arm_w, ups_w, syn_w, dloss, loss4, g_y, g_arm, g_ups, g_syn, ws, ws_bytes,
                       stream, nullptr);
}

int coolchic_train_step(const cc_problem* p, const float* img, const float* u, float dloss, float* loss4,
                        float* theta, float* grad, float* m, float* v, int32_t* step, float lr, float beta1,
                        float beta2, float eps, void* ws, size_t ws_bytes, void* stream) {
  if (!p || !theta || !grad || !m || !v || !step) return CC_EINVAL;
  if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return CC_EINVAL;
  int64_t na = 0, nu = 0, ns = 0;
  if (coolchic_param_count(&p->arch, &na, &nu, &ns) <= 0) return CC_EUNSUPPORTED;
  const int64_t ny = coolchic_latent_count(p);
  if (ny <= 0) return CC_EINVAL;
  const FusedAdam f{theta, grad, m, v, step, lr, beta1, beta2, eps};
  return backward_impl(p, img, theta, u, theta + ny, theta + ny + na, theta + ny + na + nu, dloss, loss4, grad,
                       grad + ny, grad + ny + na, grad + ny + na + nu, ws, ws_bytes, stream, &f);
}

}  // extern "C"

// ------------------------------------------------ allocation-free training step

// The workspace of coolchic_train_step_noalloc: one copy per device, resident
// until the process ends (it is .bss of the code object: nothing is stored in
// the library file).  In host code `scratch` names a host-side stand-in, not
// device memory: only the address hipGetSymbolAddress returns for a device is
// ever handed to a kernel or a HIP call.
static __device__ __align__(256) unsigned char scratch[CC_NOALLOC_SCRATCH_BYTES];

namespace cc {
namespace {

void* g_scratch[MAX_DEVICES];  // device address of `scratch` on each device, set once
std::mutex g_scratch_mu;

// Looks up (once per device, with that device current) the device address of
// the static scratch array.
int scratch_for_current_device(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return CC_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return CC_EHIP;
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return CC_OK;
}

}  // namespace
}  // namespace cc

extern "C" {

int coolchic_train_step_noalloc(const cc_problem* p, const float* img, const float* u, float dloss, float* loss4,
                                float* theta, float* grad, float* m, float* v, int32_t* step, float lr, float beta1,
                                float beta2, float eps, void* stream) {
  // sizes first: a problem whose workspace does not fit is refused before
  // anything touches the device
  const size_t need = coolchic_workspace_bytes(p, CC_WS_BACKWARD);
  if (need == 0) {
    const int rc = check_problem(p);
    return rc ? rc : CC_EINVAL;
  }
  if (need > CC_NOALLOC_SCRATCH_BYTES) return CC_ESCRATCH;
  if (!theta || !grad || !m || !v || !step) return CC_EINVAL;
  if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return CC_EINVAL;
  int64_t na = 0, nu = 0, ns = 0;
  if (coolchic_param_count(&p->arch, &na, &nu, &ns) <= 0) return CC_EUNSUPPORTED;
  const int64_t ny = coolchic_latent_count(p);
  if (ny <= 0) return CC_EINVAL;
  void* ws = nullptr;
  int rc = scratch_for_current_device(&ws);
  if (rc) return rc;
  const FusedAdam f{theta, grad, m, v, step, lr, beta1, beta2, eps};
  return backward_impl(p, img, theta, u, theta + ny, theta + ny + na, theta + ny + na + nu, dloss, loss4, grad,
                       grad + ny, grad + ny + na, grad + ny + na + nu, ws, CC_NOALLOC_SCRATCH_BYTES, stream, &f,
                       /*one_stream=*/true);
}

}  // extern "C"

namespace cc {
namespace {

// Host-side plan of a batch.
struct BatchPlan {
  int n = 0, L = 0, device = 0, shared = 0, arm_first = 0, ups_tile = UF_T_BATCH;
  const void *armk = nullptr, *t0k = nullptr, *bwk = nullptr, *hdk = nullptr;
  // device arrays inside the workspace
  ArmArgs* d_arm = nullptr;
  UpsFwdArgs* d_upf = nullptr;
  SynArgs* d_syn = nullptr;
  UpsBwdArgs* d_upb[MAXL] = {};
  CombineArgs *d_comb_side = nullptr, *d_comb_main = nullptr;
  WorkItem *w_arm = nullptr, *w_upf = nullptr, *w_t0 = nullptr, *w_syn = nullptr, *w_head = nullptr,
           *w_upb[MAXL] = {}, *w_comb_side = nullptr, *w_comb_main = nullptr;
  int n_arm = 0, n_upf = 0, n_t0 = 0, n_syn = 0, n_head = 0, n_upb[MAXL] = {}, n_comb_side = 0, n_comb_main = 0;
};

// level-1 tile side of the batched upsampling forward; 0 for an invalid choice
int batch_ups_tile(const cc_batch_tuning* tune) {
  const int t = tune ? tune->ups_tile : 0;
  return t == 0 ? UF_T_BATCH : (t == 16 || t == 32) ? t : 0;
}

int share(int total, long long part, long long whole, int cap) {
  if (total <= 0) return 0;  // default grid
  long long g = (long long)total * part / whole;
  return (int)std::max(1LL, std::min<long long>(g, cap));
}

// Per-image plans for a batch and the layout of the batch workspace (bytes).
int batch_layout(int n, const cc_problem* probs, const cc_batch_tuning* tune, std::vector<Plan>& plans,
                 std::vector<size_t>& img_off, size_t* desc_off, size_t* total_bytes) {
  if (n <= 0 || !probs) return CC_EINVAL;
  long long tiles_arm = 0, tiles_syn = 0;
  plans.resize(n);
  for (int k = 0; k < n; ++k) {
    int rc = make_plan(&probs[k], CC_WS_BACKWARD, &plans[k], 0, 0, BATCH_SIDE_LEVELS);
    if (rc) return rc;
    const cc_arch &a = probs[k].arch, &a0 = probs[0].arch;
    if (std::memcmp(&a, &a0, sizeof(cc_arch)) || probs[k].quant != probs[0].quant) return CC_EINVAL;
    if (plans[k].K != 8) return CC_EUNSUPPORTED;  // the batch runs 8-tap upsamplers only
    tiles_arm += plans[k].tiles.n_tiles;
    tiles_syn += plans[k].syn_tiles;
  }
  const int ta = tune ? tune->arm_blocks : 0, ts = tune ? tune->syn_blocks : 0;
  if (tune && (tune->arm_first < 0 || tune->arm_first > 2)) return CC_EINVAL;
  const int ut = batch_ups_tile(tune);
  if (!ut) return CC_EINVAL;
  img_off.resize(n);
  size_t cur = 0;
  for (int k = 0; k < n; ++k) {
    const int ga = share(ta, plans[k].tiles.n_tiles, tiles_arm, 4096);
    const int gs = share(ts, plans[k].syn_tiles, tiles_syn, 4096);
    make_plan(&probs[k], CC_WS_BACKWARD, &plans[k], ga, gs, BATCH_SIDE_LEVELS);
    img_off[k] = cur;
    cur += (plans[k].total * sizeof(float) + 255) / 256 * 256;
  }
  *desc_off = cur;
  // descriptors and work-lists
  const int L = probs[0].arch.n_levels;
  size_t d = 0;
  auto blk = [&](size_t bytes) { d += (bytes + 255) / 256 * 256; };
  blk(sizeof(ArmArgs) * n);
  blk(sizeof(UpsFwdArgs) * n);
  blk(sizeof(SynArgs) * n);
  for (int s = 0; s + 1 < L; ++s) blk(sizeof(UpsBwdArgs) * n);
  blk(sizeof(CombineArgs) * n);
  blk(sizeof(CombineArgs) * n);
  long long items = 0;
  for (int k = 0; k < n; ++k) {
    const Plan& P = plans[k];
    // the combine launches: reduction and fold blocks, and the loss block
    items += P.arm_grid + P.syn_grid + t0_tiles(P.geo.H, P.geo.W) + P.head_grid + P.red_grid + P.fold_grid0 +
             P.fold_grid1 + 1;
    items += cdiv(P.geo.lh[1], ut) * cdiv(P.geo.lw[1], ut);
    for (int s = 0; s + 1 < L; ++s) items += (long long)P.ups_grid[s] * P.ups_chunks[s];
  }
  blk(sizeof(WorkItem) * items + 256 * (L + 8));
  *total_bytes = cur + d;
  return CC_OK;
}

}  // namespace
}  // namespace cc

struct cc_batch {
  cc::BatchPlan p;
};

extern "C" {

size_t coolchic_batch_workspace_bytes(int32_t n, const cc_problem* probs, const cc_batch_tuning* tune) {
  std::vector<Plan> plans;
  std::vector<size_t> off;
  size_t d = 0, total = 0;
  if (batch_layout(n, probs, tune, plans, off, &d, &total)) return 0;
  return total;
}

int coolchic_batch_create(int32_t n, const cc_problem* probs, const cc_image_io* io, const cc_batch_tuning* tune,
                          float dloss, void* ws, size_t ws_bytes, cc_batch** out) {
  if (!out) return CC_EINVAL;
  *out = nullptr;
  if (!io || !ws) return CC_EINVAL;
  std::vector<Plan> plans;
  std::vector<size_t> img_off;
  size_t desc_off = 0, total = 0;
  int rc = batch_layout(n, probs, tune, plans, img_off, &desc_off, &total);
  if (rc) return rc;
  if (ws_bytes < total) return CC_EWORKSPACE;
  for (int k = 0; k < n; ++k) {
    const cc_image_io& q = io[k];
    if (!q.img || !q.y || !q.arm_w || (!q.ups_w && plans[k].n_ups) || !q.syn_w || !q.loss4 || !q.g_y || !q.g_arm ||
        (!q.g_ups && plans[k].n_ups) || !q.g_syn)
      return CC_EINVAL;
    if (needs_noise(probs[k].quant) && !q.u) return CC_EINVAL;
  }
  const Plan& P0 = plans[0];
  const int L = P0.geo.L;
  BatchPlan B;
  B.n = n;
  B.L = L;
  B.shared = plans[0].shared;
  B.arm_first = tune ? tune->arm_first : 0;
  B.ups_tile = batch_ups_tile(tune);
  B.armk = arm_kernel_for(P0.C, P0.NH, true, true);
  B.t0k = syn_t0_kernel_for(P0.Hs, P0.nres, true);
  B.bwk = syn_bwd_kernel_for(P0.Hs, P0.nres, true);
  B.hdk = syn_head_bwd_kernel_for(P0.Hs, P0.nres, true);
  if (!B.armk || !B.t0k || !B.bwk || !B.hdk) return CC_EUNSUPPORTED;
  if (hipGetDevice(&B.device) != hipSuccess) return CC_EHIP;
  // host copies of every argument block and work-list
  std::vector<ArmArgs> h_arm(n);
  std::vector<UpsFwdArgs> h_upf(n);
  std::vector<SynArgs> h_syn(n);
  std::vector<std::vector<UpsBwdArgs>> h_upb(L, std::vector<UpsBwdArgs>(n));
  std::vector<CombineArgs> h_comb_side(n), h_comb_main(n);
  std::vector<WorkItem> w_arm, w_upf, w_t0, w_syn, w_head, w_comb_side, w_comb_main;
  std::vector<std::vector<WorkItem>> w_upb(L);
  BwdSet* b = new (std::nothrow) BwdSet;
  if (!b) return CC_EINVAL;
  for (int k = 0; k < n; ++k) {
    const cc_image_io& q = io[k];
    const Plan& P = plans[k];
    float* W = (float*)((char*)ws + img_off[k]);
    build_backward(&probs[k], P, W, q.img, q.y, q.u, q.arm_w, q.ups_w, q.syn_w, dloss, q.loss4, q.g_y, q.g_arm,
                   q.g_ups, q.g_syn, b);
    h_arm[k] = b->arm; h_upf[k] = b->upf; h_syn[k] = b->syn;
    h_comb_side[k] = b->comb_side; h_comb_main[k] = b->comb_main;
    for (int s = 0; s + 1 < L; ++s) h_upb[s][k] = b->upb[s];
    for (int i = 0; i < P.arm_grid; ++i) w_arm.push_back(WorkItem{k, i, P.arm_grid, 0});
    // the batched upsampling forward takes tiles of side B.ups_tile
    const int upf = b->upf_grid ? cdiv(P.geo.lh[1], B.ups_tile) * cdiv(P.geo.lw[1], B.ups_tile) : 0;
    for (int i = 0; i < upf; ++i) w_upf.push_back(WorkItem{k, i, upf, 0});
    for (int i = 0; i < b->t0_grid; ++i) w_t0.push_back(WorkItem{k, i, b->t0_grid, 0});
    for (int i = 0; i < P.syn_grid; ++i) w_syn.push_back(WorkItem{k, i, P.syn_grid, 0});
    for (int i = 0; i < P.head_grid; ++i) w_head.push_back(WorkItem{k, i, P.head_grid, 0});
    for (int s = 0; s + 1 < L; ++s)
      for (int c = 0; c < P.ups_chunks[s]; ++c)
        for (int i = 0; i < P.ups_grid[s]; ++i) w_upb[s].push_back(WorkItem{k, i, P.ups_grid[s], c});
    for (int i = 0; i < b->comb_side_grid; ++i) w_comb_side.push_back(WorkItem{k, i, b->comb_side_grid, 0});
    for (int i = 0; i < b->comb_main_grid; ++i) w_comb_main.push_back(WorkItem{k, i, b->comb_main_grid, 0});
  }
  delete b;
  // upload: argument blocks, then work-lists
  char* base = (char*)ws + desc_off;
  size_t d = 0;
  int err = 0;
  auto put = [&](const void* src, size_t bytes) -> void* {
    void* dst = base + d;
    if (bytes && hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) err = 1;
    d += (bytes + 255) / 256 * 256;
    return dst;
  };
  B.d_arm = (ArmArgs*)put(h_arm.data(), sizeof(ArmArgs) * n);
  B.d_upf = (UpsFwdArgs*)put(h_upf.data(), sizeof(UpsFwdArgs) * n);
  B.d_syn = (SynArgs*)put(h_syn.data(), sizeof(SynArgs) * n);
  for (int s = 0; s + 1 < L; ++s) B.d_upb[s] = (UpsBwdArgs*)put(h_upb[s].data(), sizeof(UpsBwdArgs) * n);
  B.d_comb_side = (CombineArgs*)put(h_comb_side.data(), sizeof(CombineArgs) * n);
  B.d_comb_main = (CombineArgs*)put(h_comb_main.data(), sizeof(CombineArgs) * n);
  auto putw = [&](std::vector<WorkItem>& v, WorkItem** dst, int* cnt) {
    *cnt = (int)v.size();
    *dst = (WorkItem*)put(v.data(), sizeof(WorkItem) * v.size());
  };
  putw(w_arm, &B.w_arm, &B.n_arm);
  putw(w_upf, &B.w_upf, &B.n_upf);
  putw(w_t0, &B.w_t0, &B.n_t0);
  putw(w_syn, &B.w_syn, &B.n_syn);
  putw(w_head, &B.w_head, &B.n_head);
  for (int s = 0; s + 1 < L; ++s) putw(w_upb[s], &B.w_upb[s], &B.n_upb[s]);
  putw(w_comb_side, &B.w_comb_side, &B.n_comb_side);
  putw(w_comb_main, &B.w_comb_main, &B.n_comb_main);
  if (err || desc_off + d > ws_bytes) return err ? CC_EHIP : CC_EWORKSPACE;
  cc_batch* h = new (std::nothrow) cc_batch;
  if (!h) return CC_EINVAL;
  h->p = B;
  *out = h;
  return CC_OK;
}

int coolchic_batch_backward(const cc_batch* batch, void* stream) {
  if (!batch) return CC_EINVAL;
  const BatchPlan& B = batch->p;
  hipStream_t st = (hipStream_t)stream;
  int rc, dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return CC_EHIP;
  if (dev != B.device) return CC_EINVAL;  // the plan's buffers live on another device
  auto go = [&](int stage, const void* fn, int grid, int block, void* descs, void* work) -> int {
    if (grid <= 0) return CC_OK;
    void* argv[] = {&descs, &work};
    const bool timed = stage != CC_STAGE_NONE && stage == g_stage && g_ev_begin && g_ev_end;
    if (timed && hipEventRecord(g_ev_begin, st) != hipSuccess) return CC_EHIP;
    if (hipLaunchKernel(fn, dim3(grid), dim3(block), argv, 0, st) != hipSuccess) return CC_EHIP;
    if (timed && hipEventRecord(g_ev_end, st) != hipSuccess) return CC_EHIP;
    return CC_OK;
  };
  Side* sd = nullptr;
  if ((rc = side_for(st, &sd))) return rc;
  std::lock_guard<std::mutex> lock(sd->mu);
  (void)hipGetLastError();
  // the ARM launch goes to the side stream (it depends on nothing the main
  // stream computes): first, after the residual-conv backward, or after the
  // head backward
  auto arm = [&]() -> int {
    int r = fork_to(sd, st);
    if (r) return r;
    void* descs = B.d_arm;
    void* work = B.w_arm;
    void* argv[] = {&descs, &work};
    const bool timed = g_stage == CC_STAGE_ARM && g_ev_begin && g_ev_end;
    if (timed && hipEventRecord(g_ev_begin, sd->stream) != hipSuccess) return CC_EHIP;
    if (hipLaunchKernel(B.armk, dim3(B.n_arm), dim3(ARM_THREADS), argv, 0, sd->stream) != hipSuccess) return CC_EHIP;
    if (timed && hipEventRecord(g_ev_end, sd->stream) != hipSuccess) return CC_EHIP;
    return CC_OK;
  };
  if (B.arm_first == 1 && (rc = arm())) return rc;
  if ((rc = go(CC_STAGE_NONE, ups_fwd_kernel_for(B.shared, true, B.ups_tile), B.n_upf, 256, B.d_upf, B.w_upf))) return rc;
  if ((rc = go(CC_STAGE_NONE, B.t0k, B.n_t0, 256, B.d_syn, B.w_t0))) return rc;
  if ((rc = go(CC_STAGE_SYNTHESIS, B.bwk, B.n_syn, SYN_THREADS, B.d_syn, B.w_syn))) return rc;
  if (B.arm_first == 0 && (rc = arm())) return rc;
  if ((rc = go(CC_STAGE_NONE, B.hdk, B.n_head, 256, B.d_syn, B.w_head))) return rc;
  if (B.arm_first == 2 && (rc = arm())) return rc;
  // the side combine, once levels [0, BATCH_SIDE_LEVELS) of every g_y are
  // final (level 0 after the head backward, level 1 after adjoint step 0)
  auto side_combine = [&]() -> int {
    int r = side_waits(sd, st);
    if (r || B.n_comb_side <= 0) return r;
    void* descs = B.d_comb_side;
    void* work = B.w_comb_side;
    void* argv[] = {&descs, &work};
    return hipLaunchKernel((const void*)combine_kernel_batch, dim3(B.n_comb_side), dim3(256), argv, 0,
                           sd->stream) == hipSuccess ? CC_OK : CC_EHIP;
  };
  if (BATCH_SIDE_LEVELS == 1 && (rc = side_combine())) return rc;
  for (int s = 0; s + 1 < B.L; ++s) {
    if ((rc = go(CC_STAGE_NONE, ups_bwd_kernel_for(B.shared, true), B.n_upb[s], 256, B.d_upb[s], B.w_upb[s])))
      return rc;
    if (s == 0 && BATCH_SIDE_LEVELS == 2 && (rc = side_combine())) return rc;
  }
  if ((rc = join_from(sd, st))) return rc;
  if ((rc = go(CC_STAGE_NONE, (const void*)combine_kernel_batch, B.n_comb_main, 256, B.d_comb_main, B.w_comb_main)))
    return rc;
  return hipGetLastError() == hipSuccess ? CC_OK : CC_EHIP;
}

void coolchic_batch_destroy(cc_batch* batch) { delete batch; }

int coolchic_decode_synth(const cc_problem* p, const float* yq, const float* ups_w, const float* syn_w, float* xhat,
                          void* ws, size_t ws_bytes, void* stream) {
  if (!p) return CC_EINVAL;
  cc_problem q = *p;
  q.quant = CC_QUANT_ROUND;  // shape checks only; latents are used as given
  Plan P;
  int rc = make_plan(&q, CC_WS_DECODE, &P);
  if (rc) return rc;
  if (!yq || (!ups_w && P.n_ups) || !syn_w || !xhat || !ws) return CC_EINVAL;
  if (ws_bytes < P.total * sizeof(float)) return CC_EWORKSPACE;
  const void *t0k = syn_t0_kernel_for(P.Hs, P.nres, false), *resk = syn_res_fwd_kernel_for(P.Hs, P.nres, false);
  if (!t0k || !resk) return CC_EUNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  float* W = (float*)ws;
  (void)hipGetLastError();
  if ((rc = launch_expand(P, W, ups_w, st))) return rc;
  if ((rc = launch_ups_fwd(P, W, yq, nullptr, 2, ups_w, st))) return rc;
  SynArgs sa = syn_args(P, W, yq, nullptr, 2, ups_w, syn_w);
  sa.xhat = xhat;
  if ((rc = launch(t0k, t0_tiles(p->H, p->W), 256, &sa, st))) return rc;
  if ((rc = launch(resk, P.syn_grid, SYN_THREADS, &sa, st))) return rc;
  return hipGetLastError() == hipSuccess ? CC_OK : CC_EHIP;
}

int coolchic_adam_step(float* theta, const float* grad, float* m, float* v, int64_t n, int32_t* step, float lr,
                       float beta1, float beta2, float eps, void* stream) {
  if (!theta || !grad || !m || !v || !step || n <= 0) return CC_EINVAL;
  if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return CC_EINVAL;
  AdamArgs a{theta, grad, m, v, n, step, lr, beta1, beta2, eps};
  const bool vec = ((uintptr_t)theta | (uintptr_t)grad | (uintptr_t)m | (uintptr_t)v) % 16 == 0;
  // one pass of ADAM_U float4 groups per thread where that takes at most
  // 512 blocks (the completion counter takes one atomic per block)
  const int64_t per_block = 256 * 4 * ADAM_U;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + per_block - 1) / per_block, 512));
  (void)hipGetLastError();
  int rc = launch(vec ? (const void*)adam_kernel<true> : (const void*)adam_kernel<false>, grid, 256, &a,
                  (hipStream_t)stream);
  if (rc) return rc;

  return hipGetLastError() == hipSuccess ? CC_OK : CC_EHIP;
}

int coolchic_uniform_noise(float* u, int64_t n, uint64_t seed, const int32_t* step, uint32_t stream_id,
                           void* stream) {
  if (!u || n <= 0) return CC_EINVAL;
  const int64_t groups = (n + 3) / 4;
  const int grid = (int)std::min<int64_t>((groups + 255) / 256, 2048);
  (void)hipGetLastError();
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  void* argv[] = {&u, &n, (void*)&k0, (void*)&k1, &step, &stream_id};
  if (hipLaunchKernel((const void*)noise_kernel, dim3(grid), dim3(256), argv, 0, (hipStream_t)stream) != hipSuccess)
    return CC_EHIP;
  return hipGetLastError() == hipSuccess ? CC_OK : CC_EHIP;
}

int coolchic_stream_prepare(void* stream) {
  Side* sd = nullptr;
  return side_for((hipStream_t)stream, &sd);
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

int coolchic_timing_event_create(void** ev) {
  if (!ev) return CC_EINVAL;
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return CC_EHIP;
  *ev = (void*)e;
  return CC_OK;
}

int coolchic_timing_event_elapsed(void* ev_begin, void* ev_end, float* ms) {
  if (!ev_begin || !ev_end || !ms) return CC_EINVAL;
  return hipEventElapsedTime(ms, (hipEvent_t)ev_begin, (hipEvent_t)ev_end) == hipSuccess ? CC_OK : CC_EHIP;
}

int coolchic_timing_event_destroy(void* ev) {
  if (!ev) return CC_EINVAL;
  return hipEventDestroy((hipEvent_t)ev) == hipSuccess ? CC_OK : CC_EHIP;
}

}  // extern "C"

// ---------------------------------------------------------------- parameter quantisation

extern "C" int coolchic_param_quantize(const cc_arch* arch, const float* arm_w, const float* ups_w,
                                       const float* syn_w, const int32_t* step_log2, float* arm_q, float* ups_q,
                                       float* syn_q, float* bits, void* stream) {
  if (!arch || !step_log2 || !bits) return CC_EINVAL;
  if (!arch_ok(arch)) return CC_EUNSUPPORTED;
  int64_t na = 0, nu = 0, ns = 0;
  counts(arch, &na, &nu, &ns);
  if (!arm_w || !arm_q || !syn_w || !syn_q || (nu && (!ups_w || !ups_q))) return CC_EINVAL;
  ParamQArgs a;
  std::memset(&a, 0, sizeof(a));
  const float* src[3] = {arm_w, ups_w, syn_w};
  float* dst[3] = {arm_q, ups_q, syn_q};
  const int64_t n[3] = {na, nu, ns};
  for (int m = 0; m < 3; ++m) {
    if (step_log2[m] < 0 || step_log2[m] > 24) return CC_EINVAL;
    a.src[m] = src[m];
    a.dst[m] = dst[m];
    a.n[m] = (int)n[m];
    a.k[m] = step_log2[m];
  }
  a.bits = bits;
  (void)hipGetLastError();
  void* argv[] = {&a};
  if (hipLaunchKernel((const void*)param_quant_kernel, dim3(3), dim3(256), argv, 0, (hipStream_t)stream) !=
      hipSuccess)
    return CC_EHIP;
  return hipGetLastError() == hipSuccess ? CC_OK : CC_EHIP;
}

// ---------------------------------------------------------------- entropy coding

namespace cc {
namespace {

struct CodecPlan {
  CodecArgs a;
  size_t off_cum, off_cum16, off_meta, off_tbl, off_dsym, off_emit[CD_MAX_SETS], total;  // bytes
  int64_t bound;
  int threads;
  size_t lds;
};

size_t take_bytes(size_t& cur, size_t n) {
  const size_t at = cur;
  cur += (n + 255) / 256 * 256;
  return at;
}

int codec_plan(const cc_problem* p, CodecPlan* cp) {
  Plan P;
  int rc = make_plan(p, CC_WS_FORWARD, &P);
  if (rc) return rc;
  if (p->H > CD_MAX_ROWS) return CC_EUNSUPPORTED;
  std::memset(cp, 0, sizeof(*cp));
  CodecArgs& a = cp->a;
  a.geo = P.geo;
  a.C = P.C;
  a.NH = P.NH;
  a.slope = P.C == 8 ? 2 : (P.C == 16 ? 3 : 4);
  const int L = P.geo.L;
  a.n_sets = L > 1 ? 2 : 1;
  a.set[0] = CodecSet{std::min(CD_LANES, P.geo.lh[0]), 0, 1};
  if (L > 1) a.set[1] = CodecSet{std::min(CD_LANES, P.geo.lh[1]), 1, L};
  a.rows_max = P.geo.lh[0];
  size_t cur = 0;
  cp->off_cum = take_bytes(cur, sizeof(uint32_t) * CD_NSCALE * CD_NMU * CD_ROW);
  cp->off_cum16 = take_bytes(cur, sizeof(uint16_t) * CD_NSCALE * CD_NMU * CD_ROW16);
  cp->off_meta = take_bytes(cur, sizeof(uint32_t) * CD_META_N);
  cp->off_tbl = take_bytes(cur, sizeof(uint16_t) * (size_t)P.geo.n_lat);
  cp->off_dsym = take_bytes(cur, sizeof(int32_t) * (size_t)P.geo.n_lat);
  int lanes = 0;
  for (int s = 0; s < a.n_sets; ++s) {
    const CodecSet& S = a.set[s];
    const int64_t nl = (int64_t)P.geo.loff[S.lv1] - P.geo.loff[S.lv0];
    a.emit_cap[s] = nl * CD_BYTES_PER_LATENT;
    cp->off_emit[s] = take_bytes(cur, (size_t)a.emit_cap[s]);
    lanes += S.n_lanes;
  }
  cp->total = cur;
  cp->bound = 8 + 4 * (int64_t)a.n_sets + 4 * (int64_t)lanes + (int64_t)CD_BYTES_PER_LATENT * P.geo.n_lat;
  cp->threads = 512;  // 8 waves: one 32-row slice each per chunk of CD_SLOTS rows
  cp->lds = codec_decode_lds_bytes(a.rows_max, (int)P.n_arm);
  return CC_OK;
}

void codec_bind(CodecPlan* cp, void* ws) {
  uint8_t* b = (uint8_t*)ws;
  CodecArgs& a = cp->a;
  a.cum = (uint32_t*)(b + cp->off_cum);
  a.cum16 = (uint16_t*)(b + cp->off_cum16);
  a.meta = (uint32_t*)(b + cp->off_meta);
  a.tbl = (uint16_t*)(b + cp->off_tbl);
  a.dsym = (int32_t*)(b + cp->off_dsym);
  for (int s = 0; s < a.n_sets; ++s) a.emit[s] = b + cp->off_emit[s];
}

constexpr int CD_TABLE_ROWS = CD_NSCALE * CD_NMU;

int launch_table(uint32_t* cum, uint16_t* cum16, uint32_t* meta, hipStream_t st) {
  void* argv[] = {&cum, &cum16, &meta};
  return hipLaunchKernel((const void*)codec_table_kernel, dim3((CD_TABLE_ROWS + 63) / 64), dim3(64), argv, 0, st) ==
                 hipSuccess
             ? CC_OK
             : CC_EHIP;
}

}  // namespace
}  // namespace cc

extern "C" {

size_t coolchic_entropy_workspace_bytes(const cc_problem* p) {
  CodecPlan cp;
  return codec_plan(p, &cp) ? 0 : cp.total;
}

int64_t coolchic_entropy_bound(const cc_problem* p) {
  CodecPlan cp;
  return codec_plan(p, &cp) ? -1 : cp.bound;
}

int coolchic_entropy_tables(uint32_t* cum, void* stream) {
  if (!cum) return CC_EINVAL;
  (void)hipGetLastError();
  const int rc = launch_table(cum, nullptr, nullptr, (hipStream_t)stream);
  if (rc) return rc;
  return hipGetLastError() == hipSuccess ? CC_OK : CC_EHIP;
}

int coolchic_entropy_encode(const cc_problem* p, const float* yq, const float* arm_w, uint8_t* out,
                            size_t out_capacity, int64_t* out_nbytes, void* ws, size_t ws_bytes, void* stream) {
  CodecPlan cp;
  int rc = codec_plan(p, &cp);
  if (rc) return rc;
  if (!yq || !arm_w || !out || !out_nbytes || !ws) return CC_EINVAL;
  if (ws_bytes < cp.total) return CC_EWORKSPACE;
  const void* prk = codec_params_kernel_for(cp.a.C);
  if (!prk) return CC_EUNSUPPORTED;
  codec_bind(&cp, ws);
  CodecArgs& a = cp.a;
  a.yq = yq;
  a.w = arm_w;
  a.out = out;
  a.out_cap = (int64_t)std::min<size_t>(out_capacity, (size_t)INT64_MAX);
  a.out_nbytes = out_nbytes;
  hipStream_t st = (hipStream_t)stream;
  (void)hipGetLastError();
  if ((rc = launch_table(a.cum, nullptr, a.meta, st))) return rc;
  if ((rc = launch(prk, cdiv(a.geo.n_lat, 128), 256, &a, st))) return rc;  // 32 latents per wave
  {
    void* argv[] = {&a};
    if (hipLaunchKernel((const void*)codec_encode_kernel, dim3(a.n_sets), dim3(64), argv, 0, st) != hipSuccess)
      return CC_EHIP;
  }
  const int pack_grid = (int)std::min<int64_t>(2048, (cp.bound + 255) / 256);
  if ((rc = launch((const void*)codec_pack_kernel, pack_grid, 256, &a, st))) return rc;
  return hipGetLastError() == hipSuccess ? CC_OK : CC_EHIP;
}

int coolchic_entropy_decode(const cc_problem* p, const uint8_t* in, size_t in_bytes, const float* arm_w,
                            float* yq_out, int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  CodecPlan cp;
  int rc = codec_plan(p, &cp);
  if (rc) return rc;
  if (!in || !arm_w || !yq_out || !status || !ws || ((uintptr_t)in & 3u)) return CC_EINVAL;
  if (ws_bytes < cp.total) return CC_EWORKSPACE;
  const void* dk = codec_decode_kernel_for(cp.a.C);
  if (!dk) return CC_EUNSUPPORTED;
  codec_bind(&cp, ws);
  CodecArgs& a = cp.a;
  a.w = arm_w;
  a.in = in;
  a.in_bytes = (int64_t)std::min<size_t>(in_bytes, (size_t)INT64_MAX);
  a.yq_out = yq_out;
  a.status = status;
  hipStream_t st = (hipStream_t)stream;
  (void)hipGetLastError();
  if (cp.lds > 64 * 1024 &&
      hipFuncSetAttribute(dk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cp.lds) != hipSuccess)
    return CC_EHIP;
  if ((rc = launch_table(a.cum, a.cum16, nullptr, st))) return rc;
  void* argv[] = {&a};
  if (hipLaunchKernel(dk, dim3(a.n_sets), dim3(cp.threads), argv, cp.lds, st) != hipSuccess) return CC_EHIP;
  return hipGetLastError() == hipSuccess ? CC_OK : CC_EHIP;
}

const char* coolchic_strerror(int code) {
  switch (code) {
    case CC_OK: return "ok";
    case CC_EINVAL: return "invalid argument (null pointer, size, or H/W not a multiple of 2^(L-1))";
    case CC_EUNSUPPORTED: return "architecture not supported by the compiled kernels";
    case CC_EWORKSPACE: return "workspace smaller than coolchic_workspace_bytes()";
    case CC_EHIP: return "HIP kernel launch failed";
    case CC_ESCRATCH: return "problem needs more workspace than the static scratch of coolchic_train_step_noalloc "
                             "(CC_NOALLOC_SCRATCH_BYTES)";
  }
  return "unknown error code";
}

}  // extern "C"

// ---------------------------------------------------------------- warm start

namespace cc {
namespace {

struct WarmPlan {
  WarmArgs a;
  int g_prep, g_conv[5], g_heads, g_df4, g_bd[5], g_h0, g_bw[5], g_comb;
  size_t total;  // floats
  CombineArgs comb;
  FinalArgs fin;
};

int warm_check(const cc_warm_problem* p) {
  if (!p) return CC_EINVAL;
  if (p->H <= 0 || p->W <= 0 || p->H % 64 || p->W % 64 || p->H > 8192 || p->W > 8192) return CC_EINVAL;
  if (p->batch < 1 || p->batch > 4096) return CC_EINVAL;
  if (!arch_ok(&p->arch)) return CC_EUNSUPPORTED;
  if (p->arch.n_levels != 7) return CC_EUNSUPPORTED;
  // every index of the batch's latents and feature maps fits in 32 bits
  if ((int64_t)p->batch * p->H * p->W * 8 >= ((int64_t)1 << 31)) return CC_EINVAL;
  return CC_OK;
}

int64_t warm_param_count(int64_t n_theta) {
  int64_t n = 0;
  for (int k = 1; k <= 4; ++k) n += WS_CH * 9 * (k == 1 ? 3 : WS_CH) + WS_CH;
  return n + 60 + 6 * 33 + 33 * n_theta;
}

// Offsets (and, with a workspace base, pointers) of every buffer.
int warm_plan(const cc_warm_problem* p, int which, WarmPlan* P, float* base) {
  int rc = warm_check(p);
  if (rc) return rc;
  if (which != CC_WS_FORWARD && which != CC_WS_BACKWARD) return CC_EINVAL;
  std::memset(P, 0, sizeof(*P));
  WarmArgs& a = P->a;
  int64_t na, nu, ns;
  counts(&p->arch, &na, &nu, &ns);
  a.B = p->batch; a.H = p->H; a.W = p->W;
  a.n_theta = (int)(na + nu + ns);
  if (a.n_theta > WS_MAX_THETA) return CC_EUNSUPPORTED;
  for (int k = 0; k <= 4; ++k) { a.h[k] = p->H >> k; a.w[k] = p->W >> k; }
  int off = 0;
  for (int l = 0; l < 7; ++l) {
    a.lh[l] = p->H >> l; a.lw[l] = p->W >> l; a.loff[l] = off;
    off += a.lh[l] * a.lw[l];
  }
  a.loff[7] = off;
  a.n_lat = off;
  int o = 0;
  for (int k = 1; k <= 4; ++k) {
    a.conv_off[k] = o;
    o += WS_CH * 9 * (k == 1 ? 3 : WS_CH) + WS_CH;
  }
  a.head_off[0] = o;
  for (int l = 1; l < 7; ++l) a.head_off[l] = o + 60 + 33 * (l - 1);
  a.ptheta = a.head_off[6] + 33;
  a.n_net = a.ptheta + 33 * a.n_theta;
  const int B = a.B;
  a.sy = 2.0f / ((float)a.n_lat * B);
  a.sth = 2.0f / ((float)a.n_theta * B);
  // grids
  P->g_prep = std::min(cdiv(a.n_net + 5 * WS_CH, 256), 1024);
  for (int k = 1; k <= 4; ++k) {
    const int64_t tiles = (int64_t)B * a.h[k] * cdiv(a.w[k], 32);
    P->g_conv[k] = (int)std::min<int64_t>((tiles + 3) / 4, 2048);
    const int64_t chunks = ((int64_t)B * a.h[k] * a.w[k] + 15) / 16;
    P->g_bw[k] = (int)std::max<int64_t>(1, std::min<int64_t>(256, (chunks + 15) / 16));
  }
  P->g_heads = (int)std::min<int64_t>(((int64_t)B * a.n_lat + 255) / 256, 2048);
  P->g_df4 = cdiv(B * a.h[4] * a.w[4], WS_DF4_POS);
  for (int k = 2; k <= 4; ++k) {
    const int64_t tiles = (int64_t)B * a.h[k - 1] * 2 * cdiv(a.w[k - 1] / 2, 32);
    P->g_bd[k] = (int)std::min<int64_t>((tiles + 3) / 4, 2048);
  }
  P->g_h0 = (int)std::min<int64_t>(((int64_t)B * p->H * p->W + 255) / 256, 1024);
  // buffers (sizes in floats; bfloat16 arrays take half a float per value)
  size_t cur = 0;
  auto put = [&](size_t nfl) -> float* {
    const size_t at = take(cur, nfl);
    return base ? base + at : nullptr;
  };
  auto put16 = [&](size_t n16) -> uint16_t* { return (uint16_t*)put((n16 + 1) / 2); };
  a.net_r = put(a.n_net);
  a.wf[1] = put16(WS_CH * 32);
  for (int k = 2; k <= 4; ++k) a.wf[k] = put16(WS_CH * 9 * WS_CH);
  for (int k = 1; k <= 4; ++k) a.f[k] = put16((size_t)B * a.h[k] * a.w[k] * WS_CH);
  a.gap = put((size_t)B * WS_CH);
  if (which == CC_WS_BACKWARD) {
    for (int k = 2; k <= 4; ++k) a.wt[k] = put16(9 * WS_CH * WS_CH);
    for (int k = 1; k <= 4; ++k) a.dp[k] = put16((size_t)B * a.h[k] * a.w[k] * WS_CH);
    a.y = put((size_t)B * a.n_lat);
    a.theta = put((size_t)B * a.n_theta);
    a.dgap = put((size_t)B * WS_CH);
    a.lpart_y = put(P->g_heads);
    a.lpart_th = put(B);
    for (int k = 1; k <= 4; ++k)
      a.part_conv[k] = put((size_t)P->g_bw[k] * (WS_CH * 9 * (k == 1 ? 3 : WS_CH) + WS_CH));
    a.part_h456 = put((size_t)P->g_df4 * 99);
    for (int l = 1; l <= 3; ++l) a.part_h[l] = put((size_t)P->g_bd[l + 1] * 33);
    a.part_v0 = put((size_t)P->g_bd[2] * 32);
    a.part_h0 = put((size_t)P->g_h0 * 28);
    a.part_th = put((size_t)B * 33 * a.n_theta);
    // column sums of every partial block into the gradient, in layout order
    CombineArgs& ca = P->comb;
    std::memset(&ca, 0, sizeof(ca));
    ca.loss_block = -1;
    int nsg = 0, blk = 0;
    auto seg = [&](const float* src, int rows, int cols, int dst_off) {
      ca.seg[nsg] = RedSeg{src, rows, cols, cols, 16, (float*)(intptr_t)dst_off};
      ca.block_start[nsg] = blk;
      blk += cdiv(cols, 16);
      ++nsg;
    };
    for (int k = 1; k <= 4; ++k)
      seg(a.part_conv[k], P->g_bw[k], WS_CH * 9 * (k == 1 ? 3 : WS_CH) + WS_CH, a.conv_off[k]);
    seg(a.part_v0, P->g_bd[2], 32, a.head_off[0]);
    seg(a.part_h0, P->g_h0, 28, a.head_off[0] + 32);
    for (int l = 1; l <= 3; ++l) seg(a.part_h[l], P->g_bd[l + 1], 33, a.head_off[l]);
    seg(a.part_h456, P->g_df4, 99, a.head_off[4]);
    seg(a.part_th, B, 33 * a.n_theta, a.ptheta);
    ca.nseg = nsg;
    ca.block_start[nsg] = blk;
    P->g_comb = blk;
    ca.flags = put(blk);
    FinalArgs& fa = P->fin;
    fa.spart = a.lpart_y; fa.ns = P->g_heads;
    fa.rpart = a.lpart_th; fa.nr = B;
    fa.flags = ca.flags; fa.nflags = blk;
    fa.lambda = 1.0f; fa.inv_hw = 1.0f; fa.inv_3hw = 1.0f;
    fa.have_rate = 1; fa.have_sse = 1;
  }
  P->total = cur;
  return CC_OK;
}

int warm_forward_launches(WarmPlan& P, hipStream_t st, int bwd) {
  int rc;
  WarmArgs& a = P.a;
  if ((rc = launch((const void*)warm_prep_kernel, P.g_prep, 256, &a, st))) return rc;
  for (int k = 1; k <= 4; ++k) {
    void* argv[] = {&a, &k};
    if (hipLaunchKernel(warm_conv_fwd_kernel_for(k), dim3(P.g_conv[k]), dim3(256), argv, 0, st) != hipSuccess)
      return CC_EHIP;
  }
  {
    void* argv[] = {&a, &bwd};
    if (hipLaunchKernel((const void*)warm_heads_fwd_kernel, dim3(P.g_heads), dim3(256), argv, 0, st) != hipSuccess)
      return CC_EHIP;
    if (hipLaunchKernel((const void*)warm_theta_kernel, dim3(a.B), dim3(256), argv, 0, st) != hipSuccess)
      return CC_EHIP;
  }
  return CC_OK;
}

}  // namespace
}  // namespace cc

extern "C" {

int64_t coolchic_warm_param_count(const cc_arch* arch) {
  if (!arch_ok(arch)) return -1;
  int64_t na, nu, ns;
  counts(arch, &na, &nu, &ns);
  if (na + nu + ns > WS_MAX_THETA) return -1;
  return warm_param_count(na + nu + ns);
}

size_t coolchic_warm_workspace_bytes(const cc_warm_problem* p, int which) {
  WarmPlan P;
  if (warm_plan(p, which, &P, nullptr)) return 0;
  return P.total * sizeof(float);
}

int coolchic_warm_forward(const cc_warm_problem* p, const float* x, const float* net, float* y_out, float* theta_out,
                          void* ws, size_t ws_bytes, void* stream) {
  static thread_local WarmPlan P;
  int rc = warm_plan(p, CC_WS_FORWARD, &P, nullptr);
  if (rc) return rc;
  if (!x || !net || !y_out || !theta_out || !ws) return CC_EINVAL;
  if (ws_bytes < P.total * sizeof(float)) return CC_EWORKSPACE;
  warm_plan(p, CC_WS_FORWARD, &P, (float*)ws);
  P.a.x = x; P.a.net = net; P.a.y = y_out; P.a.theta = theta_out;
  P.a.f[0] = nullptr;
  (void)hipGetLastError();
  if ((rc = warm_forward_launches(P, (hipStream_t)stream, 0))) return rc;
  return hipGetLastError() == hipSuccess ? CC_OK : CC_EHIP;
}

}  // extern "C"

namespace cc {
namespace {

int warm_backward_impl(const cc_warm_problem* p, const float* x, const float* net, const float* y_target,
                       const float* theta_target, const float* g_y, const float* g_theta, float* loss4, float* g_net,
                       void* ws, size_t ws_bytes, void* stream) {
  static thread_local WarmPlan P;
  int rc = warm_plan(p, CC_WS_BACKWARD, &P, nullptr);
  if (rc) return rc;
  const bool regress = y_target && theta_target, given = g_y && g_theta;
  if (!x || !net || regress == given || !loss4 || !g_net || !ws) return CC_EINVAL;
  if (ws_bytes < P.total * sizeof(float)) return CC_EWORKSPACE;
  warm_plan(p, CC_WS_BACKWARD, &P, (float*)ws);
  WarmArgs& a = P.a;
  a.x = x; a.net = net; a.y_t = y_target; a.th_t = theta_target; a.gy_in = g_y; a.gth_in = g_theta;
  for (int s = 0; s < P.comb.nseg; ++s) P.comb.seg[s].dst = g_net + (intptr_t)P.comb.seg[s].dst;
  P.fin.loss4 = loss4;
  hipStream_t st = (hipStream_t)stream;
  (void)hipGetLastError();
  if ((rc = warm_forward_launches(P, st, 1))) return rc;
  if ((rc = launch((const void*)warm_df4_kernel, P.g_df4, 256, &a, st))) return rc;
  for (int k = 4; k >= 2; --k) {
    void* argv[] = {&a, &k};
    if (hipLaunchKernel((const void*)warm_bwd_data_kernel, dim3(P.g_bd[k]), dim3(256), argv, 0, st) != hipSuccess)
      return CC_EHIP;
  }
  if ((rc = launch((const void*)warm_head0_grad_kernel, P.g_h0, 256, &a, st))) return rc;
  for (int k = 1; k <= 4; ++k) {
    void* argv[] = {&a, &k};
    if (hipLaunchKernel(warm_bwd_weight_kernel_for(k), dim3(P.g_bw[k]), dim3(256), argv, 0, st) != hipSuccess)
      return CC_EHIP;
  }
  if ((rc = launch((const void*)combine_kernel, P.g_comb, 256, &P.comb, st))) return rc;
  if ((rc = launch((const void*)finalize_kernel, 1, 256, &P.fin, st))) return rc;
  return hipGetLastError() == hipSuccess ? CC_OK : CC_EHIP;
}

}  // namespace
}  // namespace cc

extern "C" {

int coolchic_warm_backward(const cc_warm_problem* p, const float* x, const float* net, const float* y_target,
                           const float* theta_target, float* loss4, float* g_net, void* ws, size_t ws_bytes,
                           void* stream) {
  if (!y_target || !theta_target) return CC_EINVAL;
  return warm_backward_impl(p, x, net, y_target, theta_target, nullptr, nullptr, loss4, g_net, ws, ws_bytes,
                            stream);
}

int coolchic_warm_backward_grad(const cc_warm_problem* p, const float* x, const float* net, const float* g_y,
                                const float* g_theta, float* loss4, float* g_net, void* ws, size_t ws_bytes,
                                void* stream) {
  if (!g_y || !g_theta) return CC_EINVAL;
  return warm_backward_impl(p, x, net, nullptr, nullptr, g_y, g_theta, loss4, g_net, ws, ws_bytes, stream);
}

}  // extern "C"

/*
 * coolchic.h -- C ABI of the MI355X (gfx950) Cool-chic rate-distortion pass.
 *
 * The library computes, for one image, the loss of Eq. (1) of "Overfitted
 * image coding at reduced complexity" (Blard et al.):
 *
 *     loss = D(x, x_hat) + lambda * R(y_hat) / (H * W)
 *
 * with x the image, y_hat = Q(y) the quantised latent pyramid (Section II,
 * "Decoding" and "Encoding"), R = sum over latents of -log2 p_psi(y_hat) in bits
 * (the ARM probability model, a Laplace distribution whose mean and log-scale
 * the ARM MLP outputs, scale clamped to [0.01, 100], mass taken over
 * [y_hat - 1/2, y_hat + 1/2]), D the mean over 3*H*W of the squared error, and
 * x_hat = f_theta(f_upsilon(y_hat)) (upsampling, then synthesis; Table I layer
 * types), together with its exact gradient w.r.t. y and every parameter
 * (Section IV-A: one training iteration is one forward plus one backward).
 *
 * Conventions for every entry point:
 *  - All float pointers are DEVICE pointers (HIP global memory) owned by the
 *    caller; the library keeps none of them after the call returns.  Calls are
 *    asynchronous: they only enqueue kernels on `stream` (a hipStream_t, NULL
 *    for the default stream) and return; nothing is allocated and the host is
 *    never synchronised, so a call can be captured into a HIP graph.
 *  - `ws` is a caller-owned device workspace of at least
 *    coolchic_workspace_bytes() bytes; its contents need not be initialised and
 *    are clobbered.  Two calls that overlap in time must not share `ws`.
 *  - Return value: CC_OK (0) or a negative CC_E* code; on error nothing has
 *    been enqueued (except CC_EHIP, which reports a failed launch).
 *  - Non-finite values do not fail a call: the kernels set loss4[3] to 1.0f
 *    when any loss term or gradient is NaN or infinite (0.0f otherwise).
 *
 * Layouts (all float32):
 *  - image x: planar [3][H][W], values in [0, 1].
 *  - latent pyramid (y, u, g_y, rate_map, yq_out): one buffer, level-major; level
 *    l (0 <= l < L) is row-major [H >> l][W >> l] starting at offset
 *    sum_{m < l} (H >> m) * (W >> m).
 *  - ARM parameters psi: for each hidden residual layer j: W_j [C][C] (out, in)
 *    then b_j [C]; then W_o [2][C] (row 0 = mean, row 1 = log-scale), b_o [2].
 *  - upsampling parameters upsilon: separable, [L-1][2][K]; index s produces
 *    level s from level s+1; [s][0] are the vertical taps, [s][1] the
 *    horizontal taps.  Shared: [K][K] (ky, kx), used by every step.  Output
 *    row i of a step takes tap ky from input row (i + K/2 - 1 - ky) / 2 when
 *    that is an integer, the input index clamped to the grid.
 *  - synthesis parameters theta: W1 [Hs][L], b1 [Hs], W2 [3][Hs], b2 [3]; then
 *    for each residual 3x3 conv r: W_r [3][3][3][3] (out, in, ky, kx), b_r [3].
 */
#ifndef COOLCHIC_H
#define COOLCHIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Decoder architecture (Table I notation). */
typedef struct {
  int32_t n_levels;   /* L, number of latent grids, 1..7 (1: no upsampling, no
                         upsampling parameters; ups_w and g_ups may be NULL) */
  int32_t arm_ctx;    /* C, causal neighbours fed to the ARM: 8, 16 or 24 (Table I
                         widths); the C nearest causal positions of a 7x7
                         window, ties in raster order, zero outside the grid */
  int32_t arm_layers; /* hidden C-C-LinR layers before the C-2-Lin output, 1..3 */
  int32_t ups_taps;   /* K of the stride-2 transposed convs: 4 or 8 (the batched
                         entry points: 8 only) */
  int32_t syn_hidden; /* width of the first 1x1 synthesis layer, 8..48, multiple of 8 */
  int32_t syn_res;    /* number of residual 3x3 convs 3->3 (ConvR-3), 1..2 */
  int32_t ups_shared; /* 0: each upsampling step has its own separable kernel
                         (vertical and horizontal K-tap filters); 1: one
                         non-separable K x K kernel shared by every step
                         (Table I "1-1-TConv-K") */
} cc_arch;

/* Quantisation proxy Q (Section II "Encoding"): rounding to nearest (ties to
   even) with a straight-through gradient; additive noise y + u with u in
   [-1/2, 1/2) supplied by the caller (identity gradient); or the proxy of C3
   that Section II cites, y_hat = s(s(y) + u) with s the soft rounding
   s(x) = floor(x) + 1/2 + tanh(a r) / (2 tanh(a/2)), r = x - floor(x) - 1/2
   (Agustsson & Theis 2020), gradient s'(s(y) + u) s'(y).  For
   CC_QUANT_SOFT the noise buffer u holds N_lat + 1 floats: the noise, then
   the sharpness a > 0 (read on the device, so a captured graph can anneal
   it). */
enum { CC_QUANT_ROUND = 0, CC_QUANT_NOISE = 1, CC_QUANT_SOFT = 2 };

typedef struct {
  int32_t H, W;     /* image rows and columns; both multiples of 2^(L-1) */
  cc_arch arch;
  int32_t quant;    /* CC_QUANT_ROUND, CC_QUANT_NOISE or CC_QUANT_SOFT */
  float lambda;     /* rate weight of Eq. (1) */
} cc_problem;

enum {
  CC_OK = 0,
  CC_EINVAL = -1,       /* null pointer, bad size, H/W not multiples of 2^(L-1) */
  CC_EUNSUPPORTED = -2, /* architecture outside the compiled variants */
  CC_EWORKSPACE = -3,   /* ws_bytes smaller than coolchic_workspace_bytes() */
  CC_EHIP = -4,         /* a kernel launch failed (hipGetLastError) */
  CC_ESCRATCH = -5      /* coolchic_train_step_noalloc: the problem's workspace
                           exceeds CC_NOALLOC_SCRATCH_BYTES */
};

enum { CC_WS_FORWARD = 0, CC_WS_BACKWARD = 1, CC_WS_DECODE = 2 };

/* Number of parameters of each module; returns the total, or -1 for an
   invalid architecture.  Output pointers are host pointers and may be NULL. */
int64_t coolchic_param_count(const cc_arch* arch, int64_t* n_arm, int64_t* n_ups, int64_t* n_syn);

/* Number of latents sum_l (H >> l) * (W >> l), or -1 if invalid. */
int64_t coolchic_latent_count(const cc_problem* p);

/* Device workspace bytes needed by coolchic_forward (which = CC_WS_FORWARD),
   coolchic_backward (CC_WS_BACKWARD) or coolchic_decode_synth (CC_WS_DECODE);
   0 if the problem is invalid. */
size_t coolchic_workspace_bytes(const cc_problem* p, int which);

/* Forward pass: Eq. (1) for one image.
   img [3][H][W]; y [N_lat]; u [N_lat] (required for CC_QUANT_NOISE, ignored
   otherwise, may be NULL); arm_w, ups_w, syn_w the packed parameters.
   Outputs: loss4 [4] = {loss, D, R (bits), non-finite flag}; optional (NULL to
   skip) rate_map [N_lat] per-latent rate in bits, yq_out [N_lat] quantised
   latents, xhat_out [3][H][W] synthesised image (not clamped). */
int coolchic_forward(const cc_problem* p, const float* img, const float* y, const float* u,
                     const float* arm_w, const float* ups_w, const float* syn_w,
                     float* loss4, float* rate_map, float* yq_out, float* xhat_out,
                     void* ws, size_t ws_bytes, void* stream);

/* Forward and backward (adjoint) pass: writes loss4 exactly as
   coolchic_forward does, and the gradient of dloss * loss w.r.t. y (g_y
   [N_lat]; the quantiser's gradient is the identity in both modes) and w.r.t.
   each parameter block (g_arm, g_ups, g_syn, laid out like the parameters).
   Gradients are overwritten, not accumulated.  The result is deterministic:
   repeated calls give bit-identical outputs. */
int coolchic_backward(const cc_problem* p, const float* img, const float* y, const float* u,
                      const float* arm_w, const float* ups_w, const float* syn_w, float dloss,
                      float* loss4, float* g_y, float* g_arm, float* g_ups, float* g_syn,
                      void* ws, size_t ws_bytes, void* stream);

/* One training iteration: coolchic_backward, then one coolchic_adam_step
   with the same arguments, on the packed vectors theta = [y | arm_w | ups_w |
   syn_w] (N_lat + n_arm + n_ups + n_syn floats), with grad, m and v laid
   out alike.  The Adam updates run inside the gradient reductions (each
   parameter once its gradient is final and nothing of the pass reads it any
   more), so there is no separate optimiser launch; theta, grad, m, v, step
   and loss4 end up bit-identical to the two separate calls (loss4 and grad
   are those of the parameters before the update).  u, dloss, ws, ws_bytes
   as for coolchic_backward (workspace CC_WS_BACKWARD); step, lr, beta1,
   beta2, eps as for coolchic_adam_step.  theta must not alias img or u. */
int coolchic_train_step(const cc_problem* p, const float* img, const float* u, float dloss, float* loss4,
                        float* theta, float* grad, float* m, float* v, int32_t* step, float lr, float beta1,
                        float beta2, float eps, void* ws, size_t ws_bytes, void* stream);

/* Size of the library's static device scratch used by
   coolchic_train_step_noalloc (64 MiB per device, held until the process
   ends): enough for the backward workspace of a 768x512 image with the
   largest compiled decoder (about 32 MiB) and of images up to about one
   megapixel. */
#define CC_NOALLOC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc):
   coolchic_train_step with its workspace taken from a static device array
   of CC_NOALLOC_SCRATCH_BYTES that the library owns, instead of a caller's
   ws.  Same arguments (minus ws, ws_bytes), same results, bit for bit.
   Calls no hipMalloc / hipFree and creates no stream or event: every kernel
   runs on `stream` in dependency order (so it is slower than
   coolchic_train_step, which overlaps the ARM on a side stream).  The first
   call on a device, with that device current, looks up the array's device
   address (hipGetSymbolAddress), once.
   Errors: CC_ESCRATCH (nothing enqueued) when coolchic_workspace_bytes(p,
   CC_WS_BACKWARD) exceeds CC_NOALLOC_SCRATCH_BYTES; otherwise as
   coolchic_train_step.  Every call on one device shares that device's
   array, which keeps the last call's contents (the pass overwrites every
   region it reads, so nothing needs clearing): calls that overlap in time
   on one device (concurrent streams or threads) race and give wrong
   results; serialise them. */
int coolchic_train_step_noalloc(const cc_problem* p, const float* img, const float* u, float dloss, float* loss4,
                                float* theta, float* grad, float* m, float* v, int32_t* step, float lr, float beta1,
                                float beta2, float eps, void* stream);

/* Decoder-side parallel work once the latents are known (Section II
   "Decoding", upsampling then synthesis): yq [N_lat] integer-valued latents
   (used as given), xhat [3][H][W] output, not clamped.  p->quant and
   p->lambda are ignored. */
int coolchic_decode_synth(const cc_problem* p, const float* yq, const float* ups_w, const float* syn_w,
                          float* xhat, void* ws, size_t ws_bytes, void* stream);

/* One Adam step (Kingma & Ba; the optimiser the paper trains with) on n
   parameters: m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2, theta <- theta -
   lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps) with t = step[0] + 1.
   step points to two device int32: step[0] is the number of steps already
   taken, which the call advances on the device (so a captured graph can be
   replayed); step[1] is the call's completion counter, 0 before the first
   call and left at 0.  theta, grad, m, v: device arrays of n floats. */
int coolchic_adam_step(float* theta, const float* grad, float* m, float* v, int64_t n,
                       int32_t* step, float lr, float beta1, float beta2, float eps, void* stream);

/* Streams.  coolchic_forward, coolchic_backward, coolchic_train_step and
   coolchic_batch_backward fork the ARM kernel onto a side stream and join it
   back with events.  The library keeps one side stream and event set per
   (device, caller stream), created on the first call on that stream with the
   device current, so calls on different streams run concurrently; calls on
   one stream from several threads are serialised while they enqueue.  A
   stream being captured into a graph that has no set of its own uses one the
   device already has.  coolchic_stream_prepare creates the set for `stream`
   on the current device ahead of time (for instance before the stream is
   captured); calling it is optional.  Returns CC_OK, CC_EHIP, or
   CC_EUNSUPPORTED after 256 (device, stream) pairs. */
int coolchic_stream_prepare(void* stream);

/* Measurement hook (for profilers and benchmarks, not part of the method):
   while set, every coolchic_forward / coolchic_backward call records the HIP
   event ev_begin on its stream right before the launch of the named stage and
   ev_end right after it, so hipEventElapsedTime(ev_begin, ev_end) is that
   kernel's duration.  stage: CC_STAGE_NONE clears the hook; CC_STAGE_ARM is
   the ARM kernel, CC_STAGE_SYNTHESIS the tiled synthesis kernel (residual
   convs, and in the backward the 1x1 layers' adjoint).  The events are
   hipEvent_t handles owned by the caller.  Process-wide setting: not
   thread-safe; returns CC_EINVAL for an unknown stage or a missing event. */
enum { CC_STAGE_NONE = 0, CC_STAGE_ARM = 1, CC_STAGE_SYNTHESIS = 2 };
int coolchic_set_stage_events(int stage, void* ev_begin, void* ev_end);

/* Timing events for the measurement hook (not part of the method).  A
   timing event records a GPU timestamp without the system-scope cache fence
   of a default HIP event: it orders nothing for the host or other devices,
   and timing a stage on every call then costs the pass as little as
   possible.  coolchic_timing_event_create stores a new hipEvent_t handle in
   *ev (owned by the caller, released with coolchic_timing_event_destroy);
   coolchic_timing_event_elapsed writes the milliseconds between two
   recorded events to *ms (host pointer) once both have completed
   (synchronise the stream first; HIP's not-ready error is returned as
   CC_EHIP otherwise).  CC_EINVAL for a null argument. */
int coolchic_timing_event_create(void** ev);
int coolchic_timing_event_elapsed(void* ev_begin, void* ev_end, float* ms);
int coolchic_timing_event_destroy(void* ev);

/* Uniform noise u in [-1/2, 1/2) for the training proxy y_hat = y + u
   (Section II "Encoding": the latents are optimised through a
   differentiable proxy of the quantisation).  u[4g + e] = (w_e >> 8) 2^-24
   - 1/2, where (w_0..w_3) = Philox4x32-10 (Salmon et al., SC 2011) of the
   counter (g mod 2^32, g >> 32, it, stream_id) under the key (seed mod 2^32,
   seed >> 32), and it = *step (a device int32, e.g. the step counter that
   coolchic_adam_step advances, so that a captured graph draws fresh noise on
   every replay) or 0 when step is NULL.  Enqueued on stream. */
int coolchic_uniform_noise(float* u, int64_t n, uint64_t seed, const int32_t* step, uint32_t stream_id,
                           void* stream);

/* ---- Batched overfitting: many images of uneven sizes in one launch per
   stage.  Every image has its own latents, parameters and outputs; all share
   one architecture (and quantiser).  coolchic_batch_create lays out, in the
   caller's device workspace, one backward workspace per image, the argument
   blocks of every kernel for every image, and the work-lists that map each
   work-group of a batched launch to (image, block); it uploads them with a
   synchronous copy (setup, not the hot path).  coolchic_batch_backward then
   runs the backward pass of all images (the same results as one
   coolchic_backward call per image) with one launch per stage, so a whole
   training iteration of the batch is a dozen launches and can be captured in
   a HIP graph. */
typedef struct {
  const float* img;    /* [3][H][W] */
  const float* y;      /* [N_lat] */
  const float* u;      /* [N_lat] for CC_QUANT_NOISE, else NULL */
  const float* arm_w;
  const float* ups_w;
  const float* syn_w;
  float* loss4;        /* [4] as in coolchic_backward */
  float* g_y;
  float* g_arm;
  float* g_ups;
  float* g_syn;
} cc_image_io;

/* Launch shape of the persistent kernels (tuned by the caller): total
   work-groups of the ARM launch and of the synthesis-backward launch, split
   over the images in proportion to their tiles (0 selects, per image, the
   grid coolchic_backward uses; then the results are bit-identical to it);
   arm_first selects where the ARM launch is forked onto the side stream:
   0 after the residual-conv backward, 1 before the upsampling and synthesis
   launches, 2 after the head backward; ups_tile is the side of the level-1
   tile of one work-group of the upsampling forward, 16 or 32 (0 selects 32).
   Neither changes a result; any other value is CC_EINVAL. */
typedef struct {
  int32_t arm_blocks;
  int32_t syn_blocks;
  int32_t arm_first;
  int32_t ups_tile;
} cc_batch_tuning;

typedef struct cc_batch cc_batch; /* opaque host-side plan */

/* Device workspace bytes for a batch of n problems (host arrays); 0 if any
   problem is invalid or the architectures differ.  tune may be NULL. */
size_t coolchic_batch_workspace_bytes(int32_t n, const cc_problem* probs, const cc_batch_tuning* tune);

/* Builds the plan; probs and io are host arrays of n entries (io holds device
   pointers, which must stay valid while the plan is used); dloss is the
   gradient scale of every image's loss.  *out receives a host object to free
   with coolchic_batch_destroy (NULL on any error).  Synchronises the device
   (setup call). */
int coolchic_batch_create(int32_t n, const cc_problem* probs, const cc_image_io* io, const cc_batch_tuning* tune,
                          float dloss, void* ws, size_t ws_bytes, cc_batch** out);

/* Enqueues the backward pass of every image of the batch on stream. */
int coolchic_batch_backward(const cc_batch* batch, void* stream);

void coolchic_batch_destroy(cc_batch* batch);

/* ---- Learned warm start.  Section IV-B replaces overfitting by an analysis
   transform mapping the image to the latent grids, with the decoder
   parameters learned beside it; Section V proposes to fine-tune such an
   output per image.  This network predicts, for a batch of images, the
   initial latent pyramid and decoder parameters that the overfitting then
   refines:
     trunk   f_k = bf16(ReLU(conv3x3 stride 2 (f_{k-1}) + b_k)), k = 1..4, 32
             channels, f_0 = bf16(x), zero padding, matrix-core products in
             bfloat16 with FP32 accumulation;
     latents y_l = V_l . f_l + beta_l (l = 1..4), from f_4 average-pooled by 2
             and 4 (l = 5, 6), and y_0 = conv3x3(bf16(x)) + beta_0 + V_0 . f_1
             repeated over 2x2 blocks;
     decoder theta = P mean(f_4) + pi.
   Weight matrices (conv kernels, V_l, the 3x3 level-0 kernel, P) are used
   rounded to bfloat16; biases, beta_l and pi are used as given.
   Master parameters (FP32, packed): for k = 1..4 W_k [32][3][3][C_in] (out,
   ky, kx, in; C_in = 3 for k = 1, else 32) then b_k [32]; level 0: V_0 [32],
   beta_0, K_0 [3][3][3] (ky, kx, colour); levels 1..6: V_l [32], beta_l; then
   P [n_theta][32] and pi [n_theta], n_theta = coolchic_param_count(arch).
   Images must be multiples of 64 on both sides and arch must have 7 levels. */
typedef struct {
  int32_t H, W;        /* image size (multiples of 64) */
  int32_t batch;       /* images per call */
  cc_arch arch;        /* decoder whose parameters are predicted */
} cc_warm_problem;

/* Packed master parameters of the network; -1 for an unsupported arch. */
int64_t coolchic_warm_param_count(const cc_arch* arch);

/* which = CC_WS_FORWARD or CC_WS_BACKWARD; 0 if the problem is invalid. */
size_t coolchic_warm_workspace_bytes(const cc_warm_problem* p, int which);

/* x [batch][3][H][W]; net: master parameters; y_out [batch][N_lat] (packed
   pyramid of each image, the layout coolchic_forward takes); theta_out
   [batch][n_theta] (arm, ups, syn blocks, the layout of coolchic_forward's
   weights). */
int coolchic_warm_forward(const cc_warm_problem* p, const float* x, const float* net, float* y_out,
                          float* theta_out, void* ws, size_t ws_bytes, void* stream);

/* Training loss of the batch against plain-overfit targets and its gradient
   g_net (same layout as net; overwritten).  Loss of one image: mean over its
   latents of (y - y_target)^2 plus mean over the decoder parameters of
   (theta - theta_target)^2; the batch loss is the mean over images.  The
   gradient reaching each feature map is rounded to bfloat16 before the
   convolution adjoints; a rounded weight passes its gradient to the master
   value unchanged.  loss4 (device) = {loss, latent part, parameter part,
   1 if anything was not finite}.  Recomputes the forward pass. */
int coolchic_warm_backward(const cc_warm_problem* p, const float* x, const float* net, const float* y_target,
                           const float* theta_target, float* loss4, float* g_net, void* ws, size_t ws_bytes,
                           void* stream);

/* Gradient g_net of an outer loss given its gradients g_y [batch][N_lat] and
   g_theta [batch][n_theta] with respect to the network's outputs (for
   instance the rate-distortion loss of Eq. (1) of the predicted latents and
   decoder, as coolchic_backward gives it), with the rounding points of
   coolchic_warm_backward.  loss4 = {0, 0, 0, non-finite flag}.  Recomputes
   the forward pass. */
int coolchic_warm_backward_grad(const cc_warm_problem* p, const float* x, const float* net, const float* g_y,
                                const float* g_theta, float* loss4, float* g_net, void* ws, size_t ws_bytes,
                                void* stream);

/* ---------------------------------------------------------------------
   Non-overfitted analysis transform (Section IV-B, Eq. (3)): the latents of
   every grid from the image in one forward pass, y = f_alpha(x), instead of
   overfitting them.  The paper describes the network in words only (its
   figure is not available); the reading implemented:
     block (c_in -> 64, stride s): depth-wise 7x7 convolution (zero padding
       3, stride s, bias), layer normalisation over the c_in channels of
       each position (eps 1e-6, scale and shift), 1x1 c_in -> 256 with bias,
       GELU (erf form), 1x1 256 -> 64 with bias, plus the identity branch:
       the input itself (c_in = 64, s = 1), else a 1x1 convolution c_in ->
       64 with bias of the input, 2x2 average-pooled with stride 2 when s = 2;
     level 0: block 3 -> 64 (s = 1) then two blocks 64 -> 64; levels 1..6:
       block 64 -> 64 (s = 2) then two blocks; 21 blocks, 126.6 kMAC per
       pixel;
     latent l: 1x1 convolution 64 -> 1 (with bias) of the level's last block
       output, at (H >> l) x (W >> l).
   Arithmetic: the 1x1 convolutions run on the bfloat16 matrix cores with
   FP32 accumulation -- their weights and inputs (the normalised features,
   the GELU output, the image and the pooled input of the identity branches)
   are rounded to bfloat16, and every block output is stored in bfloat16;
   the depth-wise convolutions, the normalisation, GELU, biases and the
   latent heads are FP32.
   Parameters (FP32, packed): per block in order dw_w [c_in][7][7], dw_b
   [c_in], ln_g [c_in], ln_b [c_in], W1 [256][c_in], b1 [256], W2 [64][256],
   b2 [64], and for the first block of each level Wid [64][c_in], bid [64];
   then per level the head w [64], b. */

/* Packed parameter count of the analysis transform. */
int64_t coolchic_analysis_param_count(void);

/* Device workspace bytes for n images of H x W (multiples of 64, n H W below
   2^31); 0 if the sizes are invalid. */
size_t coolchic_analysis_workspace_bytes(int32_t H, int32_t W, int32_t n);

/* x (device) [n][3][H][W] in [0, 1]; theta (device) the packed parameters;
   y (device) [n][N_lat]: each image's latents before quantisation, packed
   like coolchic_forward's y (level 0 first, raster order), N_lat over 7
   levels.  Errors: CC_EINVAL (null pointer, n < 1, H or W not a positive
   multiple of 64, n H W >= 2^31), CC_EWORKSPACE, CC_EHIP.  Enqueues on `stream`; allocates
   nothing. */
int coolchic_analysis_forward(int32_t H, int32_t W, int32_t n, const float* x, const float* theta, float* y,
                              void* ws, size_t ws_bytes, void* stream);

/* Quantisation of the decoder parameters (Section II: after the encoding the
   network parameters are quantised and entropy coded with an ad-hoc
   probability model).  Each module m (0 ARM, 1 upsampling, 2 synthesis) on a
   grid of step 2^-k, k = step_log2[m] (host array, 0..24): q = rint(theta
   2^k) (ties to even), theta_hat = q 2^-k, both exact in float32; written to
   arm_q / ups_q / syn_q (device, laid out like the inputs; they may alias
   them).  bits (device float [3]): the rate of each module, the sum over its
   parameters of -log2 of the Laplace(0, b) mass over [q - 1/2, q + 1/2] with
   b = max(mean |q|, 0.01).  ups_w / ups_q may be NULL when the architecture
   has no upsampling parameters. */
int coolchic_param_quantize(const cc_arch* arch, const float* arm_w, const float* ups_w, const float* syn_w,
                            const int32_t* step_log2, float* arm_q, float* ups_q, float* syn_q, float* bits,
                            void* stream);

/* ---- Entropy coding of the latents (Section II: the latent grids are sent
   with a range coder driven by the ARM p_psi; Section III-B: the decoder's
   ARM runs latent after latent).  The probability of a latent is the
   Laplace model of the training rate with its parameters quantised for
   coding: scale index j = rint(8 (clamp(s, ln 0.01, ln 100) - ln 0.01)) (a
   NaN s taken as ln 100), mean c + f / 16 with c = floor(mu), f =
   rint(16 (mu - c)) (16 carries into c; mu clamped to +-2^20, NaN taken as
   0), all in float32 from the ARM outputs (mu, s), which both the encoder
   and the decoder evaluate with the same fixed-order float32 code.  Table
   row (j, f) holds the frequencies 1 + floor(P (2^16 - 98)) of d = y_hat - c
   in [-48, 48] and of an escape symbol for both tails (P the Laplace(f/16,
   exp(ln 0.01 + j / 8)) masses in float64; the remainder goes to the first
   most frequent symbol).  An escaped latent sends the bit length of
   |d| - 48 (5 raw bits), its bits below the leading one (chunks of <= 8,
   most significant first) and its sign.  Coder: interleaved rANS, 32-bit
   states in [2^23, 2^31), byte renormalisation, 16-bit frequencies; level 0
   and levels 1..L-1 form two sets of min(64, rows of the set's first level)
   states, each with its own byte stream.  Decode order: step t of a grid
   decodes the latents (i, t - a i) (a = 2, 3, 4 for 8, 16, 24 context
   neighbours), rows ascending; row i is coded by state i mod n_states; the
   rows of a step go in groups of n_states consecutive rows, each group a
   round of primary symbols then rounds of the escape payloads.
   Bitstream (little-endian): "CCR1", u32 number of sets, u32 byte count of
   each set, u32 final state of every state (set 0 first), then the bytes of
   each set.  Supported: every compiled architecture with H <= 1024; the
   problem's quant and lambda are ignored.  Latents must be integers with
   |y_hat| <= 2^20. */

/* Device workspace bytes of coolchic_entropy_encode / _decode; 0 if the
   problem is invalid or unsupported. */
size_t coolchic_entropy_workspace_bytes(const cc_problem* p);

/* An output capacity that always suffices for coolchic_entropy_encode (12
   bytes per latent plus the header); -1 if the problem is invalid. */
int64_t coolchic_entropy_bound(const cc_problem* p);

/* Writes the coder's cumulative frequency tables, uint32 [75][16][99] (scale
   index j, mean offset f, symbol k = d + 48 with k = 97 the escape; entry 98
   is 2^16), to the device array cum. */
int coolchic_entropy_tables(uint32_t* cum, void* stream);

/* Encodes the integer latent pyramid yq [N_lat] (device) with the ARM
   parameters arm_w into out (device, out_capacity bytes).  *out_nbytes
   (device int64) receives the bitstream size; 0 if a latent is not an
   integer of magnitude <= 2^20 (nothing written); -size if out_capacity is
   too small (nothing written).  ws: coolchic_entropy_workspace_bytes. */
int coolchic_entropy_encode(const cc_problem* p, const float* yq, const float* arm_w, uint8_t* out,
                            size_t out_capacity, int64_t* out_nbytes, void* ws, size_t ws_bytes, void* stream);

/* Decodes a bitstream (device, in_bytes bytes, 4-byte aligned) into yq_out [N_lat] (device,
   float32 integer values), evaluating the ARM arm_w on the decoded context
   as the wavefront advances.  status (device int32 [2], one per set; the
   second is written only when L > 1): 0 on success; 1 the header does not
   match the problem or in_bytes, 2 a stream ended early, 4 the stream or the
   final states disagree with the problem (a damaged stream or other ARM
   weights); yq_out is then unspecified. */
int coolchic_entropy_decode(const cc_problem* p, const uint8_t* in, size_t in_bytes, const float* arm_w,
                            float* yq_out, int32_t* status, void* ws, size_t ws_bytes, void* stream);

/* Static description of an error code. */
const char* coolchic_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* COOLCHIC_H */

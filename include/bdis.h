/*
 * bdis.h -- C ABI of the MI355X (gfx950) Bayesian Dense Inverse Search
 * stereo library.
 *
 * Method: J. Song, Q. Zhu, J. Lin, M. Ghaffari, "Bayesian dense inverse
 * searching algorithm for real-time stereo matching in minimally invasive
 * surgery", arXiv 2106.07136.  One call runs the whole hot path on the GPU:
 * image pyramid (Sec. 1, Fig. 1), per-patch inverse-compositional LK search
 * along x (Sec. 2.1, eq. (1)), the windowed patch posterior (Sec. 2.2,
 * eqs. (3)-(4)) and the spatial-Gaussian fusion of overlapping patches
 * (Sec. 2.3, eq. (5) and the final equation), coarse to fine.
 *
 * Conventions shared by every entry point
 *   - Images are rectified 8-bit grayscale, row-major, `pitch_bytes` apart.
 *   - Output disparity is float32, row-major, `disp_pitch_elems` floats apart:
 *     disp(x, y) = d means left pixel x matches right pixel x - d; NaN marks a
 *     pixel no kept patch covers (Sec. 3.2: such pixels are not estimated).
 *   - Image and output pointers are DEVICE pointers owned by the caller.  They
 *     must stay valid until the work enqueued on `stream` has finished.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *     Calls enqueue and return; results are valid once the stream syncs.
 *   - Every entry point validates its arguments before enqueuing anything.
 *     On error nothing is enqueued, outputs are untouched, and a status < 0
 *     is returned; bdis_last_error() then holds a message.  Nothing aborts,
 *     throws or prints.
 *   - A handle is bound to one device and is not thread-safe: use one handle
 *     per host thread.  The handle owns its device workspace, grown on demand
 *     (bdis_reserve pre-sizes it) and freed by bdis_destroy.
 *   - Every compute call on a handle uses the same workspace, so calls on one
 *     handle must not overlap on the device: issue them on one stream, or
 *     order them (events) when they are on different streams.  Growing the
 *     workspace synchronises the device first.
 */
#ifndef BDIS_H
#define BDIS_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define BDIS_API __attribute__((visibility("default")))
#else
#define BDIS_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BDIS_OK = 0,
    BDIS_E_INVALID_ARG = -1,  /* bad pointer, size or parameter             */
    BDIS_E_NO_DEVICE = -2,    /* no usable gfx950 device                     */
    BDIS_E_OOM = -3,          /* device allocation failed                    */
    BDIS_E_HIP = -4,          /* a HIP runtime call failed (see last_error)  */
    BDIS_E_UNSUPPORTED = -5,  /* valid request this build does not handle    */
    BDIS_E_STATE = -6         /* call out of order (e.g. trace before run)   */
} bdis_status;

typedef enum { BDIS_FUSION_BAYES = 0, BDIS_FUSION_DIS = 1 } bdis_fusion;
typedef enum { BDIS_INIT_ZERO = 0, BDIS_INIT_LEARNED = 1 } bdis_init;

/* Method parameters.  Defaults (bdis_default_params) follow Sec. 3 of the
 * paper: sigma_r = sigma_s = 4, five window samples 0.5 px apart, gamma 0.75;
 * conv_tol = 0.05. */
typedef struct {
    uint32_t struct_size;     /* = sizeof(bdis_params), checked             */
    int32_t levels;           /* pyramid levels; 0 = auto from max_disparity:
                                 1 + ceil(log2(max_disparity / 4)); always cut
                                 so the coarsest level holds a whole patch   */
    float max_disparity;      /* level-0 pixels, used when levels == 0      */
    int32_t patch;            /* p, square patch side: 4, 6, 8, 10, 12, 16  */
    int32_t stride;           /* st, patch grid spacing, 1 <= st <= p        */
    int32_t iters;            /* K, LK iterations per level (no early exit)  */
    float sigma_r;            /* eq. (4) brightness spread, gray levels      */
    float sigma_s;            /* eq. (5) spatial spread, level pixels        */
    int32_t window;           /* samples in the posterior window (odd, <= 9) */
    float window_step;        /* spacing of the window samples, level px     */
    float gamma;              /* valid-pixel ratio below which a patch is
                                 discarded, in [0, 1]                         */
    int32_t s_mode;           /* eq. (4) "s": 0 = window samples, 1 = patch  */
    int32_t fusion;           /* bdis_fusion                                  */
    int32_t valid_lo;         /* a pixel is valid iff valid_lo <= v <= valid_hi */
    int32_t valid_hi;
    float eps_h;              /* degenerate patch iff H <= eps_h * n          */
    float conv_tol;           /* Sec. 3.2 "does not converge": a patch whose
                                 last LK step exceeds conv_tol level pixels
                                 is discarded; <= 0 turns the test off       */
    int32_t precision;        /* arithmetic of the GPU path: 0 = FP64 (the
                                 default: matches the FP64 reference to
                                 rounding), 1 = FP32 (faster, but rounding
                                 flips some discrete patch decisions, so its
                                 output is not held to that agreement)       */
    int32_t init;             /* bdis_init                                    */
    float conf_threshold;     /* learned init: confidence gate               */
    int32_t learned_fine_levels; /* learned init: levels run below the net   */
    int32_t learned_iters;    /* learned init: LK iterations per level       */
    int32_t autotune;         /* batch: 1 = per-size (patch, stride) from the
                                 tuning table set by bdis_set_tuning          */
} bdis_params;

typedef struct bdis_ctx bdis_t;
typedef struct bdisnet_ctx bdisnet_t;  /* proposal network, see below */

/* One stereo pair for bdis_compute_batch (device pointers, caller-owned).
 * max_disparity > 0 overrides the handle's for this pair (automatic level
 * count when params.levels == 0, and the staged search span). */
typedef struct {
    const uint8_t *left;
    const uint8_t *right;
    float *disp;
    int32_t width, height, pitch_bytes, disp_pitch_elems;
    float max_disparity;
} bdis_pair;

/* Sizes the library derives for one image under given parameters. */
typedef struct {
    int32_t levels;                 /* levels actually run                   */
    int32_t width[16], height[16];  /* level sizes, level 0 = input          */
    int32_t nx[16], ny[16];         /* patch grid per level                  */
    int64_t patches;                /* patches over all levels               */
    int64_t workspace_bytes;        /* device workspace for one pair         */
} bdis_plan_info;

/* Fills *p with the defaults above.  p may not be NULL. */
BDIS_API void bdis_default_params(bdis_params *p);

/* Host-only: validates p against a width x height image and describes the
 * pyramid and patch grids it implies.  No device needed.
 * Returns BDIS_OK or BDIS_E_INVALID_ARG / BDIS_E_UNSUPPORTED. */
BDIS_API bdis_status bdis_plan(const bdis_params *p, int32_t width, int32_t height, bdis_plan_info *out);

/* Creates a handle on HIP device `device`.  p is copied; NULL = defaults.
 * Errors: BDIS_E_INVALID_ARG (bad params or out == NULL), BDIS_E_NO_DEVICE
 * (no such device, or not gfx950), BDIS_E_HIP.  On error *out is NULL. */
BDIS_API bdis_status bdis_create(const bdis_params *p, int device, bdis_t **out);

/* Replaces the handle's parameters (same validation as bdis_create). */
BDIS_API bdis_status bdis_set_params(bdis_t *h, const bdis_params *p);

/* Grows the workspace so pairs up to width x height (and batches of up to
 * n_pairs such pairs) need no allocation inside bdis_compute*, for the
 * handle's current parameters (with init = learned, the network's level,
 * keep mask and output included). */
BDIS_API bdis_status bdis_reserve(bdis_t *h, int32_t width, int32_t height, int32_t n_pairs);

/* Disparity of one rectified pair, coarse to fine over the whole pyramid
 * (Sec. 2.1-2.3).  left/right: device uint8, width x height, pitch_bytes >=
 * width.  disp: device float32, disp_pitch_elems >= width.  width and height
 * must be at least the patch side. */
BDIS_API bdis_status bdis_compute(bdis_t *h, const uint8_t *left, const uint8_t *right, int32_t width,
                         int32_t height, int32_t pitch_bytes, float *disp,
                         int32_t disp_pitch_elems, void *stream);

/* bdis_compute for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels and results (bit for bit), but the workspace is a
 * library-owned array of BDIS_NOALLOC_SCRATCH_BYTES per device, created when
 * the library is loaded on that device and kept until the process ends.
 * The call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine) and does not use or grow the handle's workspace.
 *   - A request whose workspace exceeds the scratch (bdis_plan's
 *     workspace_bytes, e.g. 19.9 MiB for 1920x1080 at the defaults) fails
 *     with BDIS_E_INVALID_ARG before anything is enqueued.
 *   - Plain path only: params.init = BDIS_INIT_LEARNED gives
 *     BDIS_E_UNSUPPORTED.
 *   - Every call on a device, from any handle, shares that device's array:
 *     calls that overlap in time on one device (different streams, threads
 *     or handles) race and corrupt each other's results.  Serialise them
 *     (one stream, or events).  Nothing in the array needs to start at zero.
 *   - bdis_debug_stage is not available after this call (BDIS_E_STATE).
 *   - Per-launch profiling records nothing for this call.
 * Arguments, ownership and the other errors are those of bdis_compute. */
#define BDIS_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
BDIS_API bdis_status bdis_compute_noalloc(bdis_t *h, const uint8_t *left, const uint8_t *right, int32_t width,
                                          int32_t height, int32_t pitch_bytes, float *disp,
                                          int32_t disp_pitch_elems, void *stream);

/* Disparity with the 2-D (x, y) patch search of DIS, the method the paper
 * builds on (Sec. 2.1, Fig. 1), which tolerates imperfectly rectified pairs:
 * each patch estimates a translation (u, v) by inverse-compositional LK with
 * a 2 x 2 Hessian of the mean-normalised template gradients (degenerate when
 * its smaller eigenvalue is at most eps_h times the valid count: no 2-D
 * texture), the right image read bilinearly.  The window posterior (eqs.
 * (3)-(4)) samples along x at the converged v, the gamma gate needs all four
 * bilinear taps valid, and both components are fused with the same weights
 * (Sec. 2.3).  disp as in bdis_compute (d = -u: left (x, y) matches right
 * (x - d, y + v)); vdisp (optional, device float32, vdisp_pitch_elems >=
 * width) receives v, NaN where unestimated.  The handle's parameters apply;
 * patch sides up to 8.  Errors: as bdis_compute, and BDIS_E_UNSUPPORTED for
 * a patch above 8, eq. (2)'s fusion or the learned init. */
BDIS_API bdis_status bdis_compute_2d(bdis_t *h, const uint8_t *left, const uint8_t *right, int32_t width,
                                     int32_t height, int32_t pitch_bytes, float *disp, int32_t disp_pitch_elems,
                                     float *vdisp, int32_t vdisp_pitch_elems, void *stream);

/* One pair for bdis_compute_batch_2d: bdis_pair's fields and the vertical
 * output (device float32, NULL for none, vdisp_pitch_elems >= width). */
typedef struct {
    const uint8_t *left;
    const uint8_t *right;
    float *disp;
    float *vdisp;
    int32_t width, height, pitch_bytes, disp_pitch_elems, vdisp_pitch_elems;
    float max_disparity;
} bdis_pair2d;

/* bdis_compute_2d for n independent pairs of mixed sizes (1 <= n <= 4096)
 * in one pass: per level, one 2-D LK launch and one densification launch
 * for the pairs that have the level (at most 24 and 16 pairs a launch).
 * Each pair gets its own level count from its max_disparity (0: the
 * handle's) and the handle's patch and stride.  Each pair's results equal,
 * bit for bit, bdis_compute_2d's on a handle whose max_disparity is the
 * pair's.  `pairs` is a host array read during the call only.  Errors: as
 * bdis_compute_2d; pairs are checked before anything is enqueued. */
BDIS_API bdis_status bdis_compute_batch_2d(bdis_t *h, const bdis_pair2d *pairs, int32_t n, void *stream);

/* The same for n independent pairs of mixed sizes in one pass: each kernel of
 * the path is launched once for all pairs (level by level, coarsest first).
 * `pairs` is a HOST array of n entries, read during the call only.  Each
 * pair's result equals bdis_compute on that pair with the same parameters
 * (bit for bit).  With params.autotune = 1, each pair uses the (patch,
 * stride) that bdis_set_tuning recorded for its size class. */
BDIS_API bdis_status bdis_compute_batch(bdis_t *h, const bdis_pair *pairs, int32_t n, void *stream);

/* How bdis_compute_batch runs a batch.
 *   mode 0 (default): one launch per kernel kind and level over all pairs,
 *     the whole sequence captured once in a hipGraph and replayed while the
 *     batch (sizes, pointers, parameters) stays the same.
 *   mode 1: the same launches issued directly on the stream.
 *   mode 2: one persistent kernel over a task list of every block of every
 *     pair and level, dependencies tracked by per-job completion counters,
 *     captured with a counter-reset kernel in a hipGraph; new buffer pointers
 *     only re-upload the task tables.  Patch sides 8 and 12 only.
 * wgs_per_cu: persistent workgroups per compute unit (0 = as many as fit).
 * bdis_compute_batch_2d replays its launches from a hipGraph in mode 0 and
 * launches them directly otherwise.
 * Results are the same in every mode, bit for bit. */
BDIS_API bdis_status bdis_set_batch_mode(bdis_t *h, int32_t mode, int32_t wgs_per_cu);

/* bdis_compute_batch (modes 0 and 1, plain init) and bdis_compute_batch_2d
 * on more than 24 pairs run them as up to three groups of pairs, each
 * group's launches on a stream of its own so that they overlap: pairs go
 * largest first to the group with the fewest pixels, and each group's
 * launches take the kernel builds for its share of the compute units.  A
 * learned-init batch always runs on one stream (with its network on one
 * side stream).  Results are the same bits either way.  on: 1 (default) or
 * 0 (one stream).  Errors: BDIS_E_INVALID_ARG. */
BDIS_API bdis_status bdis_set_batch_groups(bdis_t *h, int32_t on);

/* Launch layout of the per-launch executions (bdis_compute, batch modes 0 and
 * 1).  on = 1 (default): the densification of each level >= 1 (Sec. 2.3) runs
 * inside the next finer level's LK launch -- each block writes its share of
 * the coarser field and evaluates its patches' initial-shift taps itself --
 * so a pair of L levels takes L + 1 launches after the pyramid instead of 2 L.
 * It applies to the Bayesian fusion and to LK launches of at most three blocks
 * per compute unit (one pair: latency-bound); large batches, the learned
 * injection level and eq. (2)'s fusion keep their own densify launch.  on = 0:
 * one densify launch per level.  Results are the same either way, bit for bit.  Errors:
 * BDIS_E_INVALID_ARG for a NULL handle or on not in {0, 1}. */
BDIS_API bdis_status bdis_set_fold_densify(bdis_t *h, int32_t on);

/* LK launches of the 1-D search (Sec. 2.1, eqs. (3)-(4)) with patch sides up
 * to 8 and at most patches_per_cu patches per compute unit (default 8: the
 * coarse levels of one pair) run one wave per patch, one lane per pixel,
 * instead of one lane per patch row: a shorter chain of dependent steps per
 * patch where the launch leaves the chip mostly idle.  Both kernels sum in
 * one fixed order, so results are the same bits either way.  0 = never.
 * Errors: BDIS_E_INVALID_ARG for a NULL handle or a negative count. */
BDIS_API bdis_status bdis_set_wave_lk(bdis_t *h, int32_t patches_per_cu);

/* Waits for the last bdis_compute_batch and reports whether the persistent
 * kernel had to give up a dependency wait (*flag = 1: that batch's results are
 * not valid; it cannot happen when the kernel owns the GPU).  *flag = 0 in
 * modes 0 and 1. */
BDIS_API bdis_status bdis_batch_error(bdis_t *h, int32_t *flag);

/* Autotuner table: for images whose width is <= max_width[i] (ascending),
 * use patch[i] and stride[i].  n <= 8.  n = 0 clears it. */
BDIS_API bdis_status bdis_set_tuning(bdis_t *h, int32_t n, const int32_t *max_width, const int32_t *patch,
                            const int32_t *stride);

/* Stage taps of the most recent single-pair bdis_compute, for parity checks.
 * Synchronises the handle's last stream, then copies to HOST memory `dst`
 * (capacity `bytes`):
 *   stage 0: left pyramid level `level` (float, W_l x H_l; level >= 1)
 *   stage 1: right pyramid level (float, level >= 1)
 *   stage 2: per-patch shift u after the LK iterations (float, ny x nx)
 *   stage 3: per-patch fusion weight (float, ny x nx; 0 = discarded)
 *   stage 4: per-patch outcome (int8: 0 kept, 1 degenerate, 2 diverged,
 *            3 gated by gamma)
 *   stage 5: dense field U_l in level pixels (float, W_l x H_l; level >= 1).
 *            No step of a compute reads U_1 when the level-0 LK launch
 *            densifies level 1 itself (it needs only its initial shifts), so
 *            that compute leaves U_1 unwritten; asked for it, this call
 *            first runs one densify launch of level 1 on the last stream.
 *   stage 6: per-patch initial shift u0 (float, ny x nx)
 *   stage 7: learned init only: the gate's keep mask at the injection level
 *            (uint8, W_l x H_l, level = learned_fine_levels; 1 = the
 *            network's proposal was kept, 0 = the plain field was used)
 *   stage 8: learned init only: the network's output at the 1/16 level
 *            (FP32, H_4 x W_4 x 2: disparity, confidence logit; level = 4)
 * Stages 0-3, 5 and 6 are in the handle's arithmetic type (double with
 * precision 0, float with precision 1).  Pyramid values hold validity in the
 * sign bit (negative or -0 = invalid).
 * Errors: BDIS_E_STATE (no single-pair compute yet), BDIS_E_INVALID_ARG. */
BDIS_API bdis_status bdis_debug_stage(bdis_t *h, int32_t stage, int32_t level, void *dst, size_t bytes);

/* Per-kernel timing of the handle's launches, for measurement tools.  With
 * profiling on, every kernel launch is bracketed by HIP events recorded on
 * the launch stream (this adds a small gap between launches).  Entries are
 * keyed by kernel and pyramid level, e.g. "lk_f64_p8_l0", "dense_f64_l0",
 * "pyr_f64_l1". */
typedef struct {
    char name[48];
    int32_t launches;
    double total_ms;          /* sum of event-to-event durations            */
} bdis_kernel_time;

/* on = 1 starts recording (and clears earlier records), 0 stops. */
BDIS_API bdis_status bdis_set_profiling(bdis_t *h, int32_t on);

/* Waits for the recorded launches, then writes up to cap entries to the HOST
 * array out (one per kernel name, in first-launch order) and sets *count to
 * the number of entries available.  Records stay until the next
 * bdis_set_profiling(h, 1). */
BDIS_API bdis_status bdis_get_profile(bdis_t *h, bdis_kernel_time *out, int32_t cap, int32_t *count);

/* ------------------------------------------------------------------------
 * Learned proposal network (an added serving pattern, not in the paper):
 * four 3x3 convolutions with ReLU on the 1/16 pyramid level -> (coarse
 * disparity, confidence logit).  BF16 weights and activations, FP32
 * accumulation on the matrix cores (implicit GEMM).  FP32 master weights
 * and Adam moments stay on the device.  Parameter vector layout (FP32): for
 * each layer in order, weights [3][3][C_in][C_out] (tap row, tap column,
 * input channel, output channel) then biases [C_out]; layer (C_in, C_out):
 * (16, C), (C, C), (C, C), (C, 2).  Input: NHWC bfloat16, 16 channels.
 * Output: NHWC FP32, 2 channels.  All device pointers are caller-owned.
 * ------------------------------------------------------------------------ */
/* channels C: 32 or 48.  Weights start at zero (set them before use). */
BDIS_API bdis_status bdisnet_create(int32_t channels, int device, bdisnet_t **out);
BDIS_API void bdisnet_destroy(bdisnet_t *h);               /* NULL-safe */
BDIS_API int64_t bdisnet_param_count(const bdisnet_t *h);
/* FP32 master weights from/to HOST memory (n = bdisnet_param_count);
 * setting them also clears the Adam moments.  Synchronous. */
BDIS_API bdis_status bdisnet_set_params(bdisnet_t *h, const float *host, int64_t n);
BDIS_API bdis_status bdisnet_get_params(bdisnet_t *h, float *host, int64_t n);
/* Forward of n images of hh x ww (device x, device out); the handle keeps
 * the activations for one backward. */
BDIS_API bdis_status bdisnet_forward(bdisnet_t *h, const uint16_t *x, int32_t n, int32_t hh, int32_t ww,
                                     float *out, void *stream);
/* Training loss of the last forward against target (device FP32 per pixel,
 * coarse disparity) on valid pixels (device uint8): mean over valid pixels
 * of Huber(d - t; delta) + conf_weight * BCE(sigmoid(c), [|d - t| < conf_tol]).
 * Writes the scalar to device *loss and keeps d loss / d output. */
BDIS_API bdis_status bdisnet_loss(bdisnet_t *h, const float *target, const uint8_t *valid, float delta,
                                  float conf_tol, float conf_weight, float *loss, void *stream);
/* Use a caller-supplied d loss / d output (device FP32, 2 channels) instead. */
BDIS_API bdis_status bdisnet_set_output_grad(bdisnet_t *h, const float *gout, void *stream);
/* Gradients of all parameters from the kept activations and output
 * gradient (deterministic: no atomics). */
BDIS_API bdis_status bdisnet_backward(bdisnet_t *h, void *stream);
BDIS_API bdis_status bdisnet_get_grads(bdisnet_t *h, float *host, int64_t n);
/* One Adam step (step counts from 1) on the FP32 master weights, then the
 * BF16 copies used by the kernels are refreshed. */
BDIS_API bdis_status bdisnet_adam_step(bdisnet_t *h, float lr, float beta1, float beta2, float eps,
                                       int32_t step, void *stream);
/* Checkpoints for resuming training bit for bit.  Layout (little-endian):
 * 8 bytes "BDISNET\0", uint32 version (1), int32 channels, int64 parameter
 * count n, int64 last Adam step, then n FP32 master weights (the layout of
 * bdisnet_set_params), n FP32 first and n FP32 second Adam moments:
 * bdisnet_checkpoint_bytes(h) = 32 + 12 n bytes.  Save writes to HOST memory
 * `blob` of capacity `bytes`; load restores weights, moments and step into a
 * network of the same channel count and refreshes the BF16 copies.  Both
 * synchronise the device.  Errors: BDIS_E_INVALID_ARG (capacity too small;
 * on load: wrong magic or version, another channel count, a truncated blob,
 * a non-finite value or a negative second moment). */
BDIS_API int64_t bdisnet_checkpoint_bytes(const bdisnet_t *h);
BDIS_API bdis_status bdisnet_save(bdisnet_t *h, void *blob, int64_t bytes);
BDIS_API bdis_status bdisnet_load(bdisnet_t *h, const void *blob, int64_t bytes);
/* The last step passed to bdisnet_adam_step (0 after create or
 * set_params; restored by load). */
BDIS_API int32_t bdisnet_step(const bdisnet_t *h);
/* Input of layer `layer` (0 = the network input) from the last forward, as
 * bfloat16 bits in HOST memory.  Synchronous. */
BDIS_API bdis_status bdisnet_debug_activation(bdisnet_t *h, int32_t layer, uint16_t *host, size_t elems);
BDIS_API const char *bdisnet_last_error(const bdisnet_t *h);

/* Attaches a proposal network (NULL detaches) for params.init =
 * BDIS_INIT_LEARNED.  The learned path: pyramid down to the 1/16 level, the
 * network there (pairs of one 1/16 size batched together), then a gate that
 * writes the initial field of level learned_fine_levels: u = -4 d (d the
 * network disparity read bilinearly, the factor being the scale between the
 * 1/16 level and that level) where the confidence is >= conf_threshold.  The
 * plain levels from the coarsest down to learned_fine_levels are the
 * fallback: they replace the initial field where the confidence is low.
 * They run on the caller's stream while the network runs on a second stream
 * of the handle (forked from and joined back into the caller's stream, also
 * inside a captured graph), so the network costs no time on the path.  The
 * finer levels run with learned_iters LK iterations.  The handle does not own
 * a network attached here; keep it alive while it is attached (a network the
 * handle owns, from bdis_set_net_weights, is freed first).
 * Errors: BDIS_E_INVALID_ARG (network on another device). */
BDIS_API bdis_status bdis_set_net(bdis_t *h, bdisnet_t *net);

/* Loads a network for the learned init from a bdisnet_save checkpoint (HOST
 * memory, read during the call; only its weights are used) into a network
 * the handle creates and owns, and attaches it in place of any other.  The
 * owned network is freed by bdis_destroy, by the next bdis_set_net_weights
 * and by bdis_set_net.  Errors: as bdisnet_load, BDIS_E_OOM, BDIS_E_HIP. */
BDIS_API bdis_status bdis_set_net_weights(bdis_t *h, const void *blob, int64_t bytes);

/* Network input of n pairs whose 1/16 levels have the same size: builds
 * their pyramids down to the 1/16 level and writes x (device, NHWC
 * bfloat16, n x H16 x W16 x 16): (L - 128)/64, (R - 128)/64 and
 * |L(x) - R(x - d)|/64 for d = 0..13, R's column clamped.  Used to build
 * training batches. */
BDIS_API bdis_status bdis_net_input(bdis_t *h, const bdis_pair *pairs, int32_t n, uint16_t *x, void *stream);

/* ------------------------------------------------------------------------
 * Before and after the matcher (Sec. 1: stereo under the pinhole camera
 * model is rectified and undistorted before disparity estimation; Sec. 3:
 * the data are rectified and undistorted with their calibration; Sec. 3.2:
 * errors in mm, and undistortion leaves invalid pixels at the image edges).
 * Handle-free calls on the current HIP device; errors as above, with the
 * message in bdis_last_error(NULL).
 * ------------------------------------------------------------------------ */

/* Calibration of one camera of a stereo rig.  Lens model: radial-tangential
 * (Brown-Conrady).  A rectified pixel (u, v) looks along the ray
 * ((u - ncx) / nfx, (v - ncy) / nfy, 1) of the rectified frame; R maps a
 * direction of the raw camera frame to the rectified frame (row-major), so
 * the raw frame sees R^T of that ray, projected to (x, y); the lens moves it
 * to x (1 + k1 r^2 + k2 r^4 + k3 r^6) + 2 p1 x y + p2 (r^2 + 2 x^2) and
 * y (1 + k1 r^2 + k2 r^4 + k3 r^6) + p1 (r^2 + 2 y^2) + 2 p2 x y
 * (r^2 = x^2 + y^2), and (fx, fy, cx, cy) maps that to raw pixels. */
typedef struct {
    double fx, fy, cx, cy;       /* raw camera matrix, pixels                 */
    double k1, k2, p1, p2, k3;   /* distortion of the raw image               */
    double R[9];                 /* rectifying rotation, row-major            */
    double nfx, nfy, ncx, ncy;   /* camera matrix of the rectified image      */
} bdis_camera;

/* One image to rectify: raw src (device uint8, src_pitch bytes per row) into
 * dst (device uint8, dst_pitch bytes per row), both caller-owned. */
typedef struct {
    const uint8_t *src;
    uint8_t *dst;
    int32_t src_width, src_height, src_pitch;
    int32_t dst_width, dst_height, dst_pitch;
    bdis_camera cam;
} bdis_rectify_job;

/* Rectified, undistorted images for the matcher, n = 1..8 jobs (a stereo
 * pair is 2) in one launch.  Each output pixel takes its raw image
 * bilinearly at its source position (computed in FP64 per pixel; no map is
 * stored) and rounds to the nearest gray level, halves up.  A source
 * position outside the raw image's pixel centres gives 0, below the default
 * validity band, so the matcher leaves such edge pixels out (Sec. 3.2).
 * `jobs` is a HOST array read during the call.  Errors: BDIS_E_INVALID_ARG
 * (NULL pointer, size outside [1, 65536], pitch < width, non-finite
 * calibration or a zero focal length), BDIS_E_HIP. */
BDIS_API bdis_status bdis_rectify(const bdis_rectify_job *jobs, int32_t n, void *stream);

/* Depth along the optical axis of a rectified pair: Z = focal_px *
 * baseline / d, computed in FP64 and stored as float32, in the unit of
 * `baseline` (mm for the paper's figures); NaN where d is NaN or
 * d <= min_disparity.  disp and depth: device float32, pitches in elements.
 * Errors: BDIS_E_INVALID_ARG (NULL pointer, bad size or pitch, focal_px or
 * baseline not finite and positive, min_disparity negative), BDIS_E_HIP. */
BDIS_API bdis_status bdis_depth_from_disparity(const float *disp, int32_t width, int32_t height,
                                               int32_t disp_pitch_elems, double focal_px, double baseline,
                                               float min_disparity, float *depth, int32_t depth_pitch_elems,
                                               void *stream);

/* Frees the handle and its workspace; NULL is allowed. */
BDIS_API void bdis_destroy(bdis_t *h);

/* Static text for a status code. */
BDIS_API const char *bdis_status_string(bdis_status s);

/* Last error message of h, or of the calling thread's last failed
 * bdis_create / bdis_plan when h is NULL.  Never NULL. */
BDIS_API const char *bdis_last_error(const bdis_t *h);

#ifdef __cplusplus
}
#endif
#endif /* BDIS_H */

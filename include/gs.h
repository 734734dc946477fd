/*
 * gs.h -- C interface of the MI355X (gfx950) batched Gaussian-splat renderer.
 *
 * The library renders RGB and expected depth of many pinhole cameras over
 * many 3D Gaussian-splat scenes, the renderer the paper drops into its
 * vectorised simulator (Sec. 3.2 "3D Gaussian Splatting as a Drop-in
 * Renderer": splats batch-rendered across environments; depth as a
 * by-product of the same rasterisation, Fig. "Rendering RGB and Depth";
 * thousands of environments over many scenes on one GPU, Sec. 3.3).
 * The splat model is the cited 3DGS (Sec. 2.3): EWA projection with a
 * 0.3 px^2 low-pass, SH colour, 16x16 tile binning sorted by tile and depth,
 * front-to-back compositing with alpha clamped to 0.99, contributions below
 * 1/255 skipped and the walk stopped before transmittance falls under 1e-4.
 *
 * Conventions
 *   poses       camera-to-world [R | C], 3x4 row-major FP32, OpenCV axes
 *               (x right, y down, z forward)
 *   intrinsics  (fx, fy, cx, cy) FP32 in pixels; pixel (i, j) covers
 *               [i, i+1) x [j, j+1), its centre is (i + 1/2, j + 1/2)
 *   quaternions (w, x, y, z), any non-zero norm (normalised inside)
 *   scales      linear (> 0); opacity linear in [0, 1]
 *   sh          [n][(deg+1)^2][3], real SH with Condon-Shortley phase,
 *               l-major, m = -l..l; colour = max(0, SH(d) + 0.5) with d the
 *               unit direction from the camera centre to the mean
 *   outputs     rgb [n_cams][H][W][3], depth [n_cams][H][W] (expected camera
 *               z, 0 where nothing was accumulated), alpha [n_cams][H][W]
 *               (accumulated weight = 1 - final transmittance), FP32
 *
 * Ownership: the library copies every scene it is given; callers own every
 * pointer they pass. Device pointers are HIP device addresses on the
 * context's device. Streams are hipStream_t passed as void* (NULL = the
 * default stream).
 *
 * Errors: every call returns GS_OK (0) or a negative GS_ERR_* code and never
 * throws; gs_last_error() describes the last failure of that context.
 * Argument validation is synchronous. A context is not thread-safe: use one
 * per thread or lock around it. Its calls share the context's work buffers:
 * a render (any gs_render_* call) enqueued on another stream than the
 * previous render starts on the device only after that render; the
 * upsampler calls are ordered only by their stream, so enqueue them on the
 * renders' stream or order the streams with events.
 */
#ifndef GS_H
#define GS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gs_ctx gs_ctx;

#define GS_OK 0
#define GS_ERR_INVALID_ARG (-1)
#define GS_ERR_BAD_SCENE (-2)
#define GS_ERR_OOM (-3)
#define GS_ERR_CAPACITY (-4)
#define GS_ERR_HIP (-5)
#define GS_ERR_BUSY (-6)
#define GS_ERR_NOT_TRAINED (-7)

#define GS_MEM_HOST 0
#define GS_MEM_DEVICE 1

#define GS_MODE_PLAIN 0   /* per-camera kernel sequence, eager launches */
#define GS_MODE_BATCHED 1 /* all cameras in camera chunks, one launch per stage */

typedef struct {
    int64_t n;          /* number of Gaussians, >= 1 */
    int32_t sh_degree;  /* 0..3 */
    int32_t mem_kind;   /* GS_MEM_HOST or GS_MEM_DEVICE for all five arrays */
    const float *means;   /* [n][3] world position (m) */
    const float *scales;  /* [n][3] linear standard deviations (m), > 0 */
    const float *quats;   /* [n][4] (w, x, y, z) */
    const float *opacity; /* [n] in [0, 1] */
    const float *sh;      /* [n][(sh_degree+1)^2][3] */
} gs_scene_desc;

typedef struct {
    float near_plane;  /* Gaussians with camera z <= near_plane are dropped (default 0.2) */
    float bg[3];       /* background colour added with the final transmittance (default 0) */
    int32_t mode;      /* GS_MODE_PLAIN or GS_MODE_BATCHED (default BATCHED) */
    int32_t tile_w;    /* raster tile width in pixels; 0 = tuned/default (16) */
    int32_t tile_h;    /* raster tile height; 0 = tuned/default (16) */
    int32_t lds_batch; /* records each raster wave fetches, culls and lists in LDS per
                          batch (64, 128 or 256); 0 = tuned/default (128) */
    int32_t chunk_cams;/* BATCHED: cameras per chunk (1..4096); 0 = tuned/default. A
                          chunk also ends before its cameras' scenes exceed a budget of
                          Gaussian slots sized from the device memory (84 B per slot in
                          each of the four pipelines, a third of the memory in all) */
    int32_t persistent;/* BATCHED: raster as a persistent work queue (1), a grid (0), -1 = tuned */
    int32_t use_graph; /* BATCHED: capture the step into a HIP graph and replay it (1) */
    int32_t timing;    /* record HIP events around every stage (eager renders only) */
    int32_t count_pairs; /* also count contributing / evaluated (pixel, Gaussian) pairs
                            with an instrumented raster kernel (slower; for measurement) */
    int32_t streams;   /* BATCHED: chunk pipelines, each on its own stream (1..4; 0 =
                          4): the raster of one chunk overlaps the next chunks'
                          projection and sorts (timing renders always use one) */
    int32_t sync;      /* gs_render_batch: 1 = return only when the render has finished
                          (see gs_render_batch); 0 (default) = asynchronous */
    int32_t reserved[1];
} gs_render_opts;

/* Stages timed when gs_render_opts.timing is set (indices of stage_ms). */
#define GS_STAGE_SETUP 0   /* flag reset + camera setup */
#define GS_STAGE_PROJECT 1 /* EWA projection + SH colour */
#define GS_STAGE_COMPACT 2 /* visibility scan + compaction */
#define GS_STAGE_DEPTH_SORT 3
#define GS_STAGE_EMIT 4    /* tile-count scan + instance emission */
#define GS_STAGE_TILE_SORT 5 /* tile sort; its last pass also writes the tile ranges */
#define GS_STAGE_RANGES 6    /* emptying the tile ranges before the tile sort */
#define GS_STAGE_RASTER 7
#define GS_N_STAGES 8

typedef struct {
    int64_t visible;          /* (camera, Gaussian) pairs whose footprint meets the image */
    int64_t instances;        /* (camera, tile, Gaussian) entries that were sorted */
    int64_t instance_capacity;/* current instance buffer capacity */
    int32_t regrows;          /* capacity regrowths during the last render */
    int32_t graph_captures;   /* graphs captured by this context so far */
    int32_t tile_w, tile_h, lds_batch, chunk_cams, persistent; /* choice actually used */
    int32_t stage_launches[GS_N_STAGES]; /* timed intervals per stage, one per camera chunk;
                                            the raster stage is one kernel launch */
    float stage_ms[GS_N_STAGES];         /* summed HIP-event time per stage (timing renders) */
    int64_t pairs_contrib;   /* (pixel, Gaussian) pairs accumulated (count_pairs renders) */
    int64_t pairs_evaluated; /* pairs of still-live pixels whose alpha the raster evaluated
                                (count_pairs renders) */
    int64_t pairs_issued;    /* lanes the raster's walk issued: 64 per (wave, record) step,
                                live pixels or not (count_pairs renders) */
} gs_stats;

/* Status of the context's renders. wait != 0: first wait for the last render
 * enqueued (gs_render_batch and the other render calls). Returns
 * GS_ERR_CAPACITY when a render that returned without waiting overflowed
 * the instance buffers since the last call (its frames are incomplete; the
 * buffers have been grown, so rendering again gives complete frames),
 * GS_ERR_HIP when the device reported an error, GS_OK otherwise. */
int gs_render_status(gs_ctx *ctx, int32_t wait);

/* sizeof of gs_scene_desc, gs_render_opts and gs_stats as compiled into the
 * library (lets bindings check their struct layouts). Returns GS_OK. */
int gs_abi_sizes(int32_t *scene_desc, int32_t *render_opts, int32_t *stats);

/* Fill opts with the defaults listed in gs_render_opts. */
void gs_default_opts(gs_render_opts *opts);

/* Create a context on HIP device `hip_device`. *out receives the handle.
 * Environment variables read here: GS_TRACE (one line per render on
 * stderr), GS_DEBUG (eager renders wait after every stage and name the
 * stage of a device error). */
int gs_create(int hip_device, gs_ctx **out);

/* Free every scene, workspace and captured graph of the context. */
int gs_destroy(gs_ctx *ctx);

/* Text of the last error of the context (valid until the next call). */
const char *gs_last_error(const gs_ctx *ctx);

/* Copy a scene into the library (synchronous). The library precomputes the
 * factor M = R(q) S of the 3D covariance M M^T per Gaussian and stores the
 * SH coefficients in a planar layout. Returns its id in *scene_id_out. Rejects n < 1, degree
 * outside 0..3, null arrays, non-finite values (GS_ERR_BAD_SCENE). */
int gs_upload_scene(gs_ctx *ctx, const gs_scene_desc *desc, int32_t *scene_id_out);

/* Free a scene. GS_ERR_BUSY if a captured graph still references it. */
int gs_release_scene(gs_ctx *ctx, int32_t scene_id);

/* Number of Gaussians of a scene (or a negative error). */
int64_t gs_scene_size(gs_ctx *ctx, int32_t scene_id);

/*
 * Render n_cams cameras.
 *   scene_ids   HOST int32 [n_cams]: scene of each camera (environment)
 *   poses       DEVICE float [n_cams][3][4]
 *   intrinsics  DEVICE float [n_cams][4]
 *   rgb, depth  DEVICE float outputs (layouts in the header comment)
 *   alpha       DEVICE float [n_cams][H][W] or NULL
 *   opts        NULL for defaults
 * Asynchronous on `stream`: the call enqueues the render and returns; the
 * outputs are valid once the stream has reached that point. The instance
 * buffers (tile entries of a camera chunk) are sized by the renders
 * themselves: the first render of a configuration (cameras, scenes, sizes,
 * choice, pipelines), and every render with opts->sync, timing or
 * count_pairs set, waits for the stream, grows the buffers and renders again
 * if they overflowed, so it returns complete outputs. Later renders of the
 * configuration do not wait: each call first looks, without waiting, at the
 * renders that have finished, and grows the buffers when a chunk came
 * within a fifth of their size; if a render overflowed anyway its frames are
 * incomplete and gs_render_status reports it (GS_ERR_CAPACITY, the buffers
 * already grown). In BATCHED mode with use_graph the first call for a given
 * configuration and set of buffers captures a HIP graph and later calls
 * replay it with no host synchronisation.
 */
int gs_render_batch(gs_ctx *ctx, int32_t n_cams, const int32_t *scene_ids, const float *poses,
                    const float *intrinsics, int32_t width, int32_t height, float *rgb,
                    float *depth, float *alpha, const gs_render_opts *opts, void *stream);

/*
 * Backward pass of the render (the splats of a scene are fitted by
 * rendering them differentiably against images: Sec. 2.3, Sec. 3.1).
 * Gradients of
 *     L = sum over cameras and pixels of  grad_rgb . RGB + grad_depth * depth
 *                                        + grad_alpha * alpha
 * with respect to the parameters of scene `scene_id`, for n_cams cameras of
 * that scene rendered as gs_render_batch renders them (same near plane and
 * background from opts; NULL for defaults; opts->chunk_cams bounds the
 * cameras per chunk). Every discrete decision of the forward pass (near
 * plane, the 1/255 skip, the 1e-4 stop, the 0.99 clamp, the Jacobian's
 * tangent clamp, the colour's clamp at 0) is held as the forward pass takes
 * it, so this is the derivative of the branch the render follows.
 *   poses, intrinsics  DEVICE float [n_cams][3][4], [n_cams][4]
 *   grad_rgb           DEVICE float [n_cams][H][W][3] or NULL
 *   grad_depth         DEVICE float [n_cams][H][W] or NULL (expected depth)
 *   grad_alpha         DEVICE float [n_cams][H][W] or NULL (accumulated weight)
 *                      (NULL gradients are zero; at least one is required)
 *   d_means [N][3], d_scales [N][3], d_quats [N][4] (w, x, y, z, for the
 *   quaternion as uploaded, not normalised), d_opacity [N],
 *   d_sh [N][(deg+1)^2][3]: DEVICE float outputs in the order the scene was
 *   uploaded in, overwritten (scales and opacities are the linear values the
 *   scene was uploaded with).
 * Every sum runs in a fixed order, so the result is deterministic. The call
 * waits for `stream` (the instance buffers' overflow flag is read and the
 * pass repeated with larger buffers when they overflowed).
 * GS_ERR_INVALID_ARG for a bad scene id, size or null pointer.
 */
int gs_render_backward(gs_ctx *ctx, int32_t scene_id, int32_t n_cams, const float *poses,
                       const float *intrinsics, int32_t width, int32_t height,
                       const float *grad_rgb, const float *grad_depth, const float *grad_alpha,
                       const gs_render_opts *opts, float *d_means, float *d_scales,
                       float *d_quats, float *d_opacity, float *d_sh, void *stream);

/* Camera-rate decimation (the paper renders at the camera's own frame rate,
 * below the control rate, Sec. 3.3; staggering the environments over the
 * period, so that every step renders a similar share, is this library's
 * choice):
 * renders only the cameras due at sim_step, camera i being due when
 * (sim_step + phase[i]) mod period == 0, into their own output slots; the
 * other cameras' slots are left untouched (they keep their last frame).
 * phase: HOST int32 [n_cams] (values >= 0), or NULL for phase[i] = i, which
 * spreads the cameras evenly over the period. Other arguments as
 * gs_render_batch (the batch is the full camera set; the per-subset plan and
 * graph are cached per distinct subset). *n_due_out (HOST, nullable)
 * receives the number of cameras rendered; with none due nothing is
 * enqueued. Asynchronous on stream. */
int gs_render_due(gs_ctx *ctx, int32_t n_cams, const int32_t *scene_ids, const float *poses,
                  const float *intrinsics, int32_t width, int32_t height, int64_t sim_step,
                  int32_t period, const int32_t *phase, float *rgb, float *depth, float *alpha,
                  const gs_render_opts *opts, int32_t *n_due_out, void *stream);

/* Motion blur (Sec. 3.3 and the appendix figure on motion blur: frames
 * offset along the camera's velocity over the shutter interval, blended into
 * one image). Sub-frame k < n_sub renders camera i from centre
 * C_i - v_i * dt_k, dt_k = shutter * (k + 1/2) / n_sub (the middle of the
 * k-th equal part of the exposure [t - shutter, t]; rotation unchanged).
 * Output: rgb and alpha are the means over the sub-frames, depth the
 * alpha-weighted mean of the sub-frame depths (0 where all are empty).
 *   velocities DEVICE f32 [n_cams][3], world frame (m/s); shutter >= 0 (s);
 *   1 <= n_sub <= 16; other arguments as gs_render_batch (alpha nullable;
 *   the library then keeps the weight sums in its own buffer).
 * Asynchronous on stream; sub-frames run as n_sub batched renders that add
 * into the outputs (captured graphs per sub-frame when use_graph is set). */
int gs_render_batch_motion_blur(gs_ctx *ctx, int32_t n_cams, const int32_t *scene_ids,
                                const float *poses, const float *velocities,
                                const float *intrinsics, int32_t width, int32_t height,
                                float shutter, int32_t n_sub, float *rgb, float *depth,
                                float *alpha, const gs_render_opts *opts, void *stream);

/* Calibration: the rate this GPU sustains (best of 3 timed runs after a
 * warm-up), the measured peaks beside the published ones in a roofline.
 *   kind 0: FP32 FMA lane-operations/s (8 independent chains per lane),
 *   kind 1: v_exp_f32 lane-operations/s (8 independent chains per lane),
 *   kind 2: HBM bytes/s of a 1 GiB device copy (bytes read + written).
 * *rate_out (HOST) receives the rate. Synchronous; allocates and frees its
 * own buffers (up to 2 GiB for kind 2). */
int gs_peak_probe(gs_ctx *ctx, int32_t kind, double *rate_out);

/* Counters and choices of the last gs_render_batch of the context. */
int gs_last_stats(gs_ctx *ctx, gs_stats *out);

/* Set the instance-buffer capacity (entries per chunk) used by the next
 * render; the library still grows it on overflow, up to 2^31. Drops captured
 * graphs. 1 <= cap <= 2^31, else GS_ERR_INVALID_ARG. */
int gs_set_instance_capacity(gs_ctx *ctx, int64_t cap);

/* Destroy every captured graph of the context (releases their scene refs). */
int gs_clear_graphs(gs_ctx *ctx);

/*
 * Per-Gaussian projection of one camera, for checking the projection stage.
 *   pose, intrinsics  HOST float [12], [4]
 *   out               DEVICE float [n][16]: u, v, z, opacity, conic A B C
 *                     (inverse 2D covariance incl. low-pass), r, g, b,
 *                     x0, x1, y0, y1 (inclusive pixel-centre box of
 *                     alpha >= 1/255; x0 > x1 when not visible), visible
 * Synchronous.
 */
int gs_debug_project(gs_ctx *ctx, int32_t scene_id, const float *pose, const float *intrinsics,
                     int32_t width, int32_t height, float near_plane, float *out);

/*
 * Time the batched form over candidate (tile shape, LDS batch, chunk size,
 * persistent) choices for this camera batch and remember the pick for
 * later renders with the same (W, H, camera count, scene-size bucket): the
 * candidates are tried in a fixed order of preference (the default choice
 * first), and the earliest one within 2% of the fastest is picked, so noise
 * in the timings does not flip the pick between near-equal choices.
 * With `cache_path` (JSON lines, one object per tuning: "key" = GPU
 * architecture, compute units, W, H, camera count and scene-size bucket;
 * "best" = TWxTH/bB/cC/pP; the timing table), the last entry of the file for
 * this key is used without timing anything; otherwise the tuning runs and
 * its entry is appended. Arguments as gs_render_batch (outputs are
 * scratch). Synchronous.
 */
int gs_autotune(gs_ctx *ctx, int32_t n_cams, const int32_t *scene_ids, const float *poses,
                const float *intrinsics, int32_t width, int32_t height, float *rgb, float *depth,
                const char *cache_path, void *stream);

/* ------------------------------------------------------------------------
 * Learned 4x upsampler (a workload of this renderer, not part of the paper):
 * render at W/4 x H/4 with intrinsics / 4, then four 3x3 convolutions
 * (4 -> 32 -> 32 -> 32 -> 64 channels, ReLU after the first three; BF16
 * weights and activations on MFMA, FP32 accumulation), 4x pixel shuffle plus
 * bilinear 4x upsampling of the low-resolution RGB + depth/10.
 *
 * Parameter vector (FP32, `gs_upsampler_num_params()` values), per layer
 * l = 1..4: weights [cout][3][3][cin] then bias [cout], with
 * (cin, cout) = (4, 32), (32, 32), (32, 32), (32, 64).
 * ------------------------------------------------------------------------ */

typedef struct {
    int32_t batch;   /* cameras per optimisation step (default 32) */
    int32_t steps;   /* optimisation steps */
    float lr;        /* Adam learning rate at step 0 (default 1e-3) */
    float lr_min;    /* cosine-decayed to this value at the last step */
    int32_t reserved[4];
} gs_train_opts;

/* Number of FP32 values of the parameter vector. */
int64_t gs_upsampler_num_params(void);

/* He-uniform weights from `seed`, zero biases, last layer zero (so the
 * untrained network equals bilinear upsampling); resets the Adam state. */
int gs_upsampler_init(gs_ctx *ctx, uint64_t seed);

/* Copy the parameter vector in (host, n values) or out. Setting resets Adam. */
int gs_upsampler_set_weights(gs_ctx *ctx, const float *params, int64_t n);
int gs_upsampler_get_weights(gs_ctx *ctx, float *params, int64_t n);

/* Checkpoint: parameter vector, Adam moments and Adam step to / from a file
 * (little-endian: "GSUPCKPT", u32 version 1, u32 0, i64 parameter count,
 * i32 step, u32 0, then 3 x count FP32: parameters, first moments, second
 * moments, each in the parameter-vector layout). Load restores the training
 * state exactly; a file of another version or size is GS_ERR_INVALID_ARG.
 * Synchronous. */
int gs_upsampler_save(gs_ctx *ctx, const char *path);
int gs_upsampler_load(gs_ctx *ctx, const char *path);

/* Network forward on given low-res frames.
 *   rgb_lo [n][h][w][3], depth_lo [n][h][w] DEVICE; outputs rgb_out
 *   [n][4h][4w][3], depth_out [n][4h][4w] DEVICE. Asynchronous on stream. */
int gs_upsampler_forward(gs_ctx *ctx, int32_t n, int32_t h, int32_t w, const float *rgb_lo,
                         const float *depth_lo, float *rgb_out, float *depth_out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * network forward as gs_upsampler_forward, with the same kernels and
 * bitwise the same outputs, whose activations live in a fixed scratch array
 * of 64 MiB that the library holds on every GPU it runs on until the
 * process ends (208 bytes per low-resolution pixel: frames go through it as
 * many at a time as fit, so n is unbounded). It calls no hipMalloc or
 * hipFree and no allocating library routine.
 *   Arguments as gs_upsampler_forward (all DEVICE, asynchronous on stream).
 *   GS_ERR_INVALID_ARG if one frame's activations (208 h w bytes) exceed the
 *   scratch array (h w > 322,630), GS_ERR_NOT_TRAINED before the weights
 *   are set. Every call on one GPU shares that GPU's array and keeps the last
 *   call's contents: calls that overlap on one GPU (different streams or
 *   contexts without ordering between them) race and give wrong frames. */
int gs_upsampler_forward_noalloc(gs_ctx *ctx, int32_t n, int32_t h, int32_t w,
                                 const float *rgb_lo, const float *depth_lo, float *rgb_out,
                                 float *depth_out, void *stream);

/* Forward + backward for the loss mean_p sum_c w_c (pred_c - target_c)^2,
 * w = (1, 1, 1, 0.1) over (r, g, b, depth/10), targets rgb_hi [n][4h][4w][3]
 * and depth_hi [n][4h][4w] (DEVICE). Writes the loss and the gradient of the
 * parameter vector to HOST memory. Synchronous. No parameter update. */
int gs_upsampler_grads(gs_ctx *ctx, int32_t n, int32_t h, int32_t w, const float *rgb_lo,
                       const float *depth_lo, const float *rgb_hi, const float *depth_hi,
                       float *loss_out, float *grads_out, void *stream);

/* One optimisation step on given frames: forward + backward as
 * gs_upsampler_grads, then one Adam update of every parameter (Kingma & Ba:
 * beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected moments, the update
 * count kept in the context) at learning rate lr >= 0. *loss_out (HOST,
 * nullable) receives the loss before the update. Synchronous. */
int gs_upsampler_step(gs_ctx *ctx, int32_t n, int32_t h, int32_t w, const float *rgb_lo,
                      const float *depth_lo, const float *rgb_hi, const float *depth_hi,
                      float lr, float *loss_out, void *stream);

/* One Adam update (as in gs_upsampler_step) with a caller-given gradient:
 * grads HOST [n] in the parameter-vector layout, n =
 * gs_upsampler_num_params(). For optimising the network on gradients computed
 * elsewhere. Synchronous. */
int gs_upsampler_apply_grads(gs_ctx *ctx, const float *grads, int64_t n, float lr);

/* Adam state: first and second moments (HOST [n] each, nullable) in the
 * parameter-vector layout and the number of updates so far. Synchronous. */
int gs_upsampler_get_state(gs_ctx *ctx, float *m, float *v, int64_t n, int32_t *step);

/* Learning rate gs_upsampler_train uses at optimisation step `step` (0-based)
 * of `steps`: lr_min + (lr0 - lr_min) (1 + cos(pi step / (steps - 1))) / 2,
 * i.e. lr0 at the first step and lr_min at the last (lr0 when steps <= 1). */
float gs_upsampler_lr(int32_t step, int32_t steps, float lr0, float lr_min);

/* Fallback confidence score of n low-resolution frames (rgb_lo [n][h][w][3],
 * depth_lo [n][h][w] DEVICE): for the network input (r, g, b, depth/10), the
 * sum over channels of squared differences to the right and lower
 * neighbours (where they exist), divided by h w. score_out DEVICE [n].
 * Asynchronous on stream. gs_render_batch_upsampled scores its frames so. */
int gs_upsampler_score(gs_ctx *ctx, int32_t n, int32_t h, int32_t w, const float *rgb_lo,
                       const float *depth_lo, float *score_out, void *stream);

/* Train on n_pairs cameras (scene_ids HOST, poses / full-res intrinsics
 * DEVICE): every step renders `batch` cameras at width x height (targets)
 * and at width/4 x height/4 (inputs) with the batched renderer, runs the
 * network forward and backward and applies Adam at the learning rate
 * gs_upsampler_lr(step, steps, lr, lr_min) (lr_min 0 means lr / 20);
 * cameras are taken in order, wrapping around. loss_curve (HOST, `steps`
 * values, nullable) receives each step's loss. Synchronous. */
int gs_upsampler_train(gs_ctx *ctx, const gs_train_opts *opts, int32_t n_pairs,
                       const int32_t *scene_ids, const float *poses, const float *intrinsics,
                       int32_t width, int32_t height, float *loss_curve, void *stream);

/* Upsampled render: the batch is rendered at width/4 x height/4 (intrinsics
 * given for the full resolution), upsampled by the network, and every camera
 * whose confidence score (mean squared neighbour difference of its low-res
 * RGB + depth/10) exceeds fallback_threshold is rendered again at full
 * resolution into the same output slots. score_out (DEVICE [n], nullable)
 * receives the scores, *n_fallback_out (HOST, nullable) the number of
 * re-rendered cameras. width and height must be multiples of 4.
 * The cameras to re-render are chosen on the device: the full-resolution
 * render covers the whole batch under a per-camera mask, and a masked camera
 * projects no Gaussian and keeps the network's frame. With n_fallback_out
 * null the call is asynchronous on stream, like gs_render_batch (its two
 * renders follow the same first-render and capacity rules, and
 * gs_render_status reports their overflows); with it set the call waits for
 * the count. gs_last_stats afterwards describes the full-resolution
 * render. */
int gs_render_batch_upsampled(gs_ctx *ctx, int32_t n_cams, const int32_t *scene_ids,
                              const float *poses, const float *intrinsics, int32_t width,
                              int32_t height, float *rgb, float *depth, float *score_out,
                              float fallback_threshold, int32_t *n_fallback_out,
                              const gs_render_opts *opts, void *stream);

/* Per-frame PSNR in dB of RGB clamped to [0, 1]: a, b DEVICE [n][npix][3],
 * out DEVICE [n]. Asynchronous. */
int gs_frame_psnr(gs_ctx *ctx, int32_t n, int64_t npix, const float *a, const float *b,
                  float *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GS_H */

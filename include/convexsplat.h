/*
 * convexsplat.h — C ABI of the MI355X (gfx950) differentiable rasterizer for
 * smooth 3D convexes, after "3D Convex Splatting" (Held et al., CVPR 2025).
 *
 * Conventions for every entry point
 *   - Pointers to scene, image and gradient arrays are DEVICE pointers (HBM of
 *     the context's GPU); structs (cs_scene, cs_camera, cs_params, cs_grads)
 *     themselves live in host memory and are read during the call only.
 *   - All arrays are dense, row-major, with the shapes stated below; float32,
 *     except the scene arrays, which may also hold 16-bit values (cs_scene.dtype).
 *   - The caller owns every scene, image and gradient buffer; the library never
 *     frees them.  The library owns cs_ctx, cs_fwd_state and their workspace.
 *   - Work is enqueued on `hip_stream` (a hipStream_t; NULL = the null stream)
 *     in stream order.  cs_render_forward makes one host synchronisation: a
 *     4-byte read of the number of (convex, tile) pairs to size its buffers.
 *   - A context is used by one host thread and one stream at a time; separate
 *     contexts are independent.
 *   - Return value 0 = success, a negative CS_E* code otherwise; no exception
 *     crosses the ABI; cs_last_error() describes the last failure of the
 *     calling thread.
 *
 * Parameter conventions (paper, Sec. 3.2 and 3.3): a convex is K points p_k;
 * delta (smoothness), sigma (sharpness) and opacity are the ACTIVATED values
 * (delta > 0, sigma > 0, 0 <= opacity <= 1); colour is real spherical harmonics
 * of degree D <= 3, coefficients ordered (l, m) with m ascending.
 */
#ifndef CONVEXSPLAT_H
#define CONVEXSPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CS_OK 0
#define CS_EINVAL (-1)    /* bad shape, K, degree, camera, null pointer */
#define CS_ENOMEM (-2)    /* device allocation failed or HBM budget exceeded */
#define CS_EOVERFLOW (-3) /* a fixed-capacity buffer was too small */
#define CS_EHIP (-4)      /* HIP runtime error (message in cs_last_error) */
#define CS_EBUSY (-5)     /* serving queue full */
#define CS_ENODEV (-6)    /* no usable gfx950 device */

#define CS_MAX_K 8
#define CS_MAX_SH_DEGREE 3

/* Storage formats of the scene arrays (cs_scene.dtype).  The paper's light
 * model stores its convex parameters in 16-bit precision (Sec. 4.2,
 * Experimental Setup; Supp. Initialization & Hyperparameters); the kernels convert
 * every loaded value to float32 (exactly: both 16-bit formats are subsets of
 * float32) and compute as for float32 scenes, so a 16-bit scene renders
 * exactly like the float32 scene of the same values.  Gradients stay float32. */
#define CS_DTYPE_F32 0  /* IEEE binary32 */
#define CS_DTYPE_F16 1  /* IEEE binary16 */
#define CS_DTYPE_BF16 2 /* bfloat16: the upper half of a binary32 */

typedef struct cs_ctx cs_ctx;             /* device, workspace, tuning and serving state */
typedef struct cs_fwd_state cs_fwd_state; /* what the backward pass needs from a forward pass */

/* Pinhole camera (paper Sec. 3.2, Eq. projection q = K (R p + t) with the
 * homogeneous divide): R row-major world->camera, camera axes x right, y down,
 * z forward; fx, fy, cx, cy in pixels; pixel (u, v) is sampled at
 * (u + 0.5, v + 0.5).  A convex with any point at depth <= znear is dropped. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    float znear;
} cs_camera;

/* Scene (paper Sec. 3.2 point-set convexes; Sec. 3.3 optimised parameters).
 * The five arrays hold elements of the format `dtype` (CS_DTYPE_*), aligned
 * to their element size. */
typedef struct {
    int32_t n;          /* number of convexes, >= 0 */
    int32_t k;          /* points per convex, 3 <= k <= 8 */
    int32_t sh_degree;  /* 0 <= sh_degree <= 3 */
    const void *points;  /* [n][k][3] world space */
    const void *delta;   /* [n] smoothness, activated, > 0 */
    const void *sigma;   /* [n] sharpness, activated, > 0 */
    const void *opacity; /* [n] in [0, 1] */
    const void *sh;      /* [n][(sh_degree+1)^2][3] */
    int32_t dtype;       /* CS_DTYPE_F32 (0), CS_DTYPE_F16 or CS_DTYPE_BF16 */
} cs_scene;

/* Gradients, same shapes as the scene arrays, float32 whatever the scene's
 * dtype; OVERWRITTEN by the backward call. */
typedef struct {
    float *points, *delta, *sigma, *opacity, *sh;
} cs_grads;

/* cs_params.flags bits */
#define CS_FLAG_TIMING 1         /* record hipEvents around each stage on the call's stream (see cs_timing_read) */
#define CS_FLAG_LONGEST_FIRST 2  /* compositing takes tiles in order of decreasing list length (else natural) */
#define CS_FLAG_GRAPH 4          /* batched calls: capture into a hipGraph and replay (see cs_render_forward_batch) */
#define CS_FLAG_AUTOTUNE 8       /* batched calls with tile = 0: take tile, schedule and sort digits from the tuner */
#define CS_FLAG_DIGITS(b) (((b)&15) << 8) /* radix digit width of the pair sort, 4..8 (0 = 8) */

/* Stages timed under CS_FLAG_TIMING */
enum {
    CS_STAGE_PREPROCESS = 0, /* per-convex projection, hull, lines, colour, key, tile rectangle */
    CS_STAGE_DEPTH_SORT,     /* radix sort of the convexes by depth key */
    CS_STAGE_BIN_SCAN,       /* tile counts in depth order and their exclusive scan */
    CS_STAGE_EMIT,           /* (tile, convex) pair emission */
    CS_STAGE_TILE_SORT,      /* stable radix sort of the pairs by tile */
    CS_STAGE_RANGES,         /* per-tile list ranges */
    CS_STAGE_RENDER_FWD,     /* per-tile forward compositing */
    CS_STAGE_RENDER_BWD,     /* per-tile backward compositing */
    CS_STAGE_PREPROCESS_BWD, /* per-convex backward chain rule */
    CS_STAGE_ORDER,          /* longest-first tile order */
    CS_STAGE_GRAPH_FWD,      /* a replayed forward graph, whole */
    CS_STAGE_GRAPH_BWD,      /* a replayed backward graph, whole */
    CS_NUM_STAGES
};

/* Render parameters.  eps_alpha and t_min are part of the result's definition:
 * a (pixel, convex) pair with alpha < eps_alpha is skipped, and a pixel stops
 * after the convex that brings its transmittance below t_min.  tile = 0 picks
 * the default (16); supported: 8, 16, 32.  NULL = {1e-6, 1e-5, black, 0, 0}. */
typedef struct {
    float eps_alpha, t_min;
    float background[3];
    int32_t tile;
    int32_t flags;
} cs_params;

/* Library version as major*10000 + minor*100 + patch. */
int cs_version(void);

/* Thread-local description of the last failure of this thread ("" if none). */
const char *cs_last_error(void);

/* Create a context on HIP device `device`.  hbm_budget_bytes = 0 means no
 * limit; otherwise workspace growth beyond it fails with CS_ENOMEM. */
int cs_create(int device, size_t hbm_budget_bytes, cs_ctx **out);

/* Wait for the context's work, free its workspace and the context. */
int cs_destroy(cs_ctx *ctx);

/* Forward render (paper Sec. 3.2: projection, 2D hull, hull lines, distance-
 * scaled smooth indicator of Supp. B, SH colour, front-to-back compositing of
 * the compositing equation, convexes ordered by increasing depth).
 *   out_rgb: [height][width][3] device, written.
 *   state:   if non-NULL receives a new cs_fwd_state for cs_render_backward;
 *            release it with cs_state_release.  NULL = forward only.
 * The scene arrays must stay unchanged until the matching backward call. */
int cs_render_forward(cs_ctx *ctx, const cs_scene *scene, const cs_camera *cam, const cs_params *params,
                      float *out_rgb, cs_fwd_state **state, void *hip_stream);

/* Allocation-free forward render, for callers that cannot allocate device
 * memory (tight serving loops, harnesses that forbid hipMalloc): what
 * cs_render_forward computes with state = NULL, with every buffer of the pass
 * carved from one static device array of CS_NOALLOC_SCRATCH_BYTES that each
 * device holds from its first cs_create until the process ends.  The call
 * makes no device allocation or free; like cs_render_forward it waits for the
 * 4-byte pair count (read into pinned memory made by cs_create), so it cannot
 * be captured into a graph.
 *   out_rgb: [height][width][3] device, written.  Stream-ordered on hip_stream.
 *   Limits: the per-convex buffers (about 250 B per convex), the per-tile and
 *   per-pixel ones (about 30 B per pixel) and the (tile, convex) pairs (16 B
 *   each plus sort temporaries) must fit the array: 1M convexes at 1920x1080
 *   with about 9M pairs do.  Beyond it: CS_ENOMEM with the sizes in
 *   cs_last_error; a pair count found too large after the pass ran also
 *   returns CS_ENOMEM, and out_rgb is then unspecified.
 *   Every context on a device shares that device's array, which keeps the last
 *   call's contents: calls that overlap on one device (other streams, threads
 *   or contexts) race and their results are undefined. */
#define CS_NOALLOC_SCRATCH_BYTES ((size_t)512 << 20)
int cs_render_forward_noalloc(cs_ctx *ctx, const cs_scene *scene, const cs_camera *cam, const cs_params *params,
                              float *out_rgb, void *hip_stream);

/* Backward render: gradient of sum(dl_drgb * rgb) with respect to points,
 * delta, sigma, opacity and SH (paper Sec. 3.3 optimised parameters), through
 * every step of the forward pass ("fully differentiable", Sec. 3.2).
 *   dl_drgb: [height][width][3] device.  grads: overwritten device arrays.
 * scene, cam and params must be those of the forward call that made state. */
int cs_render_backward(cs_ctx *ctx, const cs_scene *scene, const cs_camera *cam, const cs_params *params,
                       const cs_fwd_state *state, const float *dl_drgb, cs_grads *grads, void *hip_stream);

/* Release a forward state (stream-ordered after the work that uses it). */
int cs_state_release(cs_ctx *ctx, cs_fwd_state *state);

/* Batched multi-view render: n_views (1..256) views of one scene in one pass
 * (paper Sec. 3.2 for each view).  All (view, convex) instances are
 * preprocessed in one grid and depth-sorted together; their (tile, instance)
 * pairs live in one global tile space and one persistent compositing grid
 * takes the tiles of every view from per-XCD work queues.
 *   cams:    host array of n_views cameras (resolutions may differ).
 *   out_rgb: host array of n_views DEVICE pointers, each [h_v][w_v][3].
 *   state:   as for cs_render_forward (required for the backward).
 * With CS_FLAG_GRAPH the context keeps the batch's buffers (sized from the
 * first frame's pair count plus a margin) and, from the second call on,
 * replays one captured hipGraph; cameras, resolutions (within the first
 * frame's tile and pixel totals) and output pointers may change between
 * replays, the scene arrays, n_views, K and the tuning may not (a change
 * re-captures).  A graph replay makes no host synchronisation; a frame whose
 * pairs exceed the capacity is reported by cs_batch_check or the backward call
 * as CS_EOVERFLOW (the buffers have then grown: render the frame again).  In
 * graph mode a context holds one batch state at a time: the next batched
 * forward invalidates the previous one. */
int cs_render_forward_batch(cs_ctx *ctx, const cs_scene *scene, int32_t n_views, const cs_camera *cams,
                            const cs_params *params, float *const *out_rgb, cs_fwd_state **state, void *hip_stream);

/* Backward of a batched forward: gradients summed over the views.
 *   dl_drgb: host array of n_views DEVICE pointers, each [h_v][w_v][3]. */
int cs_render_backward_batch(cs_ctx *ctx, const cs_scene *scene, int32_t n_views, const cs_camera *cams,
                             const cs_params *params, const cs_fwd_state *state, const float *const *dl_drgb,
                             cs_grads *grads, void *hip_stream);

/* Waits for a forward state's work; CS_EOVERFLOW if its pair buffer overflowed. */
int cs_batch_check(cs_ctx *ctx, const cs_fwd_state *state);

/* Autotuner: times the batched forward + backward for tile sizes {8, 16, 32},
 * tile schedules {natural, longest-first} and pair-sort digit widths {6, 8} on
 * the given scene and cameras, keeps the fastest in the context (keyed by
 * K, SH degree, views and the log2 buckets of convex and pixel counts) and
 * returns it.  Batched calls with tile = 0 and CS_FLAG_AUTOTUNE use it. */
typedef struct {
    int32_t tile, longest_first, digit_bits;
    float ms;          /* fwd + bwd time of the winner */
    float ms_default;  /* fwd + bwd time of tile 16, natural order, 8-bit digits */
} cs_tuning;
int cs_autotune(cs_ctx *ctx, const cs_scene *scene, int32_t n_views, const cs_camera *cams,
                const cs_params *params, cs_tuning *out, void *hip_stream);

/* Work counters of a forward state, copied to host (synchronises the stream):
 * n_pairs = (convex, tile) pairs binned; n_evaluated = (pixel, list entry)
 * pairs the forward walk tested; n_full = those that passed the max-line test
 * and evaluated the full indicator. */
int cs_state_stats(cs_ctx *ctx, const cs_fwd_state *state, int64_t *n_pairs, int64_t *n_evaluated,
                   int64_t *n_full);

/* All work counters of the last forward (and backward, when one ran) on a
 * state, summed over the compositing workgroups (synchronises the stream).
 * They price the compositing kernels against their roofline (the per-pair
 * work of Sec. 3.1 Eqs. smoothness/sharpness, T lines per pair):
 *   pairs       (tile, convex) pairs binned
 *   tested      (pixel, convex) pairs of the forward walk inside the record's pixel box
 *   full        of those, the pairs past the max-line test (LogSumExp and sigmoid evaluated)
 *   full_bwd    the same count in the backward walk, which visits the same pairs
 *               (0 before a backward)
 *   sum_T_full  sum of the hull size T over the backward's full pairs (mean T =
 *               sum_T_full / full_bwd)
 *   wave_evals  wavefront-level record evaluations of the backward walk (some lane
 *               full); lane utilisation = full_bwd / (64 wave_evals).  The forward
 *               walk makes the same evaluations; counting there would slow it. */
typedef struct {
    int64_t pairs, tested, full, full_bwd, sum_T_full, wave_evals;
} cs_work_counters;
int cs_state_counters(cs_ctx *ctx, const cs_fwd_state *state, cs_work_counters *out);

/* Debug/parity: per-convex preprocess results copied to host memory `out`,
 * an array of n cs_debug_convex records (synchronises the stream). */
typedef struct {
    int32_t status;     /* 0 visible, 1 culled (near plane), 2 culled (hull < 3), 3 never visible (opacity <= eps) */
    int32_t T;          /* hull size */
    int32_t hull[CS_MAX_K]; /* hull point indices, positive orientation, from min (y, x) */
    uint32_t depth_key; /* bits of the float32 depth key */
    int32_t clampmask;  /* bit c: colour channel c clamped at 0 */
    double A[CS_MAX_K], B[CS_MAX_K], C[CS_MAX_K]; /* L_j(q) = A_j qx + B_j qy + C_j, pixels, unit normal */
    double d, delta_p, sigma_p; /* depth, delta' = d delta, sigma' = d sigma */
    float rgb[3];
    int32_t tile_rect[4]; /* tx0, ty0, tx1, ty1 (inclusive); empty when tx0 > tx1 */
} cs_debug_convex;

int cs_debug_preprocess(cs_ctx *ctx, const cs_scene *scene, const cs_camera *cam, const cs_params *params,
                        cs_debug_convex *out, void *hip_stream);

/* Debug/parity: the depth-ordered per-tile convex lists of a forward state,
 * copied to host.  ranges: [n_tiles][2] (start, end); ids: [n_pairs]. */
int cs_debug_tile_lists(cs_ctx *ctx, const cs_fwd_state *state, int32_t *ranges, int64_t ranges_len,
                        int32_t *ids, int64_t ids_len);

/* ---------------------------------------------------------------- serving --
 * A request renders one view of a resident scene (paper Sec. 3.2, forward
 * only).  Requests queue on the host; worker threads, each with its own HIP
 * stream, take every queued request of the oldest request's scene (up to
 * max_batch, arrival order) as one batched forward pass as soon as a worker
 * is free.  Requests that arrive while others run join the next batch, and
 * batches on different workers overlap on the device.
 * Device memory: the passes run on frames (per-pass buffers) that the server
 * owns and its workers share; a batch reuses an idle frame of its scene,
 * grown when the batch exceeds it, so a steady request mix allocates nothing.
 * Every frame, idle or in use, counts against the budget: a batch that may
 * need more memory than the budget leaves waits, after the least recently
 * used idle frames of other scenes are freed, until running batches end (a
 * batch always runs when none other does).
 * A request's latency runs from cs_serve_submit to the completion of its batch
 * (host clock).  Its image equals a lone cs_render_forward of the same view. */
typedef struct {
    int32_t workers;        /* concurrent batches (streams), >= 1 */
    int32_t max_batch;      /* views per batch, 1..256 */
    int32_t max_queue;      /* queued requests before cs_serve_submit returns CS_EBUSY */
    int32_t start_paused;   /* 1: accept requests but run nothing until cs_serve_resume */
    size_t hbm_budget_bytes;/* 0 = the context's budget (0 there = unlimited) */
    cs_params params;       /* render parameters of every request */
} cs_serve_config;

typedef struct {
    int64_t submitted, completed, failed, batches;
    double mean_batch;      /* requests per batch */
    size_t peak_bytes;      /* largest device memory held by the server's frames */
    int64_t queued, running;
    int64_t frames_created; /* frames allocated (or re-created larger) so far */
    size_t frame_bytes;     /* device memory held by the frames now */
    double mean_queue_ms;   /* mean time from submit to the start of the request's batch */
    double mean_run_ms;     /* mean time from the start of the batch to its completion */
} cs_serve_stats;

/* Start the request loop of a context (one server per context). */
int cs_serve_start(cs_ctx *ctx, const cs_serve_config *config);
/* Let a paused server run. */
int cs_serve_resume(cs_ctx *ctx);
/* Finish running batches, fail queued requests, join the workers. */
int cs_serve_stop(cs_ctx *ctx);
/* Make a scene resident for serving; the caller keeps its arrays alive and
 * unchanged until cs_scene_unregister. */
int cs_scene_register(cs_ctx *ctx, const cs_scene *scene, int32_t *scene_id);
int cs_scene_unregister(cs_ctx *ctx, int32_t scene_id);
/* Queue one request (non-blocking).  out_rgb: DEVICE [h][w][3], written when
 * the request completes.  CS_EBUSY: queue full; CS_ENOMEM: the request alone
 * exceeds the budget; CS_EINVAL: unknown scene or bad camera. */
int cs_serve_submit(cs_ctx *ctx, int32_t scene_id, const cs_camera *cam, float *out_rgb, uint64_t *request_id);
/* Block until a request completes; latency_ms (host, nullable) from submit to
 * completion.  Returns the request's status (0, or the error of its batch). */
int cs_serve_wait(cs_ctx *ctx, uint64_t request_id, double *latency_ms);
int cs_serve_get_stats(cs_ctx *ctx, cs_serve_stats *stats);

/* Accumulated GPU time per stage (ms) and number of timed launches of it, over
 * the calls made with CS_FLAG_TIMING since the last reset; waits for the
 * pending events.  ms and count are host arrays of CS_NUM_STAGES (nullable). */
int cs_timing_read(cs_ctx *ctx, double *ms, int64_t *count, int reset);

/* Mean-absolute-error loss helper for a training step: writes
 * dl_drgb = sign(rgb - target) / (3 * height * width) and, if loss is
 * non-NULL (device, one float), accumulates the mean |rgb - target| into it. */
int cs_l1_loss_grad(cs_ctx *ctx, const float *rgb, const float *target, int32_t width, int32_t height,
                    float *dl_drgb, float *loss, void *hip_stream);

/* ------------------------------------------------ adaptive density control --
 * Splitting and pruning of the convex set between optimisation steps (paper
 * Sec. 3.3, "Adaptive convex shape refinement"; Supp. Initialization &
 * Hyperparameters).  The paper splits a convex whose sharpness-gradient
 * statistic ("loss of sigma") passes a threshold into K children, one centred
 * at each of its points, scaled down, with sigma raised and opacity lowered
 * (delta kept), and prunes convexes that are nearly transparent or too large.
 * Values marked "not stated" are not given by the paper: the caller chooses. */
typedef struct {
    float opacity_min;         /* prune when opacity < opacity_min (paper: 0.03) */
    float size_max;            /* prune when the radius max_k |p_k - c| > size_max, c the point mean
                                  (paper: 0.3 x the scene size) */
    float split_threshold;     /* split when accum / denom > split_threshold (denom > 0; paper: 4e-6) */
    float child_scale;         /* child k: points p_k + child_scale (p_j - c) (paper: 0.7 indoor, 0.6 outdoor) */
    float child_sigma_scale;   /* child sigma = sigma x this (paper: higher; factor not stated) */
    float child_opacity_scale; /* child opacity = opacity x this (paper: lower; factor not stated) */
} cs_densify_params;

/* Output arrays of cs_densify (DEVICE, float32, `capacity` convexes each, the
 * scene's shapes) and src[capacity] (int32): the input convex each output
 * convex comes from. */
typedef struct {
    float *points, *delta, *sigma, *opacity, *sh;
    int32_t *src;
} cs_scene_out;

/* After a backward pass: for every convex that reached at least one tile in
 * some view of `state`, accum[i] += |g_sigma[i]| and denom[i] += the number of
 * such views (DEVICE float arrays [n], caller-owned; the sharpness-gradient
 * statistic of the split criterion).  g_sigma: the gradient the caller's
 * optimiser sees for sigma (e.g. cs_grads.sigma, or its chain to a raw
 * parameter). */
int cs_densify_accumulate(cs_ctx *ctx, const cs_fwd_state *state, const float *g_sigma, float *accum, float *denom,
                          void *hip_stream);

/* Split and prune a float32 scene into `out`.  Decisions (in float32, in a
 * fixed order): prune if opacity < opacity_min or radius^2 > size_max^2;
 * else split if denom > 0 and accum / denom > split_threshold; else keep.
 * Output order: kept convexes in input order, then the K children of each
 * split convex in input order, child k centred at point k.  *n_out (host) is
 * the output count; when it exceeds `capacity` nothing is written and
 * CS_EOVERFLOW is returned (call again with capacity >= *n_out).  Synchronises
 * the stream once (the 8-byte count read-back).  CS_EINVAL for a 16-bit scene. */
int cs_densify(cs_ctx *ctx, const cs_scene *scene, const float *accum, const float *denom,
               const cs_densify_params *params, int64_t capacity, const cs_scene_out *out, int64_t *n_out,
               void *hip_stream);

/* Photometric loss of a training step (paper Sec. 3.3, Eq. loss, with
 * lambda = 0.2 there): L = (1 - lambda) mean|rgb - target| + lambda (1 - SSIM),
 * SSIM the mean over pixels and channels of the SSIM map with an 11x11
 * Gaussian window (sigma 1.5), zero padding, C1 = 0.01^2, C2 = 0.03^2 (the
 * 3DGS convention the paper follows).  Writes dl_drgb = dL/drgb ([h][w][3],
 * DEVICE) and ADDS L to *loss (DEVICE, one float; the caller zeroes it).  The
 * mask term of the equation belongs to a learnable-mask extension that this
 * rasterizer does not have.  Uses 36 bytes per pixel of stream-ordered scratch. */
int cs_ssim_loss_grad(cs_ctx *ctx, const float *rgb, const float *target, int32_t width, int32_t height, float lambda,
                      float *dl_drgb, float *loss, void *hip_stream);

/* ---------------------------------------------------------- optimiser step --
 * Adam on the raw (optimised) parameters (paper Sec. 3.3 "Initialization and
 * losses": opacity through a sigmoid, delta and sigma through an exponential;
 * the position learning rate decays exponentially, which the caller applies
 * through lr_points per step; Supp. Initialization & Hyperparameters gives the
 * rates).  grad holds dL/d(activated value), as cs_render_backward writes it;
 * the kernel chains it through the activation at the current raw value,
 * updates raw, m and v in place (torch.optim.Adam's arithmetic: m moves
 * towards g by 1 - beta1, v = beta2 v + (1 - beta2) g^2, step lr / (1 -
 * beta1^t), denominator sqrt(v) / sqrt(1 - beta2^t) + eps) and, when
 * `activated` is non-NULL, writes the activated values of the new raw
 * parameters (the scene arrays of the next render).  All arrays DEVICE
 * float32 with the scene's shapes; SH coefficient 0 of each channel takes
 * lr_sh_dc, the others lr_sh_rest. */
typedef struct {
    float *points, *delta, *sigma, *opacity, *sh;
} cs_param_set;

typedef struct {
    float lr_points, lr_delta, lr_sigma, lr_opacity, lr_sh_dc, lr_sh_rest;
    double beta1, beta2; /* double: 1 - beta is formed before rounding to float32 */
    float eps;
    int32_t step; /* 1-based step count of the bias corrections */
} cs_adam_params;

int cs_adam_step(cs_ctx *ctx, int32_t n, int32_t k, int32_t sh_degree, const cs_grads *grad, const cs_param_set *raw,
                 const cs_param_set *m, const cs_param_set *v, const cs_param_set *activated,
                 const cs_adam_params *params, void *hip_stream);

/* Initial convex set from a point cloud (paper Sec. 3.3 "Initialization and
 * losses"; Supp. Initialization & Hyperparameters): convex i has its k points
 * on a sphere round cloud point i, at the Fibonacci-sphere directions
 * (heights 1 - (2j + 1)/k, azimuths j x the golden angle pi (3 - sqrt 5)),
 * radius radius_scale x max(mean distance to the 3 nearest other cloud
 * points, radius_min) (fewer than 3 other points: the mean over those there
 * are).  delta, sigma, opacity take the given initial (activated) values; SH
 * coefficient 0 reproduces rgb (nullable: grey 0.5), the others are 0.
 * xyz, rgb: DEVICE [n][3]; out: DEVICE arrays of the scene's shapes.  The
 * neighbour search is exact and brute force: O(n^2). */
typedef struct {
    float radius_scale; /* paper: 1.2 */
    float radius_min;   /* floor of the mean distance (coincident cloud points) */
    float delta0, sigma0, opacity0; /* paper: 0.1, 0.00095, 0.1 */
} cs_init_params;

int cs_init_from_points(cs_ctx *ctx, int32_t n, const float *xyz, const float *rgb, int32_t k, int32_t sh_degree,
                        const cs_init_params *params, const cs_param_set *out, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif

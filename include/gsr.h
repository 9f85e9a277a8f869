/*
 * gsr.h -- C ABI of the differentiable tile-based Gaussian rasteriser for
 * gfx950 (MI355X).
 *
 * What the library computes (the hot path of Gaussian-splatting RGB-D SLAM):
 *   Gaussians (centre, rotation quaternion, per-axis scale, opacity, colour;
 *   Preliminaries, 3D Gaussian Splatting, eq. 1 and its anisotropic form
 *   Sigma = R S S^T R^T given in the Introduction) and, per view, a pinhole
 *   camera (Preliminaries, Visual Geometry Residual: pi_m with fx, fy, cx, cy)
 *   and a world-to-camera pose (R_cw, t_cw; same section) go in.  Out come:
 *     - the RGB image, eq. 2; the depth image, eq. 3; the silhouette, eq. 4
 *       (Proposed Approach, Pose Estimation), composited front to back after
 *       projecting each Gaussian with Sigma' = J W Sigma W^T J^T
 *       (Introduction);
 *     - the combined photometric + depth + silhouette (+ depth prior) L1 loss
 *       used for tracking and mapping (Abstract; Pose Estimation; depth priors
 *       in the Abstract and Conclusions);
 *     - its gradients to every Gaussian parameter (Scene Optimization) and to
 *       each camera pose, both as (q, t) and in the rotation-translation
 *       decoupled form (q with the camera centre C fixed, C) used by the
 *       decoupled pose update (Pose Estimation).
 *
 * Conventions that the paper leaves open (each is a fixed part of the ABI):
 *   - quaternions are (w, x, y, z) and need not be unit: the rotation is that
 *     of q/|q|, and gradients flow through the normalisation;
 *   - scale = exp(log_scale); opacity = sigmoid(opacity_logit); colour is used
 *     as given (no activation); the background is black;
 *   - pixel (u, v) is evaluated at the continuous image point (u, v);
 *   - the 2D covariance gets blur2d (px^2) added to its diagonal;
 *   - per pixel, alpha = min(0.99, o G); Gaussians with alpha < 1/255 are
 *     skipped; a Gaussian that would take the transmittance below 1e-4 ends
 *     the pixel and is not blended; Gaussians with camera depth <= z_near are
 *     culled; depth order is (float32 camera-frame z, Gaussian index);
 *   - the depth of a Gaussian (eq. 3) is its camera-frame z;
 *   - loss per view v with P_v pixels (L = sum over views):
 *       L_v = 1/P_v sum_p w(p) [ k(p) m(p) (w_rgb sum_c |C_c - C*_c|
 *                                            + w_depth |D - D*|)
 *                                + w_sil |S - S*|
 *                                + k(p) m_pr(p) w_prior |D - D_prior| ]
 *     with m = [D* > 0], m_pr = [D_prior > 0], w the optional per-pixel
 *     weight, k = [S > sil_mask_thresh] if sil_mask_thresh >= 0 else 1
 *     (a constant mask, no gradient), d|x|/dx = sign(x) with sign(0) = 0.
 *
 * Memory and ownership:
 *   - Every tensor pointer is a DEVICE pointer to contiguous float32 data
 *     unless stated.  Images of several views are concatenated: view v owns
 *     pixels [off_v, off_v + W_v H_v) of every per-pixel array (row-major,
 *     x fastest), where off_v is the running sum of W H over earlier views;
 *     RGB images are planar per view: channel c of view v starts at
 *     3 off_v + c W_v H_v.
 *   - The caller owns all memory: inputs, outputs and one workspace buffer
 *     whose size gsr_workspace_size() returns.  The library never allocates
 *     device memory.
 *   - Outputs are overwritten, never accumulated.  Gradient outputs with a
 *     NULL pointer are skipped.
 *   - The workspace carries the forward state (sorted tile lists, per-pixel
 *     final transmittance and last contributor) from gsr_forward() to
 *     gsr_backward(); it must not be reused in between.
 *   - All work is enqueued on `stream` (a hipStream_t; NULL = the null
 *     stream) and is stream-ordered.  Only these wait on the host:
 *     gsr_plan(), gsr_check_overflow(), gsr_read_counters(), gsr_read_work(),
 *     gsr_read_timing(), gsr_autotune() and calls made with GSR_SYNC.
 *     Inputs must stay valid until the work completes.
 *   - A gsr_ctx is not thread-safe: use one per host thread.
 *
 * Errors: every call returns a gsr_status.  Arguments are validated on the
 * host before any work is enqueued; on error nothing is enqueued and
 * gsr_last_error() describes the problem.  GSR_EHIP wraps a failing HIP call.
 * Pair capacity: the (Gaussian, tile) pairs of a call must fit the
 * workspace's pair capacity.  Their number is known only on the device, so
 *   - gsr_plan() runs the binning, waits, and returns the number needed
 *     (GSR_ECAPACITY if the workspace it was given cannot hold them);
 *   - with GSR_SYNC a render call waits after its binning and returns
 *     GSR_ECAPACITY, writing no output, if the pairs do not fit;
 *   - without GSR_SYNC (and always inside a graph) the call returns GSR_OK,
 *     its outputs are undefined on an overflow, and a device flag records
 *     it: gsr_check_overflow() (or gsr_read_counters()) reads it afterwards,
 *     and the caller re-plans with a larger workspace.
 */
#ifndef GSR_H
#define GSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gsr_ctx gsr_ctx;

typedef enum {
    GSR_OK = 0,
    GSR_EINVAL = -1,       /* invalid argument (nothing was enqueued) */
    GSR_ENOMEM = -2,       /* workspace too small for this call */
    GSR_ECAPACITY = -3,    /* pair capacity exceeded (gsr_plan, GSR_SYNC, gsr_check_overflow) */
    GSR_EHIP = -4,         /* a HIP runtime call failed; gsr_last_error() has its text */
    GSR_EUNSUPPORTED = -5  /* e.g. more than GSR_MAX_VIEWS views in one call */
} gsr_status;

#define GSR_MAX_VIEWS 64

/* option flags */
#define GSR_ISOTROPIC      0x1u  /* log_scales is [N,1]: one scale for all axes (eq. 1) */
#define GSR_NO_GAUSS_GRADS 0x2u  /* skip gradients to the Gaussians (pose-only tracking) */
#define GSR_NO_POSE_GRADS  0x4u  /* skip gradients to the poses (mapping) */
#define GSR_COUNT_WORK     0x8u  /* count blend work (gsr_read_work); costs a little time */
#define GSR_PIXEL_HASH     0x10u /* the forward also writes the per-pixel decision hash that
                                    gsr_debug_pixel_state reports (test hook; 0 without it) */
#define GSR_POSE_CENTRE    0x20u /* views->trans holds each camera's centre C in world
                                    coordinates instead of t: X_c = R(q) (X_w - C).  The
                                    decoupled gradients dq_c, dc are then the gradients of the
                                    pose inputs (Pose Estimation: rotation and translation
                                    updated apart).  Not accepted by the tracking loop. */
#define GSR_SYNC           0x40u /* the call waits for its binning and returns GSR_ECAPACITY
                                    (no output written) if the pairs exceed the workspace's
                                    capacity; not allowed inside a graph capture */
#define GSR_DETERMINISTIC  0x80u /* gradients bit-reproducible run to run: each (tile, list
                                    entry) writes its partials to a row of its own and every
                                    Gaussian sums its rows in a fixed order.  Without it the
                                    backward sums each entry over a tile's pixels (wave and
                                    workgroup reductions) and adds the sums to the Gaussian's
                                    row with global float atomics, whose order varies (results
                                    differ in the last bits).  A gsr_backward() must use the
                                    flag of the gsr_forward() it follows. */

/* stages reported by gsr_read_timing() */
#define GSR_STAGE_BINNING     0  /* projection, compaction, depth sort, records, pairs, tile sort, ranges */
#define GSR_STAGE_BLEND_FWD   1  /* front-to-back compositing (eqs. 2-4) */
#define GSR_STAGE_BLEND_BWD   2  /* loss + reverse compositing -> 2D gradients per record (one kernel) */
#define GSR_STAGE_PROJECT_BWD 3  /* chain rule to the parameters, pose gradients */
#define GSR_NUM_STAGES        4

/* Pinhole camera pi_m (Preliminaries, Visual Geometry Residual).  Host memory. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
} gsr_camera;

/* The Gaussian map (eq. 1 and its anisotropic form).  Device pointers, raw
 * (unactivated) parameters: means [N,3] world metres; quats [N,4] (w,x,y,z);
 * log_scales [N,3] ([N,1] with GSR_ISOTROPIC); opacity_logits [N]; rgb [N,3].
 * With GSR_ISOTROPIC, quats is not read and may be NULL. */
typedef struct {
    int64_t n;
    const float *means, *quats, *log_scales, *opacity_logits, *rgb;
} gsr_gaussians;

/* Views: n_views cameras (host array) and world-to-camera poses (device):
 * quat [V,4] (w,x,y,z, any norm) and trans [V,3], X_c = R(q) X_w + t (with
 * GSR_POSE_CENTRE, trans is the camera centre C and X_c = R(q) (X_w - C)). */
typedef struct {
    int32_t n_views;
    const gsr_camera *cams;
    const float *quat, *trans;
} gsr_views;

typedef struct {
    float w_rgb, w_depth, w_sil, w_prior;  /* loss weights */
    float z_near;                          /* near-plane cull (camera-frame z, metres) */
    float blur2d;                          /* added to the 2D covariance diagonal (px^2), >= 0 */
    float sil_mask_thresh;                 /* < 0: off; else photometric/depth terms need S > thresh */
    int32_t tile_w, tile_h;                /* binning tile in pixels: each 8, 16 or 32; 0 and 0 = the tile
                                              gsr_autotune() chose for this input shape, else 16x16 */
    uint32_t flags;                        /* GSR_* flags */
} gsr_options;

/* Loss targets (device, concatenated like the images).  rgb [3*sumP] planar
 * per view and depth [sumP] are required; sil, prior and weight may be NULL
 * (a NULL sil target means S* = 0, a NULL prior disables the prior term, a
 * NULL weight means 1 everywhere). */
typedef struct {
    const float *rgb, *depth, *sil, *prior, *weight;
} gsr_targets;

/* Rendered images (device): rgb [3*sumP] planar per view, depth [sumP], sil [sumP]. */
typedef struct {
    float *rgb, *depth, *sil;
} gsr_images;

/* Gradients to the raw Gaussian parameters, laid out like gsr_gaussians
 * (device; NULL = skip that group). */
typedef struct {
    float *means, *quats, *log_scales, *opacity_logits, *rgb;
} gsr_gaussian_grads;

/* Pose gradients (device; NULL = skip): dq_t [V,4] = dL/dq with t fixed,
 * dt [V,3] = dL/dt, dq_c [V,4] = dL/dq with the camera centre C = -R^T t
 * fixed, dc [V,3] = dL/dC. */
typedef struct {
    float *dq_t, *dt, *dq_c, *dc;
} gsr_pose_grads;

/* Caller-owned device workspace. */
typedef struct {
    void *ptr;
    size_t bytes;
    int64_t pair_capacity;   /* (Gaussian, tile) pairs it was sized for */
} gsr_workspace;

/* Create a context on HIP device `device`.  Returns GSR_EHIP if the device
 * cannot be queried. */
gsr_status gsr_create(gsr_ctx **out, int device);

/* Destroy a context (NULL is allowed). */
void gsr_destroy(gsr_ctx *ctx);

/* Text of the last error on ctx; valid until the next call on ctx.  A NULL
 * ctx gives the text of the last failed gsr_create(). */
const char *gsr_last_error(const gsr_ctx *ctx);

/* Bytes of workspace needed for n Gaussians, these views (only the cameras
 * are read) and pair_capacity (Gaussian, tile) pairs.  Needs no device: ctx
 * may be NULL, and then an error's text is what gsr_last_error(NULL) returns. */
gsr_status gsr_workspace_size(gsr_ctx *ctx, int64_t n, const gsr_views *views, const gsr_options *opts,
                              int64_t pair_capacity, size_t *bytes);

/* Forward pass (eqs. 2-4): project, bin, sort and composite every view into
 * `out`.  Keeps the state that gsr_backward() needs in the workspace. */
gsr_status gsr_forward(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_views *views, const gsr_options *opts,
                       gsr_workspace ws, gsr_images out, void *stream);

/* Backward pass of gsr_forward(): given dL/d(rgb, depth, sil) images
 * (device, laid out like the images; any may be NULL = zero), writes the
 * gradients to the Gaussians and to the poses.  `out` must hold the images
 * gsr_forward() wrote, and ws the state it left. */
gsr_status gsr_backward(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_views *views, const gsr_options *opts,
                        gsr_workspace ws, gsr_images out, const float *g_rgb, const float *g_depth,
                        const float *g_sil, gsr_gaussian_grads *gg, gsr_pose_grads *pg, void *stream);

/* Forward, loss and backward in one call (the tracking/mapping step):
 * renders into `out`, writes the loss to loss[V + 1] (device, float64,
 * overwritten): the per-view losses loss[0..V-1], then their sum in view
 * order, loss[V] (the total the combined objective minimises), and the
 * gradients of that total. */
gsr_status gsr_render_loss_grad(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_views *views,
                                const gsr_options *opts, const gsr_targets *targets, gsr_workspace ws,
                                gsr_images out, double *loss, gsr_gaussian_grads *gg, gsr_pose_grads *pg,
                                void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): gsr_render_loss_grad()
 * with no workspace argument.  The library uses a static scratch of 128 MiB
 * per device instead, a device array held by the loaded module until the
 * process ends; the call allocates nothing (no device memory, no events).
 * The pair capacity is the largest whose layout fits the scratch.  Other
 * arguments and outputs as in gsr_render_loss_grad().  `used` (host, may be
 * NULL) receives the workspace the call used (the scratch's device address,
 * its size and that capacity), to pass to gsr_check_overflow() or
 * gsr_read_counters() afterwards: an overflow leaves the outputs undefined
 * as on the asynchronous path.  The scratch is shared by every call on the
 * device and keeps the last call's contents (each call clears what it
 * needs), so calls that overlap on one device, on different streams or host
 * threads, race.  Returns GSR_ENOMEM if the call needs more than the scratch
 * before any pair (too many views x Gaussians or pixels: use a workspace),
 * GSR_EINVAL with GSR_SYNC, GSR_EUNSUPPORTED if the device has no scratch
 * (ordinal 64 or above). */
gsr_status gsr_render_loss_grad_noalloc(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_views *views,
                                        const gsr_options *opts, const gsr_targets *targets, gsr_images out,
                                        double *loss, gsr_gaussian_grads *gg, gsr_pose_grads *pg, void *stream,
                                        gsr_workspace *used);

/* Tile autotuner.  Runs the fused call of gsr_render_loss_grad() (same
 * arguments; opts' tile is ignored) with each candidate tile size (16x16,
 * 16x8, 8x16, 8x8, 32x32, 32x16, 16x32) that fits ws, checks each once against the pair capacity
 * (a synchronisation), times `reps` calls of each with HIP events, and keeps
 * the fastest for this input shape (the views' resolutions, N rounded up to a
 * power of two, the flags); later calls with tile 0x0 use it.  Writes the
 * choice to best_tile[2] (host) and its time per call to *ms_per_call (host).
 * Outputs hold the last candidate's results (every tile gives the same
 * images).  GSR_ECAPACITY if no candidate fits the workspace. */
gsr_status gsr_autotune(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_views *views, const gsr_options *opts,
                        const gsr_targets *targets, gsr_workspace ws, gsr_images out, double *loss,
                        gsr_gaussian_grads *gg, gsr_pose_grads *pg, int32_t reps, int32_t *best_tile,
                        double *ms_per_call, void *stream);

/* Sets the tile used for an input shape (as gsr_autotune() would), e.g. from
 * a cache of earlier tuning runs.  n, views (cameras only) and flags form the
 * shape key. */
gsr_status gsr_set_tile(gsr_ctx *ctx, int64_t n, const gsr_views *views, uint32_t flags, int32_t tile_w,
                        int32_t tile_h);

/* HIP graph capture of one gsr_render_loss_grad() call (same arguments) on
 * `stream` (not the null stream).  Every pointer is baked into the graph:
 * inputs, outputs and the workspace must stay allocated and in place for as
 * long as the graph is launched; their contents may change between launches.
 * The pair capacity is checked only on the device: after launches, use
 * gsr_read_counters() to detect an overflow (then re-plan and re-capture).
 * Returns an id for gsr_graph_launch() / gsr_graph_destroy(). */
gsr_status gsr_graph_capture(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_views *views, const gsr_options *opts,
                             const gsr_targets *targets, gsr_workspace ws, gsr_images out, double *loss,
                             gsr_gaussian_grads *gg, gsr_pose_grads *pg, void *stream, int32_t *graph_id);
gsr_status gsr_graph_launch(gsr_ctx *ctx, int32_t graph_id, void *stream);
gsr_status gsr_graph_destroy(gsr_ctx *ctx, int32_t graph_id);

/* Synchronises `stream` and reads the counters of the last call on ws:
 * visible (view, Gaussian) records, (Gaussian, tile) pairs needed, and
 * whether the pair capacity overflowed (then outputs are undefined).  Any
 * of the three pointers may be NULL. */
gsr_status gsr_read_counters(gsr_ctx *ctx, gsr_workspace ws, void *stream, int64_t *n_visible, int64_t *n_pairs,
                             int32_t *overflow);

/* The capacity check of the asynchronous paths (graph launches, calls
 * without GSR_SYNC): synchronises `stream`, sets *overflowed (host) to 1 if
 * the last call on ws -- or any iteration of the last tracking or mapping
 * loop on it -- needed more pairs than the workspace holds, and then
 * returns GSR_ECAPACITY (re-plan with gsr_plan and a larger workspace);
 * GSR_OK and 0 otherwise. */
gsr_status gsr_check_overflow(gsr_ctx *ctx, gsr_workspace ws, void *stream, int32_t *overflowed);

/* Plans a call: runs its projection and binning on `stream` (same g, views
 * and opts as the call; ws may have any pair capacity, 0 included), waits,
 * and writes the number of (Gaussian, tile) pairs the call needs to
 * *pairs_needed (host).  Returns GSR_ECAPACITY (with *pairs_needed set) if
 * ws cannot hold them.  Not allowed inside a graph capture. */
gsr_status gsr_plan(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_views *views, const gsr_options *opts,
                    gsr_workspace ws, int64_t *pairs_needed, void *stream);

/* Work counters of the last call on ws made with GSR_COUNT_WORK (synchronises
 * `stream`): work[0] (pixel, entry) alpha evaluations in the forward blend,
 * work[1] contributions (alpha >= 1/255, before termination) in the forward,
 * work[2], work[3] the same in the backward blend, work[4] (wave, entry)
 * gradient reductions in the backward, work[5] the backward's work items (one
 * per tile, plus one per extra chunk of a list split across workgroups; set
 * by every call).  Host array of 6. */
gsr_status gsr_read_work(gsr_ctx *ctx, gsr_workspace ws, void *stream, int64_t *work);

/* Per-stage timing with HIP events: while enabled, every call brackets each
 * stage's launches with events on its stream.  gsr_read_timing() waits for
 * the recorded events and returns, per stage (GSR_STAGE_*), the summed
 * milliseconds and the number of timed launches since the last read (host
 * arrays of GSR_NUM_STAGES), then clears them.  Timing must stay off while a
 * stream is being captured into a graph. */
gsr_status gsr_set_timing(gsr_ctx *ctx, int32_t enable);
gsr_status gsr_read_timing(gsr_ctx *ctx, double *ms, int64_t *launches);

/* Test hook for the binning step: copies out the state that the last
 * gsr_forward() or gsr_render_loss_grad() left in ws (same g, views, opts;
 * device destinations, enqueued on stream).  rec_gid [M]: view*N+i of each
 * visible record in depth order; rec_xy [M,2]: its float32 screen mean (the
 * leading float32 part); rec_radius [M]: its float32 binning radius; rec_z
 * [M]: its float32 camera depth; ranges [T,2]: [start, end) of every tile's
 * list in the sorted pairs (tiles of all views, view by view, row-major
 * within a view); pair_rec [K]: record index of every sorted pair.  Entries
 * beyond max_rec, max_tiles and max_pairs are not written. */
gsr_status gsr_debug_binning(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_views *views, const gsr_options *opts,
                             gsr_workspace ws, int64_t max_rec, int64_t max_tiles, int64_t max_pairs,
                             uint32_t *rec_gid, float *rec_xy, float *rec_radius, float *rec_z, uint32_t *ranges,
                             uint32_t *pair_rec, void *stream);

/* Test hook: copies the per-pixel state that the last forward on ws left
 * (device destinations of sumP entries each, any may be NULL; enqueued on
 * stream): the final transmittance, the list position + 1 of the last
 * contributing entry, and a hash of the pixel's decisions (which records
 * contributed, in order, which had their alpha clamped at 0.99, and whether
 * the transmittance cut-off ended the pixel; written only by a forward with
 * GSR_PIXEL_HASH, 0 otherwise).  Equal hashes under a small
 * parameter change mean the images moved smoothly there, which is what a
 * finite-difference check of the gradients needs. */
gsr_status gsr_debug_pixel_state(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_views *views,
                                 const gsr_options *opts, gsr_workspace ws, float *t_final, uint32_t *n_last,
                                 uint32_t *hash, void *stream);

/* Self test of the wave64 primitives the kernels rely on (cross-lane sums,
 * ballots, lane ranks): writes the number of failed checks to *failures
 * (device int32), enqueued on stream.  0 is expected. */
gsr_status gsr_selftest(gsr_ctx *ctx, int32_t *failures, void *stream);

/* ======================================================================
 * Optimisation steps around the rasteriser (tracking, mapping, map growth).
 * Everything below runs on the device from device state: a whole tracking
 * or mapping loop is enqueued without host round trips and can be captured.
 * ====================================================================== */

/* Pose update of tracking.  The paper estimates the pose by gradient-based
 * optimisation of the render loss, updating rotation and translation
 * separately (tracking section: a rotation-translation decoupled strategy)
 * but gives no update rule.  This library makes, per iteration and view,
 * one Adam step (Kingma & Ba 2015, with bias correction) on the raw
 * quaternion q with dL/dq at a fixed camera centre, and one on the camera
 * centre C = -R^T t with dL/dC, then sets t = -R(q/|q|) C.  The state is
 * FP64 on the device; the pose the renderer reads is its FP32 rounding. */
typedef struct gsr_pose_adam {
    float lr_rot;  /* step size of the quaternion components */
    float lr_pos;  /* step size of the camera centre (metres) */
    float beta1, beta2, eps;
} gsr_pose_adam;

/* Doubles of optimiser state per view: q 4, C 3, m_q 4, v_q 4, m_C 3, v_C 3,
 * step 1, beta1^step 1, beta2^step 1 (the bias corrections' powers). */
#define GSR_POSE_STATE_DOUBLES 24

/* Starts the state of n_views poses (device quat [V,4], trans [V,3]) in
 * `state` (device, GSR_POSE_STATE_DOUBLES * n_views doubles): C = -R^T t,
 * zero moments, step 0.  EINVAL on NULL pointers or n_views outside
 * [1, GSR_MAX_VIEWS]. */
gsr_status gsr_pose_opt_init(gsr_ctx *ctx, int32_t n_views, const float *quat, const float *trans, double *state,
                             void *stream);

/* One step from the decoupled gradients dq_c [V,4] and dc [V,3] (device, as
 * written by the backward); rewrites quat and trans (device) from the new
 * state. */
gsr_status gsr_pose_opt_step(gsr_ctx *ctx, int32_t n_views, const float *dq_c, const float *dc,
                             const gsr_pose_adam *hp, double *state, float *quat, float *trans, void *stream);

/* The tracking loop: `iters` times render + loss + pose gradients
 * (gsr_render_loss_grad with GSR_NO_GAUSS_GRADS, at the tile shape resolved
 * as there), then gsr_pose_opt_step, all enqueued on `stream`.  quat/trans
 * (device) hold the start pose and receive the optimised one; `state` must
 * have been started by gsr_pose_opt_init.  pg must provide dq_c and dc
 * (scratch for every iteration; dq_t and dt are optional).  loss [V + 1] holds
 * the last iteration's loss; loss_hist (device, optional) receives every
 * iteration's, [iters, V].  After the loop, gsr_read_counters reports an
 * overflow if the pair capacity was exceeded in any iteration. */
gsr_status gsr_track(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams, int32_t n_views, float *quat,
                     float *trans, const gsr_options *opts, const gsr_targets *targets, gsr_workspace ws,
                     gsr_images out, double *loss, gsr_pose_grads *pg, const gsr_pose_adam *hp, double *state,
                     int32_t iters, double *loss_hist, void *stream);

/* gsr_track captured into one graph (replayed with gsr_graph_launch; every
 * replay continues from the state and pose it finds). */
gsr_status gsr_track_capture(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams, int32_t n_views,
                             float *quat, float *trans, const gsr_options *opts, const gsr_targets *targets,
                             gsr_workspace ws, gsr_images out, double *loss, gsr_pose_grads *pg,
                             const gsr_pose_adam *hp, double *state, int32_t iters, double *loss_hist, void *stream,
                             int32_t *graph_id);

/* Mapping step (scene optimisation section: the map's Gaussian parameters
 * are refined by gradient-based optimisation with the poses fixed): Adam
 * over every raw parameter array, each with its own step size. */
typedef struct gsr_map_adam {
    float lr_means, lr_quats, lr_log_scales, lr_opacity, lr_rgb;
    float beta1, beta2, eps;
} gsr_map_adam;

/* Mutable parameter arrays (device), layout as gsr_gaussians. */
typedef struct gsr_gaussians_rw {
    int64_t n;
    float *means, *quats, *log_scales, *opacity_logits, *rgb;
} gsr_gaussians_rw;

/* Bytes of mapping optimiser state for n Gaussians: a 256-byte header
 * (step count) and the two moment arrays, each segment 256-byte aligned. */
size_t gsr_map_state_size(int64_t n, int32_t isotropic);

/* Zeroes the state (device, gsr_map_state_size bytes). */
gsr_status gsr_map_opt_init(gsr_ctx *ctx, int64_t n, int32_t isotropic, void *state, void *stream);

/* One Adam step: params -= f(grads) in place, moments and step updated in
 * `state`.  grads is laid out as params (for example the output of
 * gsr_backward); a NULL array in params is skipped (its gradient must then
 * be NULL too).  FP32 arithmetic.  With isotropic, quats may be NULL. */
gsr_status gsr_map_opt_step(gsr_ctx *ctx, gsr_gaussians_rw params, const gsr_gaussian_grads *grads,
                            int32_t isotropic, const gsr_map_adam *hp, void *state, void *stream);

/* The mapping loop: `iters` times render + loss + gradients to every
 * Gaussian parameter over `views` (a window of keyframes, poses fixed: pose
 * gradients are not formed), then gsr_map_opt_step on `params` in place, all
 * enqueued on `stream`.  gg receives each iteration's gradients (scratch;
 * laid out as params).  loss [V + 1] holds the last iteration's loss (per view,
 * then the total); loss_hist
 * (device, optional) receives every iteration's, [iters, V].  `state` must
 * have been started by gsr_map_opt_init.  EINVAL with GSR_NO_GAUSS_GRADS.
 * After the loop, gsr_read_counters reports an overflow if the pair
 * capacity was exceeded in any iteration. */
gsr_status gsr_map_iterate(gsr_ctx *ctx, gsr_gaussians_rw params, const gsr_views *views, const gsr_options *opts,
                           const gsr_targets *targets, gsr_workspace ws, gsr_images out, double *loss,
                           gsr_gaussian_grads *gg, const gsr_map_adam *hp, void *state, int32_t iters,
                           double *loss_hist, void *stream);

/* gsr_map_iterate captured into one graph (replayed with gsr_graph_launch;
 * every replay continues from the parameters and state it finds). */
gsr_status gsr_map_capture(gsr_ctx *ctx, gsr_gaussians_rw params, const gsr_views *views, const gsr_options *opts,
                           const gsr_targets *targets, gsr_workspace ws, gsr_images out, double *loss,
                           gsr_gaussian_grads *gg, const gsr_map_adam *hp, void *state, int32_t iters,
                           double *loss_hist, void *stream, int32_t *graph_id);

/* New Gaussians from one RGB-D frame (initialisation section: one Gaussian
 * per pixel at the point unprojected with the pixel's depth, with the
 * pixel's colour, opacity 0.5 and a radius of one pixel, depth / focal
 * length, with f = (fx + fy) / 2; identity rotation).  A pixel qualifies if
 * its depth is > 0 and, when sil is given (the rendered silhouette of the
 * map at this pose), sil < sil_thresh: the regions the map does not cover
 * yet.  Pixels are taken in raster order; the k-th qualifying one is
 * written to row offset + k of `out` if that row is < capacity (out.n is
 * not read).  *n_new (device int64) receives the number of qualifying
 * pixels, written or not (-1 if an internal wait gave up: never expected).
 * quat [4], trans [3] (device) give the frame's world-to-camera pose;
 * rgb [3,H*W] planar, depth [H*W], sil [H*W] or NULL (device).  `work`
 * (device, gsr_densify_work_size bytes) is scratch. */
size_t gsr_densify_work_size(int32_t width, int32_t height);
gsr_status gsr_densify(gsr_ctx *ctx, gsr_camera cam, const float *quat, const float *trans, const float *rgb,
                       const float *depth, const float *sil, float sil_thresh, gsr_gaussians_rw out,
                       int32_t isotropic, int64_t offset, int64_t capacity, int64_t *n_new, void *work,
                       size_t work_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* GSR_H */

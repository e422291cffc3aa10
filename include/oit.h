/*
 * liboit — sort-free order-independent-transparency (OIT) Gaussian-splat renderer
 * for AMD Instinct MI355X (gfx950): forward, backward, active-set selection and a
 * sparse Adam step, as hand-written HIP kernels behind a plain C ABI.
 *
 * The method is SparseOIT (arXiv 2605.13855):
 *   - weighted OIT composite  C = T c0 + (1 - T) P / Q,  T = prod_i (1 - alpha_i),
 *     P = sum_i c_i alpha_i w_i,  Q = sum_i alpha_i w_i      (Sec. 3.2, Eq. "oit_rendering");
 *   - per-splat weight w = max(0, 1 - d / sigma) v(r), sigma a learnable scene scalar,
 *     v a single-channel degree-3 SH                            (Sec. 1, Eq. "sf_weight";
 *                                                               Sec. 5.1 "Implementation Details");
 *   - rasteriser that bins splats into screen tiles and sorts entries by tile only,
 *     no depth sort; one pass blends the active splats and normalises ("BAN") and
 *     updates the pre-rendered buffer of the inactive set ("BAU")     (App. A, Alg. "rasterize");
 *   - closed-form partials dC/dc, dC/dalpha, dC/dw              (App. B, Eq. "oit_rendering_detail");
 *   - active set: a splat is active if some attribute group's gradient is large
 *     (Sec. 4.1, Eq. "activeness"); only active splats are rendered against the
 *     pre-rendered image of the others and updated by Adam   (Sec. 4.1, Alg. "Active Set Method").
 *
 * Conventions for every entry point
 *   - Pointers are DEVICE pointers unless marked (host).
 *   - Splat parameters (and Adam's moments) are float32, splat-major: a group with C
 *     components is an [n][C] array (splat i's components at offset i * C), so the rows
 *     of a sparse active set are read and written in whole segments.  The colour SH is
 *     [n][16][3] (splat, coefficient, channel); quaternions are (w, x, y, z), any
 *     length.  quat, sh and vsh start on 16-byte boundaries (vector loads).
 *   - Gradients of active rows are compact and component-major: a group with C
 *     components is a [C][stride] array whose column r is active row r.
 *   - Per-view images are planar float32.  A batch of V views is packed view after
 *     view: view k starts at plane offset P * pix_base(k), pix_base(k) = sum_{j<k} H_j W_j,
 *     and holds P planes of H_k x W_k (P = 3 for images, OIT_PIXSTATE_PLANES = 6 for
 *     pixstate, 9 for pre).
 *   - Pixel (x, y) has its centre at (x + 0.5, y + 0.5); cameras are pinhole, OpenCV
 *     axes (+x right, +y down, +z forward), x_cam = R x_world + t.
 *   - The caller owns all memory (inputs, outputs and the workspace).  The library
 *     never allocates, frees or synchronises inside these calls; all work is enqueued
 *     on `stream`, so every call can be captured into a HIP graph.
 *   - Errors: invalid arguments are detected on the host and returned synchronously
 *     (OIT_ERR_INVALID, nothing is enqueued); a HIP launch error returns OIT_ERR_HIP.
 *     Data-dependent capacity overflows (more tile entries, active rows or label
 *     changes than the buffers hold) cannot be seen on the host: the kernels bound
 *     every write, set a bit in the device status word of the workspace and the
 *     results of that call are incomplete; read it with oit_read_status.
 *     oit_last_error() returns a message for the last failing call on this thread.
 *   - NaN inputs propagate; there are no device-side checks of values.
 */
#ifndef OIT_H
#define OIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *oit_stream; /* a hipStream_t */

/* planes per pixel of the forward pass's state (T, Q, F rgb, dQ/dsigma) */
#define OIT_PIXSTATE_PLANES 6

typedef enum {
    OIT_OK = 0,
    OIT_ERR_INVALID = -1,
    OIT_ERR_HIP = -2,
    OIT_ERR_CAPACITY = -3,
    OIT_ERR_WORKSPACE = -4
} oit_status;

/* bits of the device status word */
#define OIT_STATUS_PAIR_OVERFLOW 1   /* tile entries exceeded tuning.pair_capacity */
#define OIT_STATUS_ACTIVE_OVERFLOW 2 /* selection produced more rows than active capacity */
#define OIT_STATUS_DELTA_OVERFLOW 4  /* more label changes than delta capacity */

#define OIT_MAX_VIEWS 64

typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy; /* pixels */
    float R[9];           /* world -> camera rotation, row-major */
    float t[3];
    float near_z;         /* splats with camera-space depth <= near_z are culled (0.2) */
} oit_camera;             /* (host) */

typedef struct {
    int64_t n;
    const float *mean;          /* [n][3] */
    const float *log_scale;     /* [n][3]   scale = exp(log_scale) */
    const float *quat;          /* [n][4]   (w, x, y, z); 16-byte aligned */
    const float *opacity_logit; /* [n]      opacity = sigmoid(logit) */
    const float *sh;            /* [n][16][3] colour SH, degree 3; 16-byte aligned */
    const float *vsh;           /* [n][16]  view-weight SH, degree 3; 16-byte aligned */
} oit_splats;

/* Gradients of the active rows, compact: row r of a group is the r-th entry of
 * active_idx (or splat r in dense mode); group with C components is [C][stride]. */
typedef struct {
    float *mean, *log_scale, *quat, *opacity_logit, *sh, *vsh;
    int64_t stride;
} oit_grads;

#define OIT_BWD_PER_SPLAT 0 /* one splat per lane over its tile's pixels (Sec. 4.2) */
#define OIT_BWD_PER_PIXEL 1 /* one pixel per thread, an atomic per contributing pair
                               (the 3DGS baseline of Tab. "ablation", for comparison) */

typedef struct {
    int32_t tile;           /* tile edge in pixels: 8, 16 or 32 */
    int32_t batch;          /* splat records staged in LDS per forward batch: 32..256 */
    int64_t pair_capacity;  /* capacity of the (tile, splat) entry list */
    int32_t bwd_mode;       /* OIT_BWD_PER_SPLAT (default) or OIT_BWD_PER_PIXEL */
    int32_t reserved;       /* 0 */
} oit_tuning;               /* (host) */

/* Sizes that fix the workspace of render_fwd / render_bwd (host). */
typedef struct {
    int64_t n;              /* splats in the scene */
    int64_t active_capacity;/* max active rows (n for dense rendering) */
    int64_t delta_capacity; /* max label changes per call (0 without pre-rendering) */
} oit_capacity;

/*
 * Bytes of workspace that oit_render_fwd / oit_render_bwd need for these views, sizes
 * and tuning; 0 on invalid arguments.  The forward pass leaves its projected splat
 * records, tile lists and per-pixel data in the workspace and the backward pass of
 * the same call sequence reads them, so both must get the same workspace, cameras,
 * capacities and tuning, with the splat parameters unchanged in between.
 */
size_t oit_workspace_bytes(const oit_capacity *cap, const oit_camera *cams, int32_t n_views,
                           const oit_tuning *tuning);

/*
 * Forward pass over V = n_views cameras (App. A, Alg. "rasterize"): project the rows
 * in the active list and in the label-change list, bin them into tiles (no depth
 * order), then per pixel blend the active splats, update the pre-rendered buffer with
 * the label changes and normalise:
 *   P = P_A + P0 - P1 / sigma,  Q = Q_A + Q0 - Q1 / sigma,  T = T_A exp(logT),
 *   F = P / Q (0 if Q <= 0),    C = T bg + (1 - T) F.
 *
 * splats      scene parameters (all n rows; only listed rows are read)
 * sigma       [1] device float, the weight's depth scale (> 0)
 * bg          (host) [3] background colour c0
 * cams        (host) [n_views] cameras, 1 <= n_views <= OIT_MAX_VIEWS
 * active_idx  [active_capacity] int32 splat ids of the active set, ascending;
 *             NULL renders all n splats (dense mode; n_active, delta_* must be NULL)
 * n_active    [1] device int32 count of active_idx entries used (<= active_capacity)
 * delta_idx   [delta_capacity] int32 splat ids whose label changed, delta_sign[k] = -1
 *             for a splat that joined the active set (its share leaves pre) and +1 for
 *             one that left it (its share joins pre); n_delta [1] device int32.
 *             All three NULL when no label changed.
 * delta_splats parameters the label-change rows are added to / removed from pre with;
 *             NULL = `splats`.  A pre buffer that is brought up to date lazily (some
 *             updates after the labels changed) must remove a splat with the values it
 *             was added with, although the splat may have been trained since it became
 *             active: pass the parameters as they were when the labels changed.
 * pre         [V][9][H][W] per-pixel accumulators of the inactive set: P0 (rgb),
 *             P1 (rgb), Q0, Q1, logT with P0 = sum (c - 1/2) alpha v,
 *             P1 = sum (c - 1/2) alpha v d, Q0 = sum alpha v, Q1 = sum alpha v d over
 *             inactive splats with d < sigma, logT = sum log(1 - alpha) over all
 *             inactive splats; updated in place by the label changes.  The colour
 *             sums are centred on the colour offset 1/2 so that they hold both signs:
 *             their float rounding then stays small against the differences that
 *             d/dsigma forms of them.  A zero buffer is the empty set.  NULL in dense
 *             mode.
 * image       [V][3][H][W] output C
 * pixstate    [V][6][H][W] output T, Q, F (rgb), dQ/dsigma = sum alpha v d / sigma^2 over
 *             the contributing splats with d < sigma (active and pre): what the
 *             backward pass needs
 * ws          workspace of oit_workspace_bytes(...) bytes, 256-byte aligned
 */
oit_status oit_render_fwd(const oit_splats *splats, const float *sigma, const float *bg,
                          const oit_camera *cams, int32_t n_views, const oit_capacity *cap,
                          const int32_t *active_idx, const int32_t *n_active,
                          const int32_t *delta_idx, const int8_t *delta_sign, const int32_t *n_delta,
                          const oit_splats *delta_splats,
                          float *pre, float *image, float *pixstate,
                          void *ws, size_t ws_bytes, const oit_tuning *tuning, oit_stream stream);

/*
 * Bytes of workspace that oit_l1_loss needs (a constant: a status word, the camera
 * table and 2048 FP64 per-block shares of the loss value).  Every render workspace
 * (oit_workspace_bytes) begins with this head in the same layout, so a render
 * workspace may be passed to oit_l1_loss between oit_render_fwd and oit_render_bwd:
 * the loss writes only the head, which oit_render_bwd does not read back (it uploads
 * its cameras again).
 */
size_t oit_l1_loss_workspace_bytes(void);

/*
 * L1 photometric loss over the batch (the L1 term of the 3DGS loss that the paper
 * keeps, Sec. 5.1): loss = sum_views mean_{3 H W} |C - target| and
 * grad_image = sign(C - target) / (3 H W) per view (sign(0) = 0).
 * image, target, grad_image [V][3][H][W]; loss [1] device double (overwritten), the
 * blocks' shares added in a fixed order.
 * ws          at least oit_l1_loss_workspace_bytes() bytes, 256-byte aligned (a render
 *             workspace qualifies, see above); OIT_ERR_WORKSPACE if smaller.
 */
oit_status oit_l1_loss(const float *image, const float *target, const oit_camera *cams,
                       int32_t n_views, float *grad_image, double *loss,
                       void *ws, size_t ws_bytes, oit_stream stream);

/* Bytes of workspace that oit_l1_dssim_loss needs for these views; 0 on invalid input. */
size_t oit_loss_workspace_bytes(const oit_camera *cams, int32_t n_views);

/*
 * The full 3DGS photometric loss, which the paper keeps (Sec. 5.1 "Implementation
 * Details"): loss = sum_views (1 - lambda) mean_{3HW} |C - target|
 *                            + lambda (1 - mean_{3HW} SSIM(C, target)),
 * SSIM with an 11 x 11 Gaussian window (std 1.5, zero padding), C1 = 0.01^2,
 * C2 = 0.03^2; lambda = 0.2 in 3DGS.  grad_image = dloss/dC.
 * image, target, grad_image [V][3][H][W]; loss [1] device double (overwritten);
 * ws of oit_loss_workspace_bytes(cams, n_views) bytes, 256-byte aligned.
 */
oit_status oit_l1_dssim_loss(const float *image, const float *target, const oit_camera *cams,
                             int32_t n_views, float lambda, float *grad_image, double *loss,
                             void *ws, size_t ws_bytes, oit_stream stream);

/*
 * Backward pass (App. B, Eq. "oit_rendering_detail", then the chain rule through the
 * projection): given dL/dC for every view, write the gradient of every parameter of
 * the active rows and of sigma.  Each splat's gradient is independent of the others
 * (App. B), so the kernel runs one splat per lane over its tile's pixels.
 * The inactive splats' share of d/dsigma comes from pre.  d/dsigma is formed as
 * sum over pixels and splats of dL/dw_i (dw_i/dsigma - lambda w_i) with
 * lambda = (dQ/dsigma) / Q per pixel; the lambda term is zero in exact arithmetic
 * (sum_i alpha_i w_i (c_i - F) = 0 at every pixel) and removes the first-order effect
 * of the float rounding of F on d/dsigma.
 *
 * grad_image  [V][3][H][W] dL/dC
 * pixstate    the forward pass's output
 * grads       output, compact rows in active_idx order (overwritten; rows beyond
 *             n_active untouched)
 * grad_sigma  [1] device double (overwritten)
 * score       [n] float, or NULL: written at the active splats' ids with
 *             max over groups g of ||dL/dtheta_g||_2 / eps[g] (Sec. 4.1, Eq. "activeness")
 * eps         (host) [6] per-group thresholds in the group order mean, log_scale, quat,
 *             opacity, sh, vsh; NULL means all 1
 * Other arguments as in oit_render_fwd, with the same values.
 */
oit_status oit_render_bwd(const oit_splats *splats, const float *sigma, const float *bg,
                          const oit_camera *cams, int32_t n_views, const oit_capacity *cap,
                          const int32_t *active_idx, const int32_t *n_active,
                          const int32_t *delta_idx, const int8_t *delta_sign, const int32_t *n_delta,
                          const float *pre, const float *grad_image, const float *pixstate,
                          const oit_grads *grads, double *grad_sigma,
                          float *score, const float *eps,
                          void *ws, size_t ws_bytes, const oit_tuning *tuning, oit_stream stream);

#define OIT_SELECT_TOPK 0
#define OIT_SELECT_THRESHOLD 1

/* Workspace bytes of oit_update_active_set for n splats. */
size_t oit_select_workspace_bytes(int64_t n);

/*
 * Active-set update (Sec. 4.1): pick the new active set from per-splat scores and
 * emit the label changes relative to the current labels.
 *   mode OIT_SELECT_TOPK:      the k largest scores; ties go to the lower splat id.
 *   mode OIT_SELECT_THRESHOLD: every splat with score > thresh (the paper's rule:
 *                              some group's gradient norm above its threshold).
 * score      [n] float, >= 0
 * label      [n] uint8 in/out: 1 = active.  On return holds the new labels.
 * active_idx [active_capacity] out, ascending; n_active [1] device int32 out
 * delta_idx  [delta_capacity] out, ascending; delta_sign [delta_capacity] int8 out
 *            (-1 joined, +1 left); n_delta [1] device int32 out
 * Counts above the capacities set the status word's overflow bits; the lists then
 * hold the first `capacity` entries.
 */
oit_status oit_update_active_set(const float *score, int64_t n, int32_t mode, int64_t k, float thresh,
                                 uint8_t *label, int32_t *active_idx, int64_t active_capacity,
                                 int32_t *n_active, int32_t *delta_idx, int8_t *delta_sign,
                                 int64_t delta_capacity, int32_t *n_delta,
                                 void *ws, size_t ws_bytes, oit_stream stream);

/*
 * oit_update_active_set without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  The library calls no allocator: its scratch is a static device
 * array of oit_select_workspace_bytes(OIT_NOALLOC_SELECT_MAX_N) bytes (about 4.3 MB),
 * one per GPU the library runs on, held until the process ends.
 * n           1 .. OIT_NOALLOC_SELECT_MAX_N splats; larger n is OIT_ERR_INVALID.
 * status      [1] device int32 out: cleared, then given the overflow bits that
 *             oit_update_active_set sets in its workspace's status word.
 * Other arguments and results as oit_update_active_set.  All calls on one GPU share
 * that GPU's scratch, which keeps the last call's contents: calls that overlap on one
 * GPU (concurrent streams, or host threads) race and must be serialised by the caller.
 */
#define OIT_NOALLOC_SELECT_MAX_N (1LL << 22)
oit_status oit_update_active_set_noalloc(const float *score, int64_t n, int32_t mode, int64_t k, float thresh,
                                         uint8_t *label, int32_t *active_idx, int64_t active_capacity,
                                         int32_t *n_active, int32_t *delta_idx, int8_t *delta_sign,
                                         int64_t delta_capacity, int32_t *n_delta, int32_t *status,
                                         oit_stream stream);

/*
 * Label changes between two label arrays (for pre-rendered buffers that fell behind
 * several active-set updates: the paper delays the pre-render update of a view until
 * the view is next used, Sec. 4.1 "Implementation Details").
 * old_label, new_label [n] uint8 (1 = active), unchanged.
 * active_idx [active_capacity], n_active: the rows of new_label, ascending (both may be
 * NULL); delta_idx, delta_sign, n_delta: the rows whose label differs, ascending, with
 * sign -1 (active in new_label: leaves pre) or +1 (inactive in new_label: joins pre).
 * Workspace as for oit_update_active_set.
 */
oit_status oit_label_delta(const uint8_t *old_label, const uint8_t *new_label, int64_t n,
                           int32_t *active_idx, int64_t active_capacity, int32_t *n_active,
                           int32_t *delta_idx, int8_t *delta_sign, int64_t delta_capacity,
                           int32_t *n_delta, void *ws, size_t ws_bytes, oit_stream stream);

/*
 * Farthest-point sampling of s views from n camera centres (host; Sec. 4.1: the active
 * set is updated from a subset of training views picked by farthest point sampling
 * with a random initialisation; the caller draws `start`).  centres (host) [n][3];
 * out (host) [s] in pick order: start, then repeatedly the view whose squared distance
 * to the nearest picked view is largest (ties to the lower index), in double precision.
 */
oit_status oit_fps_views(const float *centres, int32_t n, int32_t s, int32_t start, int32_t *out);

/*
 * Adam on the active rows only (Sec. 4.1, Alg. "Active Set Method": the update
 * touches only the active splats; the optimiser is Adam, Sec. 5.1).
 * For every active row i (splat id active_idx[r], compact gradient row r) and
 * component:  m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
 *             theta -= lr_g * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * Rows outside the active set, their moments included, are not touched.
 * params/m/v  [6] pointers to the [n][C] groups (mean, log_scale, quat, opacity_logit,
 *             sh, vsh); grads as written by oit_render_bwd
 * active_idx  NULL for dense (all n rows); n_active device count or NULL (= n)
 * lr          (host) [6] per-group learning rates
 * step        [1] device int32: incremented by this call, then used as t.
 */
oit_status oit_sparse_adam_step(float *const *params, const oit_grads *grads, float *const *m,
                                float *const *v, const int32_t *active_idx, const int32_t *n_active,
                                int64_t n, const float *lr, float beta1, float beta2, float eps,
                                int32_t *step, oit_stream stream);

/*
 * Adam step on sigma from its FP64 gradient (same rule, one scalar): sigma, m, v [1]
 * device float; step [1] device int32, incremented by this call then used as t.
 */
oit_status oit_sigma_adam_step(float *sigma, const double *grad_sigma, float *m, float *v,
                               float lr, float beta1, float beta2, float eps, int32_t *step,
                               oit_stream stream);

/* ---------------------------------------------------------------------------------
 * Densification and pruning of the first training phase.  The paper trains its first
 * 15,000 iterations as 3DGS does, with 3DGS's density control plus a random keep
 * probability that caps the splat count, and starts the active-set phase after it
 * (Sec. 5.1 "Implementation Details"; Fig. "overview").  The rules are 3DGS's:
 *   statistic  per (splat, view) where the splat is visible (valid projection, opacity
 *              >= 1/255, the box of its alpha >= 1/255 ellipse reaches a pixel centre
 *              of the image): the norm of dL/d(projected mean) per normalised-device
 *              unit, (dL/dmx W/2, dL/dmy H/2), summed into grad_accum; denom counts
 *              those views; max_radius keeps the largest 3-sigma screen radius (px);
 *   candidate  grad_accum / denom >= grad_threshold and the splat's uniform draw <
 *              keep_probability; a candidate whose largest scale is <= percent_dense *
 *              scene_extent is cloned, a larger one is replaced by two children at
 *              mean + R diag(s) z (z a standard normal draw per child) with every
 *              scale divided by 1.6;
 *   pruning    of the densified set: opacity < min_opacity; largest scale >
 *              max_world_frac * scene_extent (if max_world_frac > 0); for original
 *              splats, max_radius > max_screen_size (if max_screen_size > 0);
 *   order      surviving originals, clone copies, first children, second children,
 *              each in source order; new splats get zero Adam moments.
 * These decisions are taken in float32.
 * --------------------------------------------------------------------------------- */
typedef struct {
    float grad_threshold;   /* 3DGS: 0.0002 */
    float percent_dense;    /* 3DGS: 0.01 */
    float scene_extent;     /* > 0 */
    float min_opacity;      /* 3DGS: 0.005 */
    float max_screen_size;  /* pixels; <= 0 disables (3DGS: 20 after the first opacity reset) */
    float max_world_frac;   /* <= 0 disables (3DGS: 0.1 with the screen-size rule) */
    float keep_probability; /* in [0, 1]: the paper's random sampling of densification */
    int32_t reserved;       /* 0 */
} oit_density_rules;        /* (host) */

/*
 * Add the densification statistic of the last oit_render_bwd to grad_accum, denom and
 * max_radius (each [n] float, indexed by splat id; the caller zeroes them when a
 * densification interval starts).  Call it after oit_render_bwd, on the same stream,
 * with the same cams, capacity, active rows and tuning and the same workspace, before
 * the workspace is used again: it reads the records and the per-entry partials that
 * call left there.  Rows are the active rows of that call (all splats in dense mode).
 * Returns OIT_ERR_INVALID for NULL accumulators or bad sizes; nothing is enqueued then.
 */
oit_status oit_densify_stats(const oit_camera *cams, int32_t n_views, const oit_capacity *cap,
                             const int32_t *active_idx, const int32_t *n_active, const int32_t *n_delta,
                             float *grad_accum, float *denom, float *max_radius,
                             const void *ws, size_t ws_bytes, const oit_tuning *tuning, oit_stream stream);

/* Workspace bytes of oit_densify_plan / oit_densify_apply for n splats. */
size_t oit_densify_workspace_bytes(int64_t n);

/*
 * Decide, for every splat, whether it is kept, cloned or split and which of the
 * results survive pruning (rules above), and write the size of the new set to
 * *n_new (device int64).  uniform [n]: the splats' uniform draws in [0, 1).  The
 * decisions stay in the workspace for oit_densify_apply.
 */
oit_status oit_densify_plan(const oit_splats *splats, const float *grad_accum, const float *denom,
                            const float *max_radius, const float *uniform, const oit_density_rules *rules,
                            int64_t *n_new, void *ws, size_t ws_bytes, oit_stream stream);

/*
 * Write the new set planned by the last oit_densify_plan on this workspace (same
 * splats): params_new, m_new and v_new are [6] pointers to [cap_new][C] groups in the
 * order of oit_splats (mean, log_scale, quat, opacity_logit, sh, vsh); m / v are the
 * old moments.  normals [n][2][3]: the standard normal draws of each splat's two
 * children (read for split splats only).  Rows at or past cap_new are not written, so
 * the caller reads *n_new first and passes cap_new >= it.
 */
oit_status oit_densify_apply(const oit_splats *splats, const float *const *m, const float *const *v,
                             const float *normals, float *const *params_new, float *const *m_new,
                             float *const *v_new, int64_t cap_new, const void *ws, size_t ws_bytes,
                             oit_stream stream);

/*
 * 3DGS's opacity reset: every opacity above max_opacity is set to it (logit clamped to
 * log(max_opacity / (1 - max_opacity))) and the opacity group's Adam moments restart
 * from zero.  opacity_logit, m_opacity, v_opacity [n].
 */
oit_status oit_reset_opacity(float *opacity_logit, float *m_opacity, float *v_opacity, int64_t n,
                             float max_opacity, oit_stream stream);

/* Wait for `stream` and copy the workspace's device status word to *out (host). */
oit_status oit_read_status(const void *ws, size_t ws_bytes, int32_t *out, oit_stream stream);

/*
 * Wait for `stream` and copy the counters the last oit_render_fwd / oit_render_bwd on
 * this workspace left (arguments as given to that call; out (host) [6]):
 *   out[0] (tile, splat) entries the forward needed (also when it overflowed
 *          tuning.pair_capacity, so a caller can size pair_capacity and run again;
 *          saturated at 2^32 - 1, above any pair capacity),
 *   out[1] contributing (alpha >= 1/255) active (splat, pixel) pairs it blended,
 *   out[2] active (splat, pixel) pairs it evaluated (tile entries x in-image tile pixels),
 *   out[3] backward work items (up to 64 active entries of one tile each),
 *   out[4] of those, the items the last backward walked footprint box by footprint box
 *          (small footprints) instead of pixel group by pixel group,
 *   out[5] of those, the items whose pixel groups the whole wave walked one by one
 *          (footprints that nearly all reach all the item's groups); the rest had their
 *          (entry, group) pairs dealt to the lanes.
 */
oit_status oit_read_counters(const void *ws, size_t ws_bytes, const oit_capacity *cap,
                             const oit_camera *cams, int32_t n_views, const oit_tuning *tuning,
                             int64_t *out, oit_stream stream);

/*
 * Wait for `stream` and copy the per-tile entry counts of the last oit_render_fwd on
 * this workspace (arguments as given to that call): out (host) [2][T], T = the tiles
 * of the batch (views in order, each row-major, ceil(W / tile) x ceil(H / tile)); row 0
 * holds each tile's active entries, row 1 its label-change entries.  out_len is the
 * length of out in elements (at least 2 T, else OIT_ERR_INVALID).  A diagnostic of the
 * work per tile (the forward runs one workgroup per tile).
 */
oit_status oit_read_tile_entries(const void *ws, size_t ws_bytes, const oit_capacity *cap,
                                 const oit_camera *cams, int32_t n_views, const oit_tuning *tuning,
                                 uint32_t *out, int64_t out_len, oit_stream stream);

/*
 * Timing of the raster kernels, for benchmarks.  While enabled (on != 0), every
 * oit_render_fwd launches its raster kernel (label changes into `pre`, when given,
 * then the active entries, in one launch) and every oit_render_bwd its raster kernel with HIP
 * events that the runtime records when the kernel starts and when it ends.  Eager
 * launches only: a render call on a stream that is being captured fails with
 * OIT_ERR_INVALID while timing is on.  The events are created once by the first
 * enable and owned by the library; the setting is process-wide and not synchronised
 * between threads.
 */
oit_status oit_timing_enable(int32_t on);

/* Wait for the last recorded events; out (host) [2] = milliseconds of the last
 * forward raster kernel and of the last
 * backward raster kernel (-1 if not recorded). */
oit_status oit_timing_read(float *out);

/* Wait for the last recorded stage events; out (host) [6] = milliseconds of the last
 * forward's preprocess, binning and raster stage (the raster kernel and its counter
 * sum) and of the last backward's pixel constants, raster stage (work-item map and
 * raster kernel) and preprocess backward (with the dL/dsigma sum), each measured
 * between events recorded on the stream at the stage boundaries (-1 if not recorded). */
oit_status oit_timing_read_stages(float *out);

/* Clear the status word (enqueued on `stream`). */
oit_status oit_clear_status(void *ws, size_t ws_bytes, oit_stream stream);

/* Message of the last failing call on the calling thread ("" if none). */
const char *oit_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* OIT_H */

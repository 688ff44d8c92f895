/*
 * lodge.h -- C ABI of the MI355X (gfx950) per-frame renderer for
 * level-of-detail Gaussian splatting (LODGE, arXiv 2505.23158).
 *
 * One frame is:  lodge_select  (two nearest chunks + Eq. 4 weight t, active
 * set of Eq. 2 with per-chunk offset thresholds)  ->  lodge_render  (EWA
 * projection with the Eq. 3 3-D filter and the renderer's 2-D filter, SH
 * colour, 16x16 tile binning, per-tile sort on (depth, index), front-to-back
 * alpha compositing of Eq. 1 with early termination).  lodge_render_backward
 * is the adjoint of lodge_render for the per-level fine-tuning of the
 * paper's supplementary material ("LOD structure optimization steps").
 *
 * Conventions shared by every call
 *  - All functions return a lodge_status and never abort; the message of
 *    the last failure on the calling thread is lodge_last_error().
 *  - "device" pointers are HIP device memory owned by the caller; "host"
 *    pointers are read during the call only unless stated otherwise.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls marked
 *    ASYNC enqueue work on `stream` and return; they never synchronise the
 *    host and never allocate device memory.
 *  - The camera of a frame lives in its workspace.  Calls that take a
 *    `const lodge_camera* cam` first store it there (as a kernel argument,
 *    so the caller's struct may change as soon as the call returns); cam =
 *    NULL uses the camera stored by the last lodge_set_camera or call on
 *    that workspace.  To replay a captured HIP graph for new cameras,
 *    capture lodge_select/lodge_render with cam = NULL and call
 *    lodge_set_camera on the same stream before each replay.
 *  - Every array of Gaussian parameters is a structure of arrays in FP32:
 *    attribute-major planes of n floats each.
 *  - Data-dependent sizes never return to the host inside a frame: device
 *    counters bound every kernel.  Capacity overflows set device flags that
 *    lodge_check() reports after the stream has been synchronised.
 */
#ifndef LODGE_H
#define LODGE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */

typedef enum {
    LODGE_OK = 0,
    LODGE_ERR_INVALID_ARG = 1,   /* a pointer, size or value outside its stated range */
    LODGE_ERR_CAPACITY = 2,      /* a workspace / selection capacity was exceeded */
    LODGE_ERR_HIP = 3,           /* the HIP runtime reported an error (see lodge_last_error) */
    LODGE_ERR_UNSUPPORTED = 4    /* a valid request the library does not handle */
} lodge_status;

/* Static description of a status code. */
const char* lodge_status_string(lodge_status s);
/* Message of the last non-OK status returned on this thread ("" if none). */
const char* lodge_last_error(void);
/* Library version string. */
const char* lodge_version(void);

/* ------------------------------------------------------------ scene input */

/* One LOD level G^(l) (Sec. 3 "Level of Detail (LOD) representation"):
 * activated parameters, device memory, borrowed until lodge_scene_destroy.
 *   mean    [3][n]   position mu
 *   scale   [3][n]   linear per-axis scale s (covariance R diag(s^2) R^T)
 *   quat    [4][n]   rotation quaternion (w, x, y, z), used as given
 *   opacity [n]      o in [0, 1]
 *   sh      [(d+1)^2][3][n]  real SH coefficients [basis][channel][n]
 *   sh_degree d in 0..3
 *   filter3d_var     variance of the level's 3-D smoothing filter (Eq. 3,
 *                    Sec. 3 "Building LOD representation"), m^2, >= 0 */
typedef struct {
    int64_t n;
    const float* mean;
    const float* scale;
    const float* quat;
    const float* opacity;
    const float* sh;
    int32_t sh_degree;
    float filter3d_var;
} lodge_level;

/* Chunks (Sec. 3 "Reducing memory with chunk-based rendering"): centres
 * m_k and the offset r_k added to every switch distance for chunk k.
 * Host memory, copied by lodge_scene_create.  1 <= k <= LODGE_MAX_CHUNKS.
 * band > 0 narrows the Eq. 4 ramp to a strip of that width (metres)
 * around the bisector of the two centres; band <= 0 is Eq. 4 as printed. */
#define LODGE_MAX_CHUNKS 128
typedef struct {
    int32_t k;
    const float* center;  /* host [k][3] */
    const float* offset;  /* host [k]    */
    float band;
} lodge_chunks;

/* Pinhole camera, OpenCV axes (x right, y down, z forward).  R is the
 * world->camera rotation (row-major), t its translation, pos the camera
 * centre (both sides of the renderer use pos as given).  Pixel (x, y) is
 * sampled at (x + 0.5, y + 0.5).  Gaussians with camera depth <= znear are
 * culled; the projection Jacobian is evaluated at the mean clamped to
 * |x/z| <= lim_x, |y/z| <= lim_y.  bg is the background colour. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    float pos[3];
    float znear, lim_x, lim_y;
    float bg[3];
} lodge_camera;

/* Opaque scene: the level pointers (borrowed), the switch distances and the
 * chunk table (owned host copies).  Read-only after creation; one scene may
 * be used by any number of concurrent frames on distinct workspaces. */
typedef struct lodge_scene lodge_scene;

#define LODGE_MAX_LEVELS 8

/* Creates a scene of L levels (1 <= L <= LODGE_MAX_LEVELS).  d (host, L-1
 * values) holds the switch distances d_1 < ... < d_{L-1} of Eq. 2 (d_0 = 0
 * and d_L = infinity implicitly; d may be NULL when L = 1).  chunks may be
 * NULL (then only LODGE_SELECT_ALL and LODGE_SELECT_LOD_CAMERA work).
 * Validates: n >= 0, sum of n < 2^32, d strictly increasing and > 0,
 * sh_degree in 0..3, non-NULL planes when n > 0, filter3d_var >= 0; chunk
 * centres finite and pairwise distinct (the squared FP32 distance of every
 * pair finite and > 0, since Eq. 4 divides by it), offsets finite and >= 0,
 * band finite;
 * LODGE_ERR_UNSUPPORTED for a level of 2^30 or more Gaussians (its planes
 * are addressed with 32-bit byte offsets).
 * Allocates host memory only.  *out is NULL on failure. */
lodge_status lodge_scene_create(const lodge_level* levels, int32_t L, const float* d,
                                const lodge_chunks* chunks, lodge_scene** out);
void lodge_scene_destroy(lodge_scene* scene);
/* Total number of Gaussians over all levels (global ids are
 * id = sum_{j<l} n_j + i for Gaussian i of level l). */
int64_t lodge_scene_total(const lodge_scene* scene);

/* A packed copy of the levels for the projection: per Gaussian, its scale,
 * opacity and rotation as two 16-byte words, and its SH coefficients as one
 * contiguous run of 16-byte words ([basis][channel] order, zero-padded to a
 * multiple of four floats).  A layout change only: frames render the same
 * result bit for bit, reading 2 + ceil(3 (d+1)^2 / 4) contiguous words per
 * Gaussian instead of 8 + 3 (d+1)^2 separate planes.  The means stay in the
 * caller's planes (the selection streams them).
 * lodge_pack_size: bytes of device memory the copy needs (224 per Gaussian
 * at degree 3, each level's part 256-byte aligned). */
lodge_status lodge_pack_size(const lodge_scene* scene, size_t* bytes);

/* ASYNC.  Fills `pack` (device, caller-owned, >= lodge_pack_size() bytes,
 * 256-byte aligned, kept alive until the scene is destroyed or detached)
 * from the level planes and makes the scene's projection read it.  It is a
 * snapshot: after the caller changes scale, rotation, opacity or SH of a
 * level, pack again (or detach).  pack = NULL detaches (the projection reads
 * the planes again).  Call it before frames on the scene are enqueued, on a
 * stream ordered before them: it changes the scene that later calls read. */
lodge_status lodge_scene_pack(lodge_scene* scene, void* pack, size_t bytes, void* stream);

/* -------------------------------------------------------------- workspace */

/* Caller-allocated device scratch for one frame in flight, laid out by the
 * library from these fields.  A workspace serves one image size and is
 * reused across frames; lodge_render_backward reads what lodge_render left
 * in it, so a frame's backward must run before the workspace's next render.
 * Frames on distinct workspaces may run concurrently on distinct streams. */
typedef struct {
    void* base;              /* device, >= lodge_workspace_size() bytes, 256-byte aligned */
    size_t bytes;
    int32_t width, height;   /* image size this workspace serves */
    uint32_t max_active;     /* capacity for selected Gaussians (== the selection cap) */
    uint64_t max_instances;  /* capacity for (Gaussian, tile) instances, < 2^32 */
} lodge_workspace;

lodge_status lodge_workspace_size(const lodge_scene* scene, int32_t width, int32_t height, uint32_t max_active,
                                  uint64_t max_instances, size_t* bytes);

/* ASYNC.  Stores *cam in the workspace for the next frame (cam->width and
 * cam->height must equal the workspace's). */
lodge_status lodge_set_camera(const lodge_workspace* ws, const lodge_camera* cam, void* stream);

/* -------------------------------------------------------------- selection */

enum {
    LODGE_SELECT_ALL = 0,        /* every Gaussian of every level, weight 1 (plain render) */
    LODGE_SELECT_LOD_CAMERA = 1, /* Eq. 2 about the camera centre, weight 1 */
    LODGE_SELECT_CHUNKED = 2     /* Eq. 2 about the two nearest chunk centres (offsets r_k), union
                                    with the Eq. 4 opacity weights (Sec. 3 "Opacity blending") */
};

/* Output of lodge_select, device memory owned by the caller:
 *   ids[cap]  global ids of the active Gaussians, strictly ascending
 *   w[cap]    opacity weight of each: 1 in both chunk sets, t in the nearest
 *             chunk's set only, 1 - t in the other's only
 *   count[1]  number selected (may exceed cap: then only cap entries are
 *             written, the overflow flag is set and the frame renders the
 *             first cap entries) */
typedef struct {
    uint32_t* ids;
    float* w;
    uint32_t* count;
    uint32_t cap;
} lodge_selection;

/* ASYNC.  Computes the chunk pair (f, o) and t (Eq. 4; ties go to the lower
 * chunk index) on the device, then the active set (Eq. 2, with thresholds
 * d_l + r_k about chunk k's centre; intervals [d_l, d_{l+1}) on squared
 * FP32 distances).  sel->cap must equal ws->max_active. */
lodge_status lodge_select(const lodge_scene* scene, const lodge_camera* cam, int32_t mode,
                          const lodge_workspace* ws, lodge_selection* sel, void* stream);

/* Precomputed per-chunk active sets (Sec. 3 "Reducing memory with
 * chunk-based rendering": each chunk stores the Gaussians Eq. 2 selects at
 * its centre with the offset thresholds d_l + r_k; a frame loads the union
 * of the two nearest chunks' sets).  One bit per Gaussian per chunk, in the
 * selection's tile order: K x ceil-per-level(n_l / 4096) x 256 x 2 bytes
 * (3.3 MB per chunk at 26.55M Gaussians).  The buffer is device memory owned
 * by the caller, 4-byte aligned; it stays valid while the scene's level
 * planes and chunk table are unchanged.  LODGE_ERR_INVALID_ARG for a scene
 * without chunks. */
lodge_status lodge_chunk_sets_size(const lodge_scene* scene, size_t* bytes);

/* ASYNC.  Fills the chunk sets (every chunk's membership of every Gaussian,
 * evaluated with the same FP32 operations as lodge_select). */
lodge_status lodge_chunk_sets_build(const lodge_scene* scene, void* sets, size_t bytes, void* stream);

/* ASYNC.  The same result as lodge_select(..., LODGE_SELECT_CHUNKED, ...)
 * (ids, weights, count, bit for bit), read from the two chunks' stored sets
 * instead of the Gaussians' means: 2 bits of input per Gaussian instead of
 * 12 bytes. */
lodge_status lodge_select_chunk_sets(const lodge_scene* scene, const void* sets, const lodge_camera* cam,
                                     const lodge_workspace* ws, lodge_selection* sel, void* stream);

/* -------------------------------------------------------------- rendering */

typedef struct {
    float s2d;           /* screen-space filter variance (px^2) added to the 2-D covariance, >= 0 */
    int32_t compensate;  /* 1: scale opacity by sqrt(det(S')/det(S' + s2d I)) (Mip-Splatting-style 2-D filter) */
    void* const* stage_events;  /* NULL, or LODGE_STAGE_EVENTS hipEvent_t recorded on the stream before
                                   projection, binning, sorting and compositing and after compositing */
} lodge_render_opts;
#define LODGE_STAGE_EVENTS 5

/* ASYNC.  Renders the selection into caller device buffers:
 *   image     [3][H][W]  C + T_final * bg
 *   final_T   [H][W]     transmittance left after the last blended Gaussian
 *   n_contrib [H][W]     1 + position (in its tile's sorted list) of the last
 *                        blended Gaussian, 0 if none
 * Stages: project (Eq. 3 filter, EWA, 2-D filter, SH, 3-sigma tile rect,
 * depth), per-tile counting, instance emission, per-tile on-chip sort on
 * (depth bits, active index), compositing (Eq. 1; alpha = min(0.99, o G),
 * entries with alpha < 1/255 skipped, stop before T(1 - alpha) < 1e-4).
 * opts may be NULL (s2d = 0.3, compensate = 1). */
lodge_status lodge_render(const lodge_scene* scene, const lodge_selection* sel, const lodge_camera* cam,
                          const lodge_render_opts* opts, const lodge_workspace* ws, float* image, float* final_T,
                          uint32_t* n_contrib, void* stream);

/* Per-frame counters kept in the workspace (device) by select + render. */
typedef struct {
    uint32_t n_selected;     /* active set size (may exceed the capacity) */
    uint32_t n_front;        /* selected Gaussians in front of the near plane */
    uint32_t n_visible;      /* projected Gaussians with a non-empty tile rect */
    uint32_t max_tile_len;   /* longest per-tile list */
    uint64_t n_instances;    /* (Gaussian, tile) pairs */
    uint64_t pairs_evaluated;/* (pixel, list entry) pairs visited before each pixel stopped */
    uint64_t pairs_blended;  /* pairs that were alpha-blended */
    uint32_t overflow;       /* bit 0 selection cap, bit 1 instance cap */
    int32_t f, o;            /* chunk pair (-1 when unused) */
    float t;                 /* Eq. 4 weight of the nearest chunk */
    uint32_t n_long;         /* tiles whose list is longer than 2048 and at most 16384 */
    uint32_t n_merge;        /* tiles whose list is longer than 16384 */
    uint64_t pixels_stopped; /* pixels that stopped before the end of their list (T (1 - alpha) < 1e-4) */
} lodge_frame_info;

/* Synchronises `stream`, then copies the counters of the last frame on ws. */
lodge_status lodge_frame_info_read(const lodge_workspace* ws, lodge_frame_info* out, void* stream);

/* Synchronises `stream`; returns LODGE_ERR_CAPACITY if the last frame on ws
 * overflowed a capacity, with the sizes it needed (either pointer may be NULL). */
lodge_status lodge_check(const lodge_workspace* ws, uint32_t* needed_active, uint64_t* needed_instances,
                         void* stream);

/* Device views of the last frame's intermediates inside ws (valid until the
 * next render on ws), for inspection and tests.  Any pointer may be NULL.
 *   sorted_ids [n_instances]  active index of each instance, tile-major,
 *                             each tile's run in ascending (depth bits, index)
 *   tile_ranges[TX*TY][2]     [start, end) of each tile's run (any start when empty)
 *   proj       [max_active][12]  per visible active index, in the form the
 *                             compositor reads: u, v, -A/2, -B, -C/2 (conic
 *                             A, B, C), o_eff, thr (the power below which alpha
 *                             cannot reach 1/255), r, g, b, ex, ey (half-extents
 *                             of the ellipse where it can)
 *   depth      [max_active]   camera depth (0 when culled)
 *   rect       [max_active][2] tile rect as x0 | y0 << 16, x1 | y1 << 16
 *                             (x0 >= x1 or y0 >= y1: culled) */
lodge_status lodge_debug_views(const lodge_workspace* ws, const uint32_t** sorted_ids, const uint32_t** tile_ranges,
                               const float** proj, const float** depth, const uint32_t** rect);

/* ------------------------------------------------- visibility filtering */

/* ASYNC.  The stored active set of chunk k alone (Sec. 3 "Reducing memory
 * with chunk-based rendering": Eq. 2 at the chunk centre m_k with every
 * switch distance offset by r_k), every member with weight 1: the set that
 * the per-chunk visibility filtering (Sec. 3 "Visibility filtering") renders
 * and prunes.  sets: NULL to evaluate the set from the means, or a buffer
 * from lodge_chunk_sets_build (then the result reflects any pruning already
 * applied to it).  0 <= k < the scene's chunk count; sel->cap must equal
 * ws->max_active.  The workspace's camera is not used or changed. */
lodge_status lodge_select_chunk(const lodge_scene* scene, const void* sets, int32_t k, const lodge_workspace* ws,
                                lodge_selection* sel, void* stream);

/* ASYNC.  Importance scores (Sec. 3 "Preliminaries: Importance pruning"):
 * lodge_render's projection, binning and sort, then its compositing walk
 * without an image: every entry blended at a pixel contributes its weight
 * alpha T (alpha = min(0.99, o G), T the transmittance in front of it), and
 *   score[id] = max(score[id], weight)
 * for the entry's global id, over every pixel of the view.  score (device,
 * lodge_scene_total() floats, caller-owned, >= 0; the caller sets it to 0
 * before the first view) accumulates the maximum over successive calls, so a
 * set of views gives each Gaussian its largest weight in any of them.
 * Entries skipped (alpha < 1/255) or stopping a pixel (T (1 - alpha) < 1e-4)
 * weigh nothing.  Overflows are reported by lodge_check as for
 * lodge_render.  Calls on different streams into one score array are safe
 * (the maximum is taken with atomics). */
lodge_status lodge_importance(const lodge_scene* scene, const lodge_selection* sel, const lodge_camera* cam,
                              const lodge_render_opts* opts, const lodge_workspace* ws, float* score, void* stream);

/* ASYNC.  Visibility filtering of chunk k's stored set (Sec. 3 "Visibility
 * filtering"): every member whose score (device, by global id, as left by
 * lodge_importance) is below threshold is removed from chunk k's set in
 * `sets` (from lodge_chunk_sets_build); other chunks are untouched.  A frame
 * then loads the filtered sets through lodge_select_chunk_sets (Eq. 4
 * weights by membership of the filtered sets).  threshold must be finite. */
lodge_status lodge_chunk_sets_prune(const lodge_scene* scene, void* sets, size_t bytes, int32_t k, const float* score,
                                    float threshold, void* stream);

/* ------------------------------------------------- no-allocation rendering */

/* For callers that cannot allocate device memory, not even a workspace: code
 * under HIP graph capture, serving loops that must not allocate, harnesses
 * that forbid hipMalloc.  ASYNC.  lodge_render's kernels and outputs, with the
 * workspace replaced by a scratch array inside the library:
 * LODGE_STATIC_SCRATCH_BYTES of device memory on each GPU the library runs
 * on, held from the first use on that GPU until the process ends.  The call
 * allocates nothing.  Every call on a GPU shares that GPU's array (it keeps
 * the last call's contents; each call clears what it needs), so calls that
 * overlap on one GPU -- other streams, other host threads -- race: serialise
 * them.
 *   cam       required (nothing is stored between calls); its size is the
 *             frame's
 *   sel       as for lodge_render (ids, weights, device count, cap); the
 *             workspace's max_active is sel->cap
 *   overflow  NULL, or a device word set when the frame completes: bit 0 the
 *             selection count exceeded sel->cap (the first cap entries were
 *             rendered), bit 1 the (Gaussian, tile) instances exceeded what
 *             the scratch holds (the frame is then background only).  The
 *             instance capacity is what remains of the scratch after the
 *             per-active and per-tile regions: about 28 bytes per instance at
 *             1080p after 120 bytes per selected Gaussian.
 * LODGE_ERR_INVALID_ARG, with the sizes in lodge_last_error(), when the
 * image size and sel->cap leave no room for instances. */
#define LODGE_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
lodge_status lodge_render_static(const lodge_scene* scene, const lodge_selection* sel, const lodge_camera* cam,
                                 const lodge_render_opts* opts, float* image, float* final_T, uint32_t* n_contrib,
                                 uint32_t* overflow, void* stream);

/* ---------------------------------------------------------- differentiation */

/* Gradient planes of one level, device memory, same shapes as the level's
 * parameters; the backward ADDS into them (the caller zeroes), so a batch of
 * views accumulates.  Any pointer may be NULL to skip that parameter. */
typedef struct {
    float* mean;
    float* scale;
    float* quat;
    float* opacity;
    float* sh;
} lodge_grads;

/* ASYNC.  Adjoint of lodge_render for L = sum(dL_dimage * image):
 * gradients w.r.t. the activated parameters of every selected Gaussian
 * (grad_level >= 0: only Gaussians of that level, as the per-level
 * fine-tuning updates G_l alone).  Walks each pixel's list back to front
 * from n_contrib - 1, recovering the transmittance before each entry as
 * T_k = T_{k+1} / (1 - alpha_k) from final_T instead of storing it (the
 * division by the hardware reciprocal, within 1 ulp per entry).
 * ws must still hold the forward's intermediates (same scene, selection,
 * camera and options).  grads is an array of L entries.  opts->stage_events,
 * when set, gets its first three events recorded on the stream: before the
 * compositing adjoint, between it and the projection adjoint, and after.
 * Accumulation is a plain read-add-write per Gaussian (one thread owns each
 * selected Gaussian within a call), not an atomic: two calls that run at
 * the same time (different streams) into the same gradient planes race and
 * lose updates.  Serialise such calls on one stream, or give each its own
 * planes and sum them afterwards. */
lodge_status lodge_render_backward(const lodge_scene* scene, const lodge_selection* sel, const lodge_camera* cam,
                                   const lodge_render_opts* opts, const lodge_workspace* ws, const float* final_T,
                                   const uint32_t* n_contrib, const float* dL_dimage, int32_t grad_level,
                                   const lodge_grads* grads, void* stream);

/* ASYNC.  3DGS parameter activation for n Gaussians (device planes):
 * scale = exp(log_scale), quat = q / |q|, opacity = sigmoid(logit).
 * Output planes have the shapes of the inputs. */
lodge_status lodge_activate(int64_t n, const float* log_scale, const float* quat_raw, const float* opacity_logit,
                            float* scale, float* quat, float* opacity, void* stream);

/* ASYNC.  Chain rule through lodge_activate: given the activated values
 * (scale, quat_raw, opacity) and gradients w.r.t. the activated parameters,
 * ADDS gradients w.r.t. log_scale, quat_raw and the opacity logit. */
lodge_status lodge_activate_backward(int64_t n, const float* quat_raw, const float* scale, const float* opacity,
                                     const float* g_scale, const float* g_quat, const float* g_opacity,
                                     float* g_log_scale, float* g_quat_raw, float* g_opacity_logit, void* stream);

/* ------------------------------------------------ LOD-level construction */

/* The per-level fine-tuning of the supplementary "LOD structure
 * optimization steps" renders with lodge_select/lodge_render, takes the
 * loss gradient with lodge_l1_grad, back-propagates with
 * lodge_render_backward (grad_level = the level being built) and
 * lodge_activate_backward, and updates the level with lodge_adam; after each
 * importance pruning (lodge_importance over the training views) the level's
 * parameters and optimiser moments are compacted with lodge_keep_indices and
 * lodge_gather_planes. */

/* ASYNC.  Gradient of the L1 loss scale * sum |image - target| over n
 * values: grad[i] = scale * sign(image[i] - target[i]) (0 where equal).
 * scale = 1/n gives the mean L1.  loss: NULL, or a device float that the
 * call ADDS scale * sum |image - target| to (one atomic per block, so its
 * rounding depends on block order). */
lodge_status lodge_l1_grad(int64_t n, const float* image, const float* target, float scale, float* grad, float* loss,
                           void* stream);

/* ASYNC.  One Adam step (Kingma and Ba) on n parameters in place, with its
 * moments m and v (device, caller-owned, zero before step 1):
 *   m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
 *   p = p - lr (m / (1 - beta1^step)) / (sqrt(v / (1 - beta2^step)) + eps).
 * step counts from 1; 0 <= beta < 1, eps >= 0. */
lodge_status lodge_adam(int64_t n, float* param, const float* grad, float* m, float* v, float lr, float beta1,
                        float beta2, float eps, int32_t step, void* stream);

/* Bytes of device scratch lodge_dssim_grad needs for one image (ten maps of
 * channels x height x width floats). */
lodge_status lodge_dssim_scratch_size(int32_t width, int32_t height, int32_t channels, size_t* bytes);

/* ASYNC.  The D-SSIM term of the construction loss (the paper's DSSIM + L1):
 * SSIM of image and target ([channels][height][width], device) per channel
 * with the 11 x 11 Gaussian window of sigma 1.5, C1 = 0.01^2, C2 = 0.03^2 and
 * zero padding; grad (device, same shape) receives
 *   grad += weight * d(1 - mean SSIM) / d image,
 * and loss (device float, NULL to skip) += weight * (1 - mean SSIM) (one
 * atomic per block).  Run lodge_l1_grad first with scale (1 - lambda) / n and
 * this with weight lambda for the 3DGS loss (1 - lambda) L1 + lambda D-SSIM.
 * scratch: device, lodge_dssim_scratch_size bytes, caller-owned. */
lodge_status lodge_dssim_grad(int32_t width, int32_t height, int32_t channels, const float* image, const float* target,
                              float weight, float* grad, float* loss, void* scratch, size_t scratch_bytes,
                              void* stream);

/* Bytes of device scratch lodge_keep_indices needs for n items (n < 2^32). */
lodge_status lodge_keep_scratch_size(int64_t n, size_t* bytes);

/* ASYNC.  Importance pruning of one level: idx (device, n entries of room)
 * receives, ascending, the indices i < n with score[i] >= threshold, and
 * *count (device) their number.  scratch: device, lodge_keep_scratch_size
 * bytes, caller-owned. */
lodge_status lodge_keep_indices(int64_t n, const float* score, float threshold, uint32_t* idx, uint32_t* count,
                                void* scratch, size_t scratch_bytes, void* stream);

/* ASYNC.  Compaction of `planes` planes of n_in floats (in: [planes][n_in],
 * device) to the kept items: out[p][j] = in[p][idx[j]] for j < min(*count,
 * n_out) (out: [planes][n_out], device).  Indices >= n_in are skipped. */
lodge_status lodge_gather_planes(int32_t planes, int64_t n_in, int64_t n_out, const float* in, const uint32_t* idx,
                                 const uint32_t* count, float* out, void* stream);

/* ------------------------------------- measurement and verification helpers */

/* Not part of the method: the device's achievable rates, against which the
 * kernels' roofline fractions are reported beside the data-sheet peaks, and
 * the FP32 division and square root of the library's build. */

/* ASYNC.  Copies `bytes` (a multiple of 16) from src to dst (device, 16-byte
 * aligned, not overlapping) with a coalesced streaming kernel: the HBM rate
 * of a kernel that reads and writes once is 2 * bytes over its time.
 * LODGE_ERR_INVALID_ARG for NULL or misaligned buffers. */
lodge_status lodge_microbench_copy(const void* src, void* dst, size_t bytes, void* stream);

/* The grid lodge_microbench_read uses for `bytes`: *blocks blocks of 256
 * threads (out then needs *blocks x 256 floats). */
lodge_status lodge_microbench_read_blocks(size_t bytes, uint32_t* blocks);

/* ASYNC.  Reads `bytes` (a multiple of 16) of src (device, 16-byte aligned)
 * with a coalesced streaming kernel of `blocks` blocks of 256 threads (the
 * count lodge_microbench_read_blocks gives), each thread writing the sum of
 * what it read to out[thread] (device, blocks x 256 floats): the HBM rate of
 * a kernel that only reads is bytes over its time.  LODGE_ERR_INVALID_ARG for
 * NULL or misaligned buffers or blocks == 0. */
lodge_status lodge_microbench_read(const void* src, size_t bytes, float* out, uint32_t blocks, void* stream);

/* ASYNC.  q[i] = a[i] / b[i] and r[i] = sqrt(a[i]) for i < n (device
 * buffers), compiled with the library's flags.  The selection, tile
 * rectangles and depth keys match an IEEE FP32 evaluation bit for bit only
 * if these are correctly rounded; this call lets a test compare them with
 * the host's.  LODGE_ERR_INVALID_ARG for a NULL buffer. */
lodge_status lodge_fp32_div_sqrt(const float* a, const float* b, float* q, float* r, size_t n, void* stream);

/* ASYNC.  blocks x 256 threads, each running 8 independent chains of `iters`
 * dependent FP32 FMAs x <- fma(x, a, b) from x = 0..7, and writing the sum of
 * its chains to out[thread] (device, blocks x 256 floats): 8 * iters * 256 *
 * blocks non-packed VALU lane-ops.  LODGE_ERR_INVALID_ARG for out == NULL or
 * blocks == 0. */
lodge_status lodge_microbench_fma(float* out, uint32_t blocks, uint32_t iters, float a, float b, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LODGE_H */

/*
 * gs.h -- C ABI of the MI355X (gfx950) batched 3D Gaussian Splatting
 * training step: Gaussians x cameras -> images, loss -> parameter gradients,
 * and the optimizer step with the batch-size scaling rules.
 *
 * Paper: "On Scaling Up 3D Gaussian Splatting Training" (arXiv 2406.18533).
 * Each entry point cites the passage that defines the operation it runs.
 *
 * Conventions shared by every call
 * --------------------------------
 * - All pointers are DEVICE memory unless marked [host]. The caller allocates
 *   and owns every buffer; the library never allocates on these paths and
 *   keeps no pointer after a call returns (a captured HIP graph keeps the
 *   pointers, so the caller keeps those buffers alive while it replays).
 * - Every call is stream-ordered on `stream` and returns without waiting for
 *   the device, except gs_bin_sort with check = 1.
 * - dtype selects the arithmetic type of every floating-point buffer of the
 *   call: GS_F32 (the training path) or GS_F64 (used for finite-difference
 *   checks). Index and count buffers are integers whatever dtype is.
 * - Errors: a call returns GS_OK or a negative gs_status and then leaves its
 *   outputs unspecified; gs_last_error() returns a message for the calling
 *   thread. No C++ exception crosses this boundary.
 *
 * Gaussian parameters (section 2 "3D Gaussian Splatting", four learnable
 * quantities per Gaussian: position, scale + rotation, opacity, 48 SH values)
 * are one planar block params[59][n] (row-major, row stride n):
 *   rows 0-2 mean (world), 3-5 log-scale, 6-9 quaternion (w, x, y, z; it is
 *   normalised inside), 10 opacity logit, 11 + 3k + c the degree-3 SH
 *   coefficient k = l*l + l + m of colour channel c.
 * Gradients and both Adam moments use the same layout.
 *
 * Images: views are concatenated in call order; view v holds rgb [3][H][W]
 * and one value per pixel [H][W] for final transmittance and last position.
 * Pixel (x, y) has its centre at (x + 1/2, y + 1/2).
 *
 * Tiles: 16x16 pixel blocks (section 3.1 "Pixel-wise Distribution"),
 * serialised across the batch: global tile id = tiles of earlier views +
 * ty * ceil(W/16) + tx.
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_VERSION_STRING "gsmi 1.0 gfx950"
#define GS_TILE 16
#define GS_MAX_VIEWS 64
#define GS_PARAM_ROWS 59
#define GS_REC 12           /* scalars per projected record and per projected-gradient record */

typedef enum {
    GS_OK = 0,
    GS_ERR_ARG = -1,          /* invalid argument (null pointer, size, view count, dtype) */
    GS_ERR_CAPACITY = -2,     /* more sorted instances than bins->capacity */
    GS_ERR_HIP = -3,          /* a HIP runtime call or kernel launch failed */
    GS_ERR_UNSUPPORTED = -4   /* device is not gfx950 */
} gs_status;

typedef enum { GS_F32 = 0, GS_F64 = 1 } gs_dtype;

/* A pinhole camera. R is world -> camera (row-major), t its translation, so a
 * world point x maps to R x + t in the camera frame (+x right, +y down, +z
 * forward); the camera centre is -R^T t. Pixels project to
 * (fx X/Z + cx, fy Y/Z + cy). Gaussians with Z <= znear are culled.
 * Image sides are 1..65536 pixels with at most 2^22 16x16 tiles per view
 * (e.g. 32768 x 32768); other sizes are rejected with GS_ERR_ARG. */
typedef struct gs_camera {
    int32_t width, height;
    double fx, fy, cx, cy;
    double R[9];
    double t[3];
    double znear;
} gs_camera;

/* Sorted instance buffers: the per-pixel depth-ordered lists of intersecting
 * Gaussians that the paper calls the Z-buffer (appendix A.2 "Z-buffer"),
 * stored per 16x16 tile. */
typedef struct gs_bins {
    int64_t capacity;         /* entries of tile_keys and ids; < 2^32 */
    uint32_t *tile_keys;      /* [capacity] global tile id of each sorted instance */
    uint32_t *ids;            /* [capacity] Gaussian index of each sorted instance */
    uint32_t *ranges;         /* [total_tiles][2] start, end into ids; (0, 0) when empty */
    int64_t *n_instances;     /* [1] instance count K (may exceed capacity) */
    int32_t *overflow;        /* [1] 1 if K > capacity, else 0 */
    void *workspace;          /* gs_bin_workspace_bytes(n, views, capacity, total_tiles) */
    size_t workspace_bytes;
} gs_bins;

#define GS_SCHED_PER_TILE 0    /* one workgroup per tile, XCD-aware tile order */
#define GS_SCHED_PERSISTENT 1  /* persistent workgroups, cost-balanced chunks + stealing */
#define GS_SCHED_XCD_SPLIT 2   /* one workgroup per tile; each XCD takes one of 8 cost-balanced
                                  contiguous chunks of the serialised tiles (Algorithm 1, G = 8) */
#define GS_SCHED_LPT 3         /* one workgroup per tile, tiles in decreasing estimated cost
                                  (longest processing time first); tile_cost NULL = per-tile */
#define GS_SCHED_XCD_LPT 4     /* the XCD split, each chunk's tiles in decreasing estimated cost;
                                  tile_cost NULL = per-tile */
#define GS_SCHED_LPT_HEAD 5    /* the heaviest eighth of the tiles first in decreasing estimated
                                  cost, then the rest in index order; tile_cost NULL = per-tile */

/* Launch shape of the two render kernels and the state of the persistent
 * scheduler (the single-GPU counterpart of section 3.2 "Iterative Workload
 * Rebalancing" and Algorithm 1 "Calculation of Division Points"). In
 * persistent mode each gs_render_fwd / gs_render_bwd call first runs
 * Algorithm 1 on tile_cost (see gs_sched_plan), then launches `workers`
 * workgroups that take tiles from the `queues` cost-balanced chunks. In
 * XCD-split mode it runs Algorithm 1 with 8 chunks (queues is ignored) and
 * launches one workgroup per tile, the workgroups of XCD x (b mod 8 = x)
 * taking chunk x: the 8 XCDs, each with its own L2, play the part of the
 * paper's GPUs. In LPT mode it orders the tiles by decreasing tile_cost (a
 * counting sort over cost classes 2^(1/4) apart) and workgroup b takes the
 * b-th: the greedy longest-processing-time-first rule for the makespan of
 * a queue of tasks on identical workers; the workspace holds the order. In
 * XCD-LPT mode it runs Algorithm 1 with 8 chunks as in the XCD split and
 * orders each chunk's tiles by decreasing tile_cost. LPT-head mode orders
 * only the heaviest cost classes holding an eighth of the tiles, the rest
 * following in index order (their neighbours share L2 lines). */
typedef struct gs_sched {
    int32_t mode;             /* GS_SCHED_PER_TILE, _PERSISTENT, _XCD_SPLIT, _LPT, _XCD_LPT or _LPT_HEAD */
    int32_t px_per_thread;    /* 1, 2 or 4: 256, 128 or 64 threads per 16x16 tile */
    int32_t chunk;            /* records staged in LDS per step: 32, 64, 128 or 256 */
    int32_t workers;          /* persistent workgroups (0 = as many as fit on the GPU at once) */
    int32_t queues;           /* Algorithm 1 chunks, a multiple of 8 (0 = 64) */
    int32_t reserved;
    const uint32_t *tile_cost;/* [total_tiles] estimated cost per tile (NULL = uniform) */
    void *workspace;          /* gs_sched_workspace_bytes(total_tiles, queues) */
    size_t workspace_bytes;
} gs_sched;

/* Adam hyper-parameters [host]. lr[g] is the base learning rate of group g:
 * 0 rows 0-2 (mean), 1 rows 3-5 (log-scale), 2 rows 6-9 (quaternion),
 * 3 row 10 (opacity), 4 rows 11-13 (SH degree 0), 5 rows 14-58 (SH degree >= 1). */
typedef struct gs_adam_hparams {
    double lr[6];
    double beta1, beta2, eps;
    int32_t batch_size;       /* b: lr * sqrt(b), beta^b */
    int32_t zero_grad;        /* 1: write 0 into grad after the update */
} gs_adam_hparams;

/* Densification thresholds [host] (appendix A.1). A Gaussian is selected
 * when its statistic count c > 0 and sum s >= grad_threshold * c (compared in
 * double); selected Gaussians whose largest log-scale exceeds
 * split_log_scale are split, the others cloned. A Gaussian (or a clone, or a
 * split child) is pruned when its opacity logit < prune_logit or its largest
 * log-scale > prune_log_scale; a child's largest log-scale is its parent's
 * minus log(1.6), so children are pruned when the parent's exceeds
 * prune_log_scale + log(1.6). Comparing logits and log-scales (not opacities
 * and scales) keeps every decision exact on the stored values. */
typedef struct gs_densify_hparams {
    double grad_threshold;    /* on the mean of the per-view statistic (pixels) */
    double split_log_scale;   /* log(percent_dense * scene extent) in 3DGS terms */
    double prune_logit;       /* log(o_min / (1 - o_min)) */
    double prune_log_scale;   /* log of the largest world scale kept (+inf: no size pruning) */
} gs_densify_hparams;

/* ------------------------------------------------------------------ library */
const char *gs_version(void);
/* Message of the last failed call on this thread ("" if none). */
const char *gs_last_error(void);
/* Checks that `device` is a gfx950 GPU and makes it current for later calls
 * from this thread. GS_ERR_UNSUPPORTED otherwise. */
gs_status gs_init(int32_t device);

/* ------------------------------------------------------------------ sizes */
/* Bytes of a projected buffer: views * n records of GS_REC scalars, then two
 * planar uint32 side arrays [views][n] (tiles touched, FP32 depth bits) and
 * one planar uint64 array [views][n] (tile rectangle). */
size_t gs_projected_bytes(gs_dtype dtype, int64_t n, int32_t views);
/* Sum over the views of ceil(W/16) * ceil(H/16) [host cameras]; -1 (with
 * gs_last_error set) when a camera is rejected. */
int64_t gs_total_tiles(const gs_camera *cams_host, int32_t views);
/* Total pixels over the views [host cameras]; -1 as above. */
int64_t gs_total_pixels(const gs_camera *cams_host, int32_t views);
size_t gs_bin_workspace_bytes(int64_t n, int32_t views, int64_t capacity, int64_t total_tiles);
size_t gs_sched_workspace_bytes(int64_t total_tiles, int32_t queues);
size_t gs_loss_workspace_bytes(const gs_camera *cams_host, int32_t views);
/* Workspace of gs_loss_l1_dssim: three coefficient maps of 3 H W scalars
 * per view (dtype), then one double per (tile, channel) and 64 more. 0
 * (with gs_last_error set) when a camera or the dtype is rejected. */
size_t gs_loss_dssim_workspace_bytes(gs_dtype dtype, const gs_camera *cams_host, int32_t views);

/* ------------------------------------------------------------------ forward */
/* Gaussian transformation (section 2.1, step 1): for every view v and
 * Gaussian i, the on-screen position x_{v,i}, depth_{v,i}, footprint radius
 * radius_{v,i} and view-dependent colour c_{v,i}. Writes projected
 * [views][n][GS_REC] records:
 *   0 u, 1 v, 2-4 conic (a, b, c) = inverse of the 2x2 screen covariance,
 *   5 opacity, 6-8 rgb, 9 radius (integer valued), 10 depth, 11 tiles touched.
 * The screen covariance is J W Sigma W^T J^T + 0.3 I with Sigma =
 * R(q) diag(exp(2 l)) R(q)^T and J the perspective Jacobian at the centre
 * (its x/z, y/z clamped to 1.3x the half field of view); radius =
 * ceil(3 sqrt(largest eigenvalue)); rgb = max(0, SH(direction) + 1/2).
 * After the records the buffer holds, for every (view, Gaussian), tiles
 * touched and the FP32 bits of depth as planar uint32 arrays, then the
 * touched tile rectangle as a planar uint64 array (tile columns x0, x1 and
 * rows y0, y1, inclusive, in 16-bit fields from the low end) (see
 * gs_projected_bytes). Only pairs that touch a tile are written: their
 * record, depth bits and rectangle. For every other pair (culled: behind
 * znear or non-finite; or off-screen) only tiles touched = 0 is written, and
 * its record, depth bits and rectangle keep whatever the buffer held; readers
 * select records by the side array's tiles touched.
 * params: [59][n]. cams_dev: [views] cameras in device memory (read by the
 * kernel, so a captured graph sees updated poses); cams_host: the same
 * cameras [host] (image sizes). Requires 1 <= views <= GS_MAX_VIEWS,
 * views * n < 2^32 and one view's records under 4 GiB (n < 89M in FP32,
 * 44M in FP64); GS_ERR_ARG otherwise. */
gs_status gs_project(gs_dtype dtype, const void *params, int64_t n, const gs_camera *cams_dev,
                     const gs_camera *cams_host, int32_t views, void *projected, void *stream);

/* Z-buffer construction (section 2.1 step 2 intersection test; appendix A.2):
 * every (view, Gaussian) with tiles touched > 0 emits one instance per tile
 * of its footprint rectangle, and the instances are sorted by
 * (global tile, FP32 bits of depth, Gaussian index) - a (view, tile, depth)
 * radix sort - then [start, end) is found for every tile.
 * The rectangle is the bounding box of the footprint circle over pixel
 * centres clipped to the image, decided in FP32:
 *   x in [ceil(u - r - 1/2), floor(u + r - 1/2)], likewise y.
 * If K > capacity nothing is written past capacity, *overflow = 1 and the
 * bins are unusable. check = 1 waits for the stream and returns
 * GS_ERR_CAPACITY in that case; check = 0 never synchronises (graph-safe).
 * projected: output of gs_project for the same n and cameras. */
gs_status gs_bin_sort(gs_dtype dtype, const void *projected, int64_t n, const gs_camera *cams_host,
                      int32_t views, gs_bins *bins, int32_t check, void *stream);

/* Test helper: 64-bit keys (tile << 32 | FP32 depth bits) of the first
 * min(K, capacity) sorted instances into keys_out [capacity]. */
gs_status gs_bins_keys64(gs_dtype dtype, const void *projected, int64_t n, const gs_camera *cams_host,
                         int32_t views, const gs_bins *bins, uint64_t *keys_out, void *stream);

/* Rendering (section 2.1 step 2): per pixel, walk its tile's list in order;
 * a Gaussian intersects the pixel if the pixel centre lies within radius of
 * (u, v); alpha = min(0.99, opacity exp(-(a dx^2 + c dy^2)/2 - b dx dy)) is
 * skipped below 1/255; the walk stops before a Gaussian that would bring the
 * transmittance T below 1e-4; otherwise C += rgb alpha T, T *= 1 - alpha.
 * Writes rgb = C + T bg, final_T and last (list position after the last
 * blended Gaussian) for every pixel. Optional (nullable) per global tile:
 * tile_work_fwd = list entries walked, tile_work_bwd = max of last; the
 * scheduler uses them as the next cost estimates. pair_stats: nullable [2]
 * device counters, incremented by (pixel, Gaussian) pairs evaluated and
 * blended (a separate kernel variant; for measurement). bg: [host] 3
 * floats. sched: launch shape; NULL = per-tile, 256 threads, chunk 64. */
gs_status gs_render_fwd(gs_dtype dtype, const void *projected, int64_t n, const gs_bins *bins,
                        const gs_camera *cams_host, int32_t views, const float *bg, const gs_sched *sched,
                        void *rgb, void *final_T, uint32_t *last, uint32_t *tile_work_fwd,
                        uint32_t *tile_work_bwd, uint64_t *pair_stats, void *stream);

/* Back-propagation through rendering and transformation (section 2.1,
 * "standard approaches to backpropagation"; appendix A.3: render backward is
 * pixel-wise, transformation backward Gaussian-wise): gs_render_bwd_pixels
 * followed by gs_project_bwd with clear = 1. dprojected [views][n][GS_REC]
 * must be all zero on entry (allocate it zeroed once) and is all zero again
 * on return. Adds (+=) the parameter gradients into grad [59][n]. */
gs_status gs_render_bwd(gs_dtype dtype, const void *params, int64_t n, const void *projected,
                        const gs_bins *bins, const gs_camera *cams_dev, const gs_camera *cams_host,
                        int32_t views, const float *bg, const gs_sched *sched, const void *final_T,
                        const uint32_t *last, const void *dL_drgb, void *dprojected, void *grad,
                        void *stream);

/* Render backward (pixel-wise half). Given dL/drgb, recomputes the blend of
 * every pixel in reverse from final_T and last (T_k = T_{k+1} / (1 - alpha_k),
 * colour behind k composed from the background forward), and adds (+=) the
 * per-(view, Gaussian) gradients of (u, v, a, b, c, opacity, r, g, b) into
 * slots 0-8 of dprojected [views][n][GS_REC]. bins, final_T and last must
 * come from the gs_bin_sort / gs_render_fwd of the same projected buffer. */
gs_status gs_render_bwd_pixels(gs_dtype dtype, const void *projected, int64_t n, const gs_bins *bins,
                               const gs_camera *cams_host, int32_t views, const float *bg,
                               const gs_sched *sched, const void *final_T, const uint32_t *last,
                               const void *dL_drgb, void *dprojected, void *stream);

/* Transformation backward (Gaussian-wise half): chain rule from dprojected
 * through colour (SH, clamp mask, view direction), conic, EWA covariance,
 * perspective Jacobian (zero through a clamped coordinate), camera
 * transform, rotation (with the normalisation), scale and sigmoid, summed
 * over the views and added (+=) into grad [59][n]. Depth, radius and the
 * tile rectangle carry no gradient. clear = 1 zeroes the dprojected records
 * it read (those with tiles touched > 0), leaving dprojected all zero. */
gs_status gs_project_bwd(gs_dtype dtype, const void *params, int64_t n, const gs_camera *cams_dev,
                         const gs_camera *cams_host, int32_t views, const void *projected,
                         void *dprojected, int32_t clear, void *grad, void *stream);

/* Loss (section 2.1 step 3, L1 part): loss = (scale/views) sum_v mean over
 * the 3 H W values of |rgb - target|, the batch loss being the mean of
 * per-view losses (section 4, g = sum_k g_k / b). Writes dL_drgb =
 * scale sign(rgb - target) / (3 H W views) (sign(0) = 0) and *loss_dev (one
 * double, device). scale = 1 for a batch; a caller that walks a batch of b
 * views one view at a time passes 1/b. workspace: gs_loss_workspace_bytes.
 * Deterministic. */
gs_status gs_loss_l1(gs_dtype dtype, const void *rgb, const void *target, const gs_camera *cams_host,
                     int32_t views, double scale, void *dL_drgb, double *loss_dev, void *workspace,
                     size_t workspace_bytes, void *stream);

/* Loss (section 2.1 step 3, both terms: L1 per pixel and SSIM over pixel
 * windows): per view, over its 3 H W values,
 *   loss_v = (1 - lam) mean |rgb - target| + lam (1 - mean SSIM),
 * SSIM computed per colour channel over an 11x11 Gaussian window of standard
 * deviation 1.5 (normalised), zero padding outside the image, C1 = 0.01^2,
 * C2 = 0.03^2: SSIM = (2 mx my + C1)(2 cov + C2) / ((mx^2 + my^2 + C1)
 * (var_x + var_y + C2)) from the window's means, variances and covariance.
 * *loss_dev = (scale / views) sum_v loss_v (one double, device; summed per
 * 16x16 tile and channel, then over those in a fixed order: deterministic).
 * dL_drgb (like rgb) = the exact gradient of that loss with respect to rgb
 * (sign(0) = 0 for the L1 part). lam in [0, 1]. The paper names the two
 * terms but not their weight, window or constants: the window and
 * constants are SSIM's definition (Wang, Bovik, Sheikh, Simoncelli, IEEE
 * Trans. Image Processing 13(4), 2004) and lam = 0.2 the weight of the 3D
 * Gaussian splatting loss (Kerbl et al., ACM Trans. Graphics 42(4), 2023).
 * rgb/target: [3][H][W] per view, views concatenated; values are not
 * clamped. workspace: gs_loss_dssim_workspace_bytes; its contents on return
 * are scratch. The gradient is written by a second pass over coefficient
 * maps the first pass leaves in the workspace, so dL_drgb must not alias
 * rgb or target. */
gs_status gs_loss_l1_dssim(gs_dtype dtype, const void *rgb, const void *target, const gs_camera *cams_host,
                           int32_t views, double lam, double scale, void *dL_drgb, double *loss_dev,
                           void *workspace, size_t workspace_bytes, void *stream);

/* Render forward with the L1 loss fused into its output stage: everything
 * gs_render_fwd writes (without pair_stats), plus dL_drgb exactly as
 * gs_loss_l1 writes it for the same rgb (bit for bit: the gradient at a
 * pixel depends only on its final colour, so it is written as the pixel
 * finishes) and *loss_dev, the same loss summed per tile and then over the
 * tiles in a fixed order (deterministic; equal to gs_loss_l1's value up to
 * the order of the double-precision sum). target/dL_drgb: like rgb.
 * workspace: gs_loss_workspace_bytes (one double per tile, plus 64 for the
 * block sums of the final reduction). */
gs_status gs_render_fwd_l1(gs_dtype dtype, const void *projected, int64_t n, const gs_bins *bins,
                           const gs_camera *cams_host, int32_t views, const float *bg, const gs_sched *sched,
                           void *rgb, void *final_T, uint32_t *last, uint32_t *tile_work_fwd,
                           uint32_t *tile_work_bwd, const void *target, double scale, void *dL_drgb,
                           double *loss_dev, void *workspace, size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): gs_render_fwd_l1
 * without the workspace argument. The per-tile loss shares and their block
 * sums live in a fixed scratch array inside the library, one per device,
 * held until the process ends (GS_NOALLOC_MAX_TILES + 64 doubles, 8 MiB).
 * Calls with more than GS_NOALLOC_MAX_TILES tiles over the views return
 * GS_ERR_ARG. Every call on a device shares that device's scratch, so calls
 * that overlap on one device (other streams, other threads) race and must be
 * ordered by the caller; a call leaves only scratch contents that the next
 * call overwrites before reading. Outputs and every other argument exactly as
 * gs_render_fwd_l1. */
#define GS_NOALLOC_MAX_TILES (1 << 20)
gs_status gs_render_fwd_l1_noalloc(gs_dtype dtype, const void *projected, int64_t n, const gs_bins *bins,
                                   const gs_camera *cams_host, int32_t views, const float *bg, const gs_sched *sched,
                                   void *rgb, void *final_T, uint32_t *last, uint32_t *tile_work_fwd,
                                   uint32_t *tile_work_bwd, const void *target, double scale, void *dL_drgb,
                                   double *loss_dev, void *stream);

/* ------------------------------------------------------------------ optimizer */
/* Adam with the batch scaling rules of section 4: learning rate
 * lr * sqrt(batch_size) (eq. "lambda") and beta1^b, beta2^b (eq. "beta").
 * Every element of params/grad/m/v ([59][n]) is updated (dense):
 *   t = ++(*step_dev); m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
 *   p -= (lr' / (1 - b1^t)) m / (sqrt(v) / sqrt(1 - b2^t) + eps).
 * step_dev: [1] device step counter, incremented on the device so graph
 * replays advance it. scratch: [2] device doubles for the bias corrections.
 * skip_flag: nullable device int32; when it holds a non-zero value (e.g. the
 * bins overflow flag of this step) the update is skipped: params, moments
 * and the step counter stay unchanged (grad is still zeroed if asked).
 * h: [host]. */
gs_status gs_adam_step(gs_dtype dtype, void *params, void *grad, void *m, void *v, int64_t n,
                       const gs_adam_hparams *h, int64_t *step_dev, double *scratch,
                       const int32_t *skip_flag, void *stream);

/* Transformation backward fused with the Adam step: the parameter gradient
 * that gs_project_bwd (clear = 1) would add into an all-zero grad is applied
 * to params/m/v exactly as gs_adam_step applies it (same arithmetic in the
 * same order, so params, m and v equal the two calls bit for bit), without
 * writing the gradient out: the Gaussian-wise gradient (appendix A.3) and the
 * dense optimizer update (section 4) become one pass over the parameters.
 * dprojected is consumed and left all zero, as with clear = 1. grad [59][n]
 * is scratch that must be all zero on entry and is all zero again on return
 * (rows 0-2 carry part of the position gradient between the two kernels).
 * step_dev, scratch, skip_flag and h as for gs_adam_step; a skipped step
 * still consumes dprojected. */
gs_status gs_project_bwd_adam(gs_dtype dtype, void *params, int64_t n, const gs_camera *cams_dev,
                              const gs_camera *cams_host, int32_t views, const void *projected,
                              void *dprojected, void *grad, void *m, void *v, const gs_adam_hparams *h,
                              int64_t *step_dev, double *scratch, const int32_t *skip_flag, void *stream);

/* ------------------------------------------------------------------ densification */
/* Densification statistic (appendix A.1: position variance across steps,
 * read as the gradient of the loss w.r.t. each Gaussian's projected
 * centre). For every view v and Gaussian i whose record touches a tile
 * (tiles touched > 0): accum[i] += scale * |(dL/du, dL/dv)| of that record in
 * dprojected (pixels), count[i] += 1. Pass scale = batch size so that each
 * term is the gradient of that view's own loss. Call it after the render
 * backward and before gs_project_bwd / gs_project_bwd_adam, which clear
 * dprojected. accum [n] float, count [n] int32, device; both accumulate
 * (zero them to start a new interval). */
gs_status gs_densify_stats(gs_dtype dtype, const void *projected, const void *dprojected, int64_t n,
                           int32_t views, double scale, float *accum, int32_t *count, void *stream);

/* Bytes of workspace for gs_densify_plan / gs_densify_apply on n Gaussians. */
size_t gs_densify_workspace_bytes(int64_t n);

/* Densification, first half: classifies every Gaussian with the rules of
 * gs_densify_hparams and counts the output per class. Writes counts_dev[3]
 * (device int64): kept originals K, clones C, split pairs S; the output has
 * K + C + 2 S Gaussians. The classes and per-block offsets stay in the
 * workspace for gs_densify_apply; read counts_dev on the host to size the
 * output. params [59][n]. */
gs_status gs_densify_plan(gs_dtype dtype, const void *params, int64_t n, const float *accum,
                          const int32_t *count, const gs_densify_hparams *h, void *workspace,
                          size_t workspace_bytes, int64_t *counts_dev, void *stream);

/* Densification, second half: writes the new parameters and Adam moments
 * [59][n_out], n_out = K + C + 2 S from the plan, in this order: kept
 * originals, clones (exact copies), first split children, second split
 * children, each group in index order. A split child k of Gaussian i has
 * mean + R(q) (exp(log-scale) * noise[k][.][i]), log-scale - log(1.6) and
 * every other parameter of i; the split parent is removed. Moments are
 * copied for kept originals and zero for clones and children. noise:
 * [2][3][n] standard normal draws (device, dtype), supplied by the caller so
 * that results are reproducible. The workspace must hold the plan of the
 * same params and h; outputs must not alias inputs. Writes beyond n_out are
 * never made, whatever the plan says. */
gs_status gs_densify_apply(gs_dtype dtype, const void *params, const void *m, const void *v, int64_t n,
                           const void *noise, const void *workspace, size_t workspace_bytes, void *params_out,
                           void *m_out, void *v_out, int64_t n_out, void *stream);

/* Opacity reset (appendix A.1): opacity logit = min(logit, max_logit) for
 * every Gaussian; the opacity row of m and v is zeroed. In place. */
gs_status gs_reset_opacity(gs_dtype dtype, void *params, void *m, void *v, int64_t n, double max_logit,
                           void *stream);

/* ------------------------------------------------------------------ scheduler */
/* Algorithm 1 ("Calculation of Division Points") on the device with G =
 * Q = sched->queues: CT = cumsum(ET) with ET_j = tile_cost[j] + 1,
 * thresholds q * CT[last] / Q, DP = left searchsorted, DP[Q] = total tiles.
 * Queue q = serialised tiles [DP[q], DP[q+1]) belongs to XCD q div (Q/8), so
 * consecutive (spatially adjacent) chunks share an XCD's L2; an idle
 * persistent workgroup steals from the other queues of its XCD first, then
 * from other XCDs. Resets the queue cursors. The render calls run it
 * themselves in persistent mode; it is exported for tests.
 * dp_out: optional [queues + 1] int32 copy of DP (device). */
gs_status gs_sched_plan(const gs_sched *sched, const gs_camera *cams_host, int32_t views,
                        int32_t *dp_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* GS_H */

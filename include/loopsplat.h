/*
 * loopsplat.h - C ABI of the MI355X (gfx950) Gaussian-splat rasterizer and
 * 3DGS registration library (libloopsplat.so).
 *
 * The operations follow LoopSplat (Zhu et al., "LoopSplat: Loop Closure by
 * Registering 3D Gaussian Splats"):
 *   - a submap is a set of 3D Gaussians with mean, covariance, opacity and RGB
 *     colour (Sec. 3.1, Eq. 1); the covariance is parametrised by per-axis
 *     scales (Sec. 3.1, Eq. 5) and a rotation quaternion;
 *   - colour and depth are rendered from a pose and compared with RGB-D
 *     measurements through L1 losses (Sec. 3.1 tracking loss, Eq. 2; Sec. 3.2
 *     registration loss);
 *   - the pose is optimised as a rigid correction applied to the submap in
 *     the frame of the previous camera (supplement, frame-to-model tracking);
 *   - registration localises every keyframe of one submap in the other and
 *     fuses the per-view estimates by weighted rotation averaging (Sec. 3.2,
 *     Eq. 7), optionally with per-view exposure coefficients (supplement);
 *   - the submap-update loss mixes L1 and SSIM for colour, L1 for depth and an
 *     isotropic scale regulariser (Sec. 3.1, Eq. 3-5);
 *   - after pose-graph optimisation submaps and keyframes are moved by their
 *     corrections (Sec. 3.3, Eq. 8); loop candidates are filtered by the
 *     geometric overlap ratio of two submaps (supplement, Eq. 9).
 *
 * Conventions shared by every call
 *   - Every call returns an ls_status.  Negative values are errors; the detail
 *     string is available from ls_last_error() (thread-local).  No call
 *     throws or aborts.
 *   - All tensor arguments are float32/int32 *device* pointers owned by the
 *     caller unless stated otherwise; the library never frees them.
 *   - Device work is enqueued on the given HIP stream and is asynchronous
 *     unless the call says it blocks.  Calls that share a workspace must be
 *     ordered on one stream.
 *   - Gaussians are structure-of-arrays: mean [3][n], log_scale [3][n],
 *     quat [4][n] = (w, x, y, z) unnormalised, opacity_logit [n], rgb [3][n].
 *   - A pose is 7 floats (q_w, q_x, q_y, q_z, t_x, t_y, t_z): a rigid
 *     correction Delta applied in camera coordinates after the job's
 *     world-to-camera transform, p = R(q/|q|) (R_cw mu + t_cw) + t.
 *   - Camera axes: x right, y down, z forward; pixel (i, j) is sampled at
 *     (i + 0.5, j + 0.5).
 *   - Images of render r are planar: rgb [3][H_r][W_r] starting at float
 *     offset 3 * pix_off[r]; depth/alpha/T_final/n_last [H_r][W_r] starting
 *     at pix_off[r], where pix_off is the exclusive prefix sum of H_r * W_r.
 *   - "Item" i = item_off[r] + g names Gaussian g of render r, item_off being
 *     the exclusive prefix sum of the jobs' Gaussian counts.
 */
#ifndef LOOPSPLAT_H
#define LOOPSPLAT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ls_status;
#define LS_OK 0
#define LS_NOT_READY 1
#define LS_ERR_INVALID (-1)   /* bad argument; nothing was enqueued */
#define LS_ERR_CAPACITY (-2)  /* a buffer is too small; required size reported */
#define LS_ERR_BUDGET (-3)    /* request larger than the server's memory budget */
#define LS_ERR_HIP (-4)       /* a HIP runtime call failed */
#define LS_ERR_NONFINITE (-5) /* non-finite input or loss */

/* Rasterizer constants (readings of the 3D Gaussian Splatting renderer the
 * paper builds on; the paper does not restate them). */
#define LS_TILE 16              /* 16x16-pixel tiles */
#define LS_NEAR_Z 0.2f          /* cull z <= 0.2 m */
#define LS_EPS_2D 0.3f          /* 2D low-pass dilation, px^2 */
#define LS_ALPHA_MIN (1.0f / 255.0f)
#define LS_ALPHA_MAX 0.99f
#define LS_T_STOP 1e-4f
#define LS_REC_FLOATS 12        /* floats per projected record, see ls_projected */

const char* ls_last_error(void);
/* Library version as major * 10000 + minor * 100 + patch. */
int32_t ls_version(void);
/* sizeof of a public struct named by its type name (e.g. "ls_render_job"),
 * or -1 for an unknown name; lets a binding verify its layouts without a GPU. */
int64_t ls_struct_size(const char* name);

typedef struct {
  int32_t n;                  /* number of Gaussians (>= 0) */
  const float* mean;          /* [3][n] metres, in the job's world frame */
  const float* log_scale;     /* [3][n] log of the per-axis standard deviations */
  const float* quat;          /* [4][n] (w, x, y, z), any non-zero length */
  const float* opacity_logit; /* [n]    opacity = sigmoid(opacity_logit) */
  const float* rgb;           /* [3][n] colour, used as given (no SH) */
} ls_gaussians;

typedef struct {
  float fx, fy, cx, cy; /* pinhole intrinsics in pixels */
  int32_t width, height;
} ls_intrinsics;

/* One render: a Gaussian set seen by one camera (Sec. 3.1 renders a submap
 * at a keyframe pose).  w2c is a row-major 3x4 world-to-camera transform. */
typedef struct {
  ls_gaussians g;
  ls_intrinsics K;
  float w2c[12];
} ls_render_job;

/* A batch of R render jobs that share every launch.  Created once (it uploads
 * the job table to the device), reused across iterations; the Gaussian arrays
 * the jobs point to must stay allocated (their values may change). */
typedef struct ls_batch ls_batch;

typedef struct {
  int32_t renders;        /* R */
  int64_t items;          /* M = sum of n over jobs */
  int32_t tiles;          /* total 16x16 tiles over all renders */
  int64_t pixels;         /* total pixels over all renders */
  size_t workspace_bytes; /* bytes of ls_bins.work needed for the queried capacity */
} ls_batch_info;

/* Creates a batch from R >= 1 jobs (host array, copied).  Allocates the
 * device job table.  Errors: LS_ERR_INVALID for R < 1, n < 0, non-positive
 * image sizes or focal lengths, or NULL Gaussian arrays with n > 0. */
ls_status ls_batch_create(const ls_render_job* jobs, int32_t R, ls_batch** out);
ls_status ls_batch_destroy(ls_batch* b);
/* Sizes of the batch and the workspace needed for `capacity` tile instances. */
ls_status ls_batch_query(const ls_batch* b, int64_t capacity, ls_batch_info* info);
/* Host copies of the per-render offsets: item_off, pix_off [R+1] and
 * tile_off [R+1] (any may be NULL). */
ls_status ls_batch_offsets(const ls_batch* b, int64_t* item_off, int64_t* pix_off, int32_t* tile_off);

/* Projected splats, one record per item, caller-owned device buffers.
 *   rec    [M][12]: (u, v, A, B,  C, opacity, z, 0,  r, g, b, 0) where (u, v)
 *          is the projected centre in pixels, (A, B, C) the conic (inverse
 *          2D covariance, sigma = A dx^2/2 + B dx dy + C dy^2/2), z the
 *          camera-space depth.  16-byte aligned.
 *   radius [M]: ceil(3 sqrt(lambda_max(Sigma_2D))) in pixels, 0 = culled
 *   tiles  [M]: number of tiles of the item's tile rectangle, 0 = culled
 *   aux    [M][12] or NULL: camera-space mean (x, y, z) and covariance
 *          (xx, xy, xz, yy, yz, zz), 0, 0, 0 - kept by the forward for the
 *          backward; required by ls_render_bwd*.  16-byte aligned.
 * rec and aux of a culled item are left as they were (only its radius and
 * tiles, 0, are written). */
typedef struct {
  float* rec;
  int32_t* radius;
  int32_t* tiles;
  float* aux;
} ls_projected;

/* EWA projection of every item (the splatting step the paper's renderer
 * inherits from 3D Gaussian Splatting; Sec. 3.1 Eq. 1 parameters).
 *   pose: device [R][7] pose corrections, or NULL for identity.
 * Per item: Sigma = R(q) diag(s)^2 R(q)^T, camera transform W = R(q_d) R_cw,
 * Sigma_2D = J W Sigma W^T J^T + 0.3 I with the perspective Jacobian J at the
 * camera-space mean; culled when z <= 0.2 m, det <= 0 or the tile rectangle
 * [floor((u-r)/16), floor((u+r)/16)+1) x (same in v), clamped to the image's
 * tile grid, is empty.  Errors: LS_ERR_INVALID (NULL outputs). */
ls_status ls_project(const ls_batch* b, const float* pose, const ls_projected* out, hipStream_t s);

/* Tile instance lists, caller-owned device buffers.
 *   capacity     number of instance slots in tile_of / item
 *   tile_of [capacity] global tile index (tile_off[r] + ty * tiles_x + tx)
 *   item    [capacity] item index of each instance
 *   range   [tiles][2] [start, end) of each tile's list (empty tiles: 0, 0)
 *   count   [4] int32: {instances kept = min(I, capacity), overflow flag,
 *           instances required I, 0}
 *   work    workspace of ls_batch_info.workspace_bytes (256-byte aligned),
 *           zero-filled by the caller before its first use; also used by
 *           ls_render_bwd (the persistent backward kernels keep their
 *           tile-queue counters here and leave them zero). */
typedef struct {
  int64_t capacity;
  uint32_t* tile_of;
  int32_t* item;
  int32_t* range;
  int32_t* count;
  void* work;
} ls_bins;

/* Tile binning: every item with tiles > 0 is listed once in each tile of its
 * rectangle (recomputed in FP32 from rec.u, rec.v and radius), and the list
 * is ordered by (tile, FP32 depth bit pattern, item) - depth order with ties
 * broken by Gaussian index.  Runs entirely on the device (depth radix sort of
 * the items, scan, emission, tile radix sort).  When I > capacity, count[1]
 * is set to 1, only the first `capacity` instances are kept and the lists are
 * not valid; the caller re-runs with capacity >= count[2].  Errors:
 * LS_ERR_INVALID (NULL buffers, capacity < 0). */
ls_status ls_bin_sort(const ls_batch* b, const ls_projected* p, const ls_bins* bins, hipStream_t s);

typedef struct {
  float* rgb;      /* see image layout above */
  float* depth;    /* sum_i w_i z_i (not normalised by alpha) */
  float* alpha;    /* 1 - T_final */
  float* T_final;  /* final transmittance */
  int32_t* n_last; /* list entries visited before compositing stopped */
} ls_image;

/* Front-to-back compositing (RGB, depth, alpha) per 16x16 tile: for each
 * pixel and each entry of its tile's list in order, alpha = min(0.99,
 * o exp(-sigma)); entries with sigma < 0 or alpha < 1/255 are skipped; the
 * loop stops before the entry that would take T below 1e-4; otherwise
 * w = alpha T, C += w c, D += w z, T *= 1 - alpha.  rgb gets + T bg.
 * bg: host float[3] or NULL (zero).  It also records in bins->work which
 * list entries each 8x8 band of a tile composited; the backward calls read
 * those records, so `fwd` passed to them must be this call's output on the
 * same bins (no ls_render_fwd or ls_bin_sort on them in between). */
ls_status ls_render_fwd(const ls_batch* b, const ls_projected* p, const ls_bins* bins, const float* bg,
                        const ls_image* out, hipStream_t s);

/* Upstream gradients dL/d(image), same layouts as ls_image (any may be NULL
 * = zero); scale: device [R] per-render factor applied to all three, or NULL. */
typedef struct {
  const float* rgb;
  const float* depth;
  const float* alpha;
  const float* scale;
} ls_image_grad;

/* Gradient outputs (accumulated with +=) for one render's Gaussian set, same
 * SoA layouts as ls_gaussians; NULL members are not computed. */
typedef struct {
  float* mean;
  float* log_scale;
  float* quat;
  float* opacity_logit;
  float* rgb;
} ls_gaussian_grads;

/* Adam state of one parameter array of a Gaussian set (fused backward):
 * first and second moments (device, the array's layout) and its rate. */
typedef struct {
  float* m;
  float* v;
  float lr;
} ls_adam_array;

/* Per render: the five arrays in ls_gaussians order. */
typedef struct {
  ls_adam_array mean, log_scale, quat, opacity_logit, rgb;
} ls_gaussian_adam;

/* Adam state of the renders' pose corrections: device [R][7] moments and
 * the rates of the quaternion and translation parts. */
typedef struct {
  float* m;
  float* v;
  float lr_rot;
  float lr_trans;
} ls_pose_adam;

#define LS_ADAM_FUSED_MAX_RENDERS 16

/* Backward of ls_project + ls_render_fwd (= ls_render_bwd_tiles followed by
 * ls_render_bwd_project).  Recomputes the per-pixel transmittance back to
 * front from T_final / n_last (no per-pixel lists are stored), walking only
 * the list entries the last ls_render_fwd on these bins composited in each
 * band (fwd must be that call's output), reduces the per-Gaussian image-space
 * gradients within each tile, then chains them through the projection.
 *   grads:     host array [R] of per-render outputs, or NULL (pose only).
 *              Jobs sharing a Gaussian set may share output arrays.
 *   pose_grad: device [R][7], accumulated, or NULL; needs `pose`.
 * Two modes:
 *   - full (grads != NULL): per-tile sums of each Gaussian's image-space
 *     gradients are added to a per-item accumulator in ls_bins.work (float
 *     atomics, so reproducible to rounding, not bitwise); the accumulator must
 *     be zero before the first backward on a workspace and
 *     ls_render_bwd_project clears it again;
 *   - pose only (grads == NULL, LS_BWD_POSE_ONLY): each Gaussian's pose
 *     Jacobian is applied inside the tile and a 12-value partial is written
 *     per tile, summed per render in a fixed order: no atomics, bit-identical
 *     results that do not depend on the other renders of the batch.
 * Errors: LS_ERR_INVALID. */
ls_status ls_render_bwd(const ls_batch* b, const float* pose, const ls_projected* p, const ls_bins* bins,
                        const float* bg, const ls_image* fwd, const ls_image_grad* up,
                        const ls_gaussian_grads* grads, float* pose_grad, hipStream_t s);

/* First half of ls_render_bwd: per tile, back-to-front recomputation and the
 * per-(item, tile) sums of dL/d(u, v, conic, opacity, z, rgb) (one kernel).
 * flags: LS_BWD_POSE_ONLY keeps only what a pose correction depends on (u, v,
 * conic, z) and turns it into per-tile pose partials (`pose` may be NULL =
 * identity). */
#define LS_BWD_POSE_ONLY 1u
ls_status ls_render_bwd_tiles(const ls_batch* b, const float* pose, const ls_projected* p, const ls_bins* bins,
                              const float* bg, const ls_image* fwd, const ls_image_grad* up, uint32_t flags,
                              hipStream_t s);

/* ls_loss_l1 followed by ls_render_bwd_tiles, fused (Sec. 3.2 loss, as
 * ls_loss_l1 defines it): the per-pixel gradient, sign(x - x*) on Omega
 * times inv_count[r] for each colour channel and the depth (0 outside Omega),
 * is formed inside the compositing backward from the forward images and the
 * targets, so no gradient images are written or read.  Each tile also stores
 * its sum of the loss terms and its count of pixels in Omega in the bins
 * workspace, from which ls_loss_l1_tiles forms the loss.
 *   fwd        the forward's images: rgb, depth, T_final and n_last are read
 *   tgt_rgb, tgt_depth: device targets in the batch's image layout
 *   inv_count  device [R]: 1 / |Omega| per render, as ls_loss_l1 writes it to
 *              grad_scale for the same targets (it depends on them only)
 *   flags      0 (full mode, as ls_render_bwd_tiles) or LS_BWD_POSE_ONLY
 * The Gaussian and pose gradients equal those of ls_loss_l1 +
 * ls_render_bwd_tiles bit for bit in pose-only mode and up to the order of
 * the float atomics in full mode.  Errors: LS_ERR_INVALID (missing images,
 * targets or inv_count, unknown flags). */
ls_status ls_render_bwd_tiles_l1(const ls_batch* b, const float* pose, const ls_projected* p, const ls_bins* bins,
                                 const float* bg, const ls_image* fwd, const float* tgt_rgb, const float* tgt_depth,
                                 const float* inv_count, uint32_t flags, hipStream_t s);

/* The L1 loss of the last ls_render_bwd_tiles_l1 on these bins: loss (device
 * [R], written) = (1/|Omega|) sum over Omega of the per-pixel terms, as
 * ls_loss_l1 computes it but summed tile by tile (equal to its value up to
 * FP32 rounding); 0 for a render with no pixel in Omega. */
ls_status ls_loss_l1_tiles(const ls_batch* b, const ls_bins* bins, float* loss, hipStream_t s);

/* Second half of ls_render_bwd: chains the accumulated image-space gradients
 * through the EWA projection to the Gaussian parameters and the pose (full
 * mode), or sums the per-tile pose partials of each render (LS_BWD_POSE_ONLY;
 * grads must be NULL). */
ls_status ls_render_bwd_project(const ls_batch* b, const float* pose, const ls_projected* p, const ls_bins* bins,
                                const ls_gaussian_grads* grads, float* pose_grad, uint32_t flags, hipStream_t s);

/* Work statistics of the last forward: stats (device int64 [2], written)
 * receives {list entries evaluated (every entry up to and including the one
 * that stopped compositing), entries composited (alpha >= 1/255)} summed
 * over all pixels. */
ls_status ls_render_stats(const ls_batch* b, const ls_projected* p, const ls_bins* bins, const ls_image* fwd,
                          int64_t* stats, hipStream_t s);

/* Registration / tracking L1 loss (Sec. 3.2: L = L_col + L_depth, both L1;
 * Sec. 3.1 Eq. 2 without masks): per render
 *   L_r = (1/|Omega|) sum_{p in Omega} (sum_c |C_c - C*_c| + |D - D*|),
 * Omega = pixels with target depth > 0.
 *   loss      device [R] (written), or NULL
 *   grad_rgb, grad_depth: device, image layout; receive sign(x - x*) on
 *             Omega and 0 elsewhere (sign(0) = 0)
 *   grad_scale device [R]: receives 1/|Omega| (0 when Omega is empty), to be
 *             passed as ls_image_grad.scale. */
ls_status ls_loss_l1(const ls_batch* b, const ls_image* pred, const float* tgt_rgb, const float* tgt_depth,
                     float* loss, float* grad_rgb, float* grad_depth, float* grad_scale, hipStream_t s);

/* Weights and masks of the tracking loss (Sec. 3.1 Eq. 2 and the
 * supplement's tracking-loss details). */
typedef struct {
  float lambda_c;       /* colour weight in [0, 1]; depth gets 1 - lambda_c */
  float inlier_k;       /* inlier mask: keep pixels whose depth error is <= inlier_k x the
                           median depth error of the render (50); <= 0: no inlier mask */
  int32_t alpha_power;  /* soft alpha mask M_a = alpha^alpha_power (3); 0: no alpha mask */
  int32_t pad;
} ls_loss_params;

/* Tracking loss with masks (Sec. 3.1 Eq. 2; supplement, tracking loss): per
 * render
 *   L_r = (1/|Omega|) sum_{p in Omega} M_in M_a (lc sum_c |C_c - C*_c| + (1 - lc)|D - D*|)
 * with Omega = pixels whose target depth is > 0 (pixels without a depth
 * measurement are excluded), M_a = alpha^k a per-pixel weight through which
 * no gradient flows, and M_in = [e <= inlier_k * med], e = |D - D*| in FP32,
 * med = the lower median of e over Omega (rank floor((|Omega|-1)/2)),
 * selected exactly.  Normalising by |Omega| rather than summing scales every
 * view's loss by a constant, which leaves Adam's steps unchanged.
 *   pred      rendered images; pred->alpha is required when alpha_power > 0
 *   loss      device [R] (written), or NULL
 *   median    device [R] (written) or NULL (kept inside the batch)
 *   grad_rgb, grad_depth: device, image layout; receive M_in M_a lc sign(C - C*)
 *             and M_in M_a (1 - lc) sign(D - D*) (0 outside Omega)
 *   grad_scale device [R]: receives 1/|Omega| (0 when Omega is empty).
 * Calls on one batch share its selection workspace: do not overlap them. */
ls_status ls_loss_tracking(const ls_batch* b, const ls_image* pred, const float* tgt_rgb, const float* tgt_depth,
                           const ls_loss_params* prm, float* loss, float* median, float* grad_rgb, float* grad_depth,
                           float* grad_scale, hipStream_t s);

/* Weights of the submap-update (mapping) loss, Sec. 3.1 Eq. 3 and Eq. 4;
 * the supplement sets lambda_color = lambda_depth = 1 (and lambda_reg = 1,
 * see ls_loss_isotropic); the paper gives no lambda_ssim (0.2 is the usual
 * value). */
typedef struct {
  float lambda_ssim;   /* weight of (1 - SSIM) inside the colour term, in [0, 1] */
  float lambda_color;  /* weight of the colour term */
  float lambda_depth;  /* weight of the depth term */
  int32_t pad;
} ls_mapping_params;

/* Image part of the mapping loss (Sec. 3.1 Eq. 3 and Eq. 4): per render
 *   L_r = lc ((1 - ls) L1_rgb + ls (1 - SSIM)) + ld L1_depth,
 *   L1_rgb   = (1/|Omega|) sum_{p in Omega} sum_c |C_c - C*_c|,
 *   L1_depth = (1/|Omega|) sum_{p in Omega} |D - D*|   (0 when Omega is empty),
 * Omega = pixels with target depth > 0.  SSIM is the mean over the three
 * colour channels and all pixels of the windowed index of Wang et al. with an
 * 11 x 11 Gaussian window (sigma 1.5, weights summing to 1), zero padding
 * outside the image, C1 = 0.01^2, C2 = 0.03^2, moments E[xy] - mu_x mu_y.
 *   loss       device [R] (written), or NULL
 *   grad_rgb, grad_depth: device, image layout, or NULL; receive dL_r/dC and
 *              dL_r/dD with every weight and normalisation applied
 *   grad_scale device [R] (written with 1), or NULL: pass it as
 *              ls_image_grad.scale like the other losses' scales.
 * Uses the batch's loss scratch: do not overlap with another loss call on
 * the same batch.  Errors: LS_ERR_INVALID (NULL images or targets, weights
 * not finite or lambda_ssim outside [0, 1]). */
ls_status ls_loss_mapping(const ls_batch* b, const ls_image* pred, const float* tgt_rgb, const float* tgt_depth,
                          const ls_mapping_params* prm, float* loss, float* grad_rgb, float* grad_depth,
                          float* grad_scale, hipStream_t s);

/* Isotropic regulariser of one submap (Sec. 3.1 Eq. 5):
 *   L = lambda_reg (1/K) sum_k sum_j |s_kj - mean_j(s_kj)|,  s = exp(log_scale),
 * the mean over the three axes being differentiated through.
 *   log_scale       device [3][n] (the ls_gaussians layout), n >= 0
 *   loss            device [1] (written; 0 when n = 0)
 *   grad_log_scale  device [3][n], accumulated (+=), or NULL
 *   work            device scratch of LS_ISOTROPIC_WORK_FLOATS floats
 * The sum is taken in a fixed order (bit-reproducible).  Errors: LS_ERR_INVALID. */
#define LS_ISOTROPIC_WORK_FLOATS 256
ls_status ls_loss_isotropic(const float* log_scale, int64_t n, float lambda_reg, float* loss, float* grad_log_scale,
                            float* work, hipStream_t s);

/* One submap of a globally consistent map adjustment (Sec. 3.3, Eq. 8). */
typedef struct {
  int32_t n;        /* Gaussians (>= 0) */
  int32_t n_poses;  /* keyframe poses (>= 0; ignored when c2w is NULL) */
  float* mean;      /* device [3][n], updated in place */
  float* quat;      /* device [4][n] (w, x, y, z, any norm), updated in place */
  float* c2w;       /* device [n_poses][12] row-major 3x4 camera-to-world, updated in place, or NULL */
  float T[12];      /* host: the submap's correction [R_c | t_c], row-major 3x4; R_c a rotation */
} ls_submap_adjust;

/* Applies each submap's pose-graph correction in place (Sec. 3.3, Eq. 8):
 *   mu <- R_c mu + t_c;  Sigma <- R_c Sigma R_c^T, realised as q <- q_c q
 *   (Hamilton product with the unit quaternion of R_c, so |q| is kept and
 *   scales, opacities and colours are untouched);  T_j <- T_c T_j.
 * Up to 32 submaps share a launch; any count is accepted.  Arrays of
 * different submaps must not overlap.  Errors: LS_ERR_INVALID (count < 0,
 * NULL arrays with n > 0, a non-finite T or an R_c that is not a rotation to
 * 1e-3: |R^T R - I| or det R <= 0). */
ls_status ls_adjust_submaps(const ls_submap_adjust* subs, int32_t count, hipStream_t s);

/* Geometric overlap ratio of two submaps (supplement, loop detection, Eq. 9):
 *   OR = (1/|K|) sum_{(p,q) in K} [ |T(p) - q| < tau ],
 * K = reciprocal nearest neighbours between the Gaussian means of P moved by
 * T (an estimate of T_{P->Q}) and those of Q.  Nearest neighbours are exact
 * under FP32 decisions with a fixed rounding sequence (no fused multiply-add):
 * T(p)_r = ((R_r0 x + R_r1 y) + R_r2 z) + t_r, d^2 = (dx^2 + dy^2) + dz^2,
 * ties to the lower index; the test is d^2 < fl32(tau^2).
 *   p_mean, q_mean  device [3][np], [3][nq] (the ls_gaussians layout)
 *   T_pq            host, row-major 3x4
 *   nn_pq, nn_qp    device [np], [nq] (written): index of the nearest point of
 *                   the other set (-1 when that set is empty)
 *   counts          device int32 [2] (written): {|K|, pairs closer than tau};
 *                   OR = counts[1] / counts[0] (0 when |K| = 0)
 *   work            device scratch of ls_overlap_workspace_size(np, nq) bytes
 * The means must be finite (they are not checked; a non-finite coordinate
 * gives unspecified matches).  ls_overlap_workspace_size returns 0 for
 * negative counts.  Errors: LS_ERR_INVALID (sizes, NULL arrays, non-finite T,
 * tau not > 0), LS_ERR_CAPACITY (work_bytes too small). */
size_t ls_overlap_workspace_size(int32_t np, int32_t nq);
ls_status ls_overlap_ratio(const float* p_mean, int32_t np, const float* q_mean, int32_t nq, const float* T_pq,
                           float tau, int32_t* nn_pq, int32_t* nn_qp, int32_t* counts, void* work, size_t work_bytes,
                           hipStream_t s);

/* ls_overlap_ratio for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops and harnesses that forbid
 * hipMalloc): the same computation and results, with the workspace taken
 * from a library-owned static device array of LS_OVERLAP_NOALLOC_BYTES
 * (40 MiB), one copy per GPU, held until the process ends.  The caller still
 * passes inputs and outputs.  Calls no hipMalloc, hipFree or allocating
 * library routine.  The first call on a device looks up the array's device
 * address (hipGetSymbolAddress) with that device current; make that first
 * call outside stream capture.  Every call on a device shares its array,
 * which keeps the last call's contents (nothing in it needs clearing), so
 * calls that overlap on one device - on different streams or from different
 * threads without ordering - race and must not be issued.  The stream must
 * belong to the current device.  Errors: as ls_overlap_ratio, and
 * LS_ERR_CAPACITY when np or nq exceeds LS_OVERLAP_NOALLOC_MAX_POINTS. */
#define LS_OVERLAP_NOALLOC_MAX_POINTS 524288
#define LS_OVERLAP_NOALLOC_BYTES (40u << 20)
ls_status ls_overlap_ratio_noalloc(const float* p_mean, int32_t np, const float* q_mean, int32_t nq,
                                   const float* T_pq, float tau, int32_t* nn_pq, int32_t* nn_qp, int32_t* counts,
                                   hipStream_t s);

/* One structure-of-arrays array compacted by ls_prune_gaussians:
 * src [components][n] -> dst [components][count] (rows count floats apart,
 * the ls_gaussians layout for the new count; dst must hold components * n
 * floats, as count is only known on the device).  src and dst must not
 * overlap. */
typedef struct {
  const float* src;
  float* dst;
  int32_t components;
  int32_t pad;
} ls_prune_array;
#define LS_PRUNE_MAX_ARRAYS 16

/* Opacity pruning of a submap after its mapping optimisation (supplement,
 * Implementation Details, submap update): the Gaussians whose opacity
 * sigmoid(opacity_logit) is below o_thre are removed, the others kept in
 * their order.  The test is taken on the FP32 logit against the FP32
 * rounding of ln(o_thre / (1 - o_thre)): kept <=> logit >= that value (a
 * Gaussian at the threshold is kept; a NaN logit is pruned).
 *   opacity_logit device [n]
 *   arrays        host [narrays] (0..LS_PRUNE_MAX_ARRAYS) arrays to compact
 *                 with the same selection (Gaussian parameters, optimiser
 *                 moments, ...); the opacity logits themselves only if listed
 *   kept_index    device int32 [n] (written): the kept Gaussians' indices,
 *                 ascending, in its first count entries
 *   count         device int32 [1] (written): number kept
 *   work          device scratch of ls_prune_workspace_size(n) bytes
 * Errors: LS_ERR_INVALID (n < 0, o_thre outside (0, 1), NULL pointers,
 * too many arrays, components < 0), LS_ERR_CAPACITY (work too small). */
size_t ls_prune_workspace_size(int32_t n);
ls_status ls_prune_gaussians(const float* opacity_logit, int32_t n, float o_thre, const ls_prune_array* arrays,
                             int32_t narrays, int32_t* kept_index, int32_t* count, void* work, size_t work_bytes,
                             hipStream_t s);

/* One parameter group of a fused Adam step. */
typedef struct {
  float* param;
  float* grad; /* zeroed after use when zero_grad is set */
  float* m;
  float* v;
  int64_t n;
  float lr;
} ls_adam_group;

/* Adam (beta1, beta2, eps; bias correction with step count `step` >= 1)
 * over up to 16 groups in one launch.  The paper gives learning rates but
 * does not name the optimiser (supplement hyper-parameter tables). */
ls_status ls_adam(const ls_adam_group* groups, int32_t ngroups, int32_t step, float beta1, float beta2,
                  float eps, int32_t zero_grad, hipStream_t s);

/* ls_render_bwd_project (full mode) with one Adam step fused in, for the
 * mapping and tracking iterations (Sec. 3.1): each Gaussian's gradient of
 * this backward goes straight into an Adam update (beta1, beta2, eps, bias
 * correction of `step` >= 1, as ls_adam) of the parameters its render job
 * points to, updated in place, so the gradients never go to memory.  Culled
 * Gaussians step with zero gradients, as ls_adam does for every element.
 * Given the same gradients, the same arithmetic as ls_render_bwd_project
 * into zeroed gradient arrays followed by ls_adam over those five arrays
 * (the gradients themselves carry the float-atomic ordering of the tile
 * backward).
 *   adam:      host [R], one per render (R <= LS_ADAM_FUSED_MAX_RENDERS);
 *              renders may not share a Gaussian array (a shared set's
 *              gradient is only complete after all of its renders)
 *   pose_grad: device [R][7], accumulated, or NULL; needs `pose`
 *   pose_adam: NULL, or the poses' Adam state: then each render's pose takes
 *              the same step in the pose reduction (pose updated in place,
 *              pose_grad, required, consumed and zeroed), as ls_adam over
 *              pose_grad would
 * Errors: LS_ERR_INVALID (NULL state, too many renders, shared arrays, step
 * < 1, bad constants, pose_adam without pose and pose_grad). */
ls_status ls_render_bwd_project_adam(const ls_batch* b, float* pose, const ls_projected* p, const ls_bins* bins,
                                     const ls_gaussian_adam* adam, const ls_pose_adam* pose_adam, int32_t step,
                                     float beta1, float beta2, float eps, float* pose_grad, hipStream_t s);

/* Fills `count` int32 words at `ptr` with `value` (a kernel, never a memset
 * node, so it is safe inside captured graphs). */
ls_status ls_fill_i32(int32_t* ptr, int64_t count, int32_t value, hipStream_t s);

/* ---------------------------------------------------------------------------
 * 3DGS registration as keyframe localisation (Sec. 3.2).
 *
 * Submaps P and Q are each reconstructed from their own keyframes and are not
 * aligned; T_{P->Q} maps P's frame into Q's.  Every keyframe i of P (pose T_i
 * in P's frame, measurements (I, D)_i) is localised in Q: Q is rendered with
 * world-to-camera Delta_i o T_i^-1 and Delta_i is optimised (Q fixed) for the
 * colour + depth loss (plain L1, or the tracking loss of Eq. 2 with its masks,
 * which discount content one submap never observed), giving
 * E_i = T_i Delta_i^-1 T_i^-1 ~ T_{P->Q}.
 * Keyframes of Q are localised in P the same way (estimates of T_{Q->P}).
 * The 2V estimates are fused by weighted rotation averaging with weights
 * 1/eps_i (Eq. 7) and a weighted mean of the translations.
 * ------------------------------------------------------------------------- */

typedef struct {
  ls_gaussians P, Q;     /* device Gaussian sets, each in its own submap frame */
  int32_t vP, vQ;        /* keyframes of P and of Q (vP + vQ >= 1) */
  const float* rgbP;     /* device [vP][3][H][W] measurements of P's keyframes */
  const float* depthP;   /* device [vP][H][W]; pixels with depth <= 0 are not used */
  const float* c2wP;     /* host   [vP][12] row-major 3x4 camera-to-world, P's frame */
  const float* rgbQ;     /* device [vQ][3][H][W] */
  const float* depthQ;   /* device [vQ][H][W] */
  const float* c2wQ;     /* host   [vQ][12], Q's frame */
  ls_intrinsics K;       /* shared by all keyframes */
} ls_pair;

typedef struct {
  int32_t iters;            /* Adam iterations per view (>= 1): the maximum when early exit is on */
  float lr_rot, lr_trans;   /* learning rates of the quaternion and the translation */
  float beta1, beta2, adam_eps;
  float exit_rel_tol;       /* early exit: a view stops once its loss has not improved on its best */
  int32_t exit_patience;    /* by more than exit_rel_tol (relative) for exit_patience iterations; 0 = off
                               (see exit_mode for the step rule) */
  int32_t loss_kind;        /* 0: plain L1 (ls_loss_l1); 1: tracking loss with masks (ls_loss_tracking) */
  ls_loss_params track;     /* weights and masks when loss_kind == 1 */
  int32_t exposure;         /* 1: per-view exposure coefficients (supplement, 3DGS registration): the
                               rendered colour enters the loss and the residual as exp(a) C + b, with
                               scalars a, b per view starting at 0 and taking the pose's Adam step;
                               0: off.  A server fixes it (and lr_exposure) with its first request */
  float lr_exposure;        /* their learning rate (0.1 in the supplement) */
  int32_t joint;            /* 1: one T_{P->Q} shared by all views, each view's correction derived from
                               it, Adam on T (lr_rot, lr_trans) over the sum of the views' losses; T is
                               the estimate (no Eq. 7 fusion).  A comparison to the paper's per-view
                               estimates; ls_register_pair only, without exposure or early exit */
  int32_t exit_mode;        /* early exit rule when exit_patience > 0: 0 the loss plateau above; 1 the
                               pose step: a view stops once the largest |m_hat| / (sqrt(v_hat) + eps)
                               of its Adam update (the step in units of the learning rate) has stayed
                               below exit_rel_tol for exit_patience iterations */
  int32_t top_k;            /* views kept per direction (0: all).  The paper keeps the top-k (k = 2)
                               overlapping viewpoints found by image retrieval (Sec. 3.2; supplement,
                               3DGS registration); here a keyframe's overlap is its rendered
                               co-visibility: the fraction of its pixels with a measured depth that
                               the other submap, rendered at the keyframe pose (identity correction),
                               covers with alpha >= 0.5; ties go to the lower keyframe index.  Views
                               not kept report residual -1 and a zero estimate.  ls_register_pair only */
} ls_reg_params;

typedef struct {
  float T_PQ[12];     /* fused T_{P->Q}, row-major 3x4 */
  float* per_view_T;  /* host [vP + vQ][12] or NULL: E_i (P views: ~T_{P->Q}; Q views: ~T_{Q->P}) */
  float* residual;    /* host [vP + vQ] or NULL: eps_i, the unmasked colour + depth L1 (ls_loss_l1)
                         of each view at its final pose, whichever loss drove it */
  int32_t status;     /* LS_OK, or the error of this pair */
  int32_t iters_done; /* Adam steps of the longest-running view */
  float* exposure;    /* host [vP + vQ][2] or NULL: each view's final (a, b) when exposure is on */
  int64_t instances_required; /* ls_register_pair, LS_ERR_CAPACITY: tile instances needed (0 if the
                                 workspace, not the capacity, was short) */
  int64_t workspace_required; /* ls_register_pair: bytes of workspace the call needed */
} ls_reg_result;

/* Device bytes of the workspace ls_register_pair needs for `pair` with room
 * for `capacity` tile instances (all views' 16x16-tile lists together).
 * Host-only: no device work.  Errors: LS_ERR_INVALID (as ls_register_pair,
 * or capacity outside [0, INT32_MAX]). */
ls_status ls_register_workspace_size(const ls_pair* pair, const ls_reg_params* prm, int64_t capacity,
                                     size_t* bytes);

/* Registers one pair (Sec. 3.2: every keyframe of P localised in Q and every
 * keyframe of Q in P, then the Eq. 7 fusion) with all 2V views in one launch
 * set per iteration.  Blocks until the result is on the host.  All device
 * memory of the call is the caller's workspace `work` (work_bytes >=
 * ls_register_workspace_size(pair, prm, capacity), 256-byte aligned; no
 * allocation inside the call; contents need no initialisation and are
 * scratch afterwards); `capacity` bounds the tile instances of all views at
 * any iteration.  When the lists outgrow it (at the starting poses or during
 * the optimisation) the call returns LS_ERR_CAPACITY with
 * out->instances_required set: the caller re-runs with a larger capacity
 * (with headroom: the count changes as the poses move).  A short workspace
 * returns LS_ERR_CAPACITY with out->workspace_required set.  Errors:
 * LS_ERR_INVALID (bad sizes, NULL pointers), LS_ERR_NONFINITE (non-finite
 * poses or loss), LS_ERR_CAPACITY, LS_ERR_HIP. */
ls_status ls_register_pair(const ls_pair* pair, const ls_reg_params* prm, void* work, size_t work_bytes,
                           int64_t capacity, ls_reg_result* out, hipStream_t s);

/* Host-only fusion of per-view estimates (Eq. 7 + weighted translation mean):
 * est [n][12] row-major 3x4, resid [n], reverse [n] (1 for a Q->P estimate,
 * inverted before averaging) -> out [12].  Weights 1/max(eps, 1e-12); the
 * rotation maximises tr(R^T sum_i w_i R_i) over SO(3).  No GPU needed. */
ls_status ls_fuse_estimates(const double* est, const double* resid, const int32_t* reverse, int32_t n, double* out);

/* ---------------------------------------------------------------------------
 * Registration serving loop.  Loop edges are requested as submap pairs arrive
 * (Sec. 3.3: every detected loop is registered before pose-graph
 * optimisation); the server keeps admitted pairs resident and runs all of
 * their keyframe localisations together.
 *   - submit queues a request and returns a ticket (thread-safe);
 *   - a worker thread admits queued requests first-in first-out while the
 *     estimated device bytes of the active set stay within the budget and a
 *     slot is free (continuous batching at iteration granularity: requests
 *     that arrive while others run join at the next chunk boundary, finished
 *     ones leave and free their slot);
 *   - one Adam iteration over every view of every active pair is one launch
 *     set, captured once per change of the active set as a HIP graph and
 *     replayed;
 *   - finished pairs are fused on the host (Eq. 7) and posted to their ticket.
 * The caller keeps each pair's device buffers alive until its ticket's poll
 * returns a final status.
 * ------------------------------------------------------------------------- */

typedef struct ls_server ls_server;

typedef struct {
  size_t hbm_budget_bytes;  /* device bytes the server may use for resident work */
  int32_t max_slots;        /* pairs running at once (>= 1) */
  int32_t chunk_iters;      /* iterations between admission / retirement points (>= 1) */
  float instance_headroom;  /* tile-instance capacity = headroom x count measured at each rebuild
                               (>= 0.25; below 1 deliberately undersizes it, which exercises the
                               overflow-recovery path: the chunk is re-run with more room) */
  int32_t use_graphs;       /* 1: capture + replay iterations; 0: launch eagerly */
  int64_t max_active_pixels;/* admission cap on the pixels rendered per iteration by the active set
                               (0: none).  The head of the queue is admitted only into an empty
                               active set or while the sum stays within the cap.  Once one pair
                               fills the GPU, admitting more shares it between them and delays
                               every result; a cap near the size that fills the device keeps large
                               pairs first-come first-served and still batches small ones. */
} ls_server_params;

typedef struct {
  int64_t submitted, completed, failed;
  int64_t epochs;            /* active-set changes (batch rebuilds) */
  int64_t iterations;        /* batched iterations run */
  int64_t graph_replays;
  int64_t overflow_retries;  /* chunks re-run after the instance capacity overflowed */
  int64_t peak_bytes;        /* peak estimated bytes of the active set */
  int32_t active, waiting;
  int32_t peak_active;       /* most pairs active at once */
  int32_t pad;
} ls_server_stats;

/* Creates a server on the current device with its own worker thread and
 * stream.  Errors: LS_ERR_INVALID (bad parameters), LS_ERR_HIP. */
ls_status ls_server_create(const ls_server_params* prm, ls_server** out);
/* Queues a pair (copied; device pointers referenced).  The server reads the
 * pair's device buffers on its own streams: every read is ordered after the
 * work queued on `producer` at the time of the call (an event is recorded
 * there), so buffers still being written on that stream are read complete;
 * with producer NULL the buffers must already be complete.  Errors:
 * LS_ERR_INVALID (including Adam beta1/beta2/eps different from the first
 * request the server saw), LS_ERR_NONFINITE (non-finite keyframe poses or
 * Gaussian parameters; checked on the device before queueing, after the
 * producer's work), LS_ERR_BUDGET (the pair alone exceeds the budget). */
ls_status ls_register_submit(ls_server* sv, const ls_pair* pair, const ls_reg_params* prm, hipStream_t producer,
                             uint64_t* ticket);
/* LS_NOT_READY while the ticket runs; otherwise fills `out` (per_view_T and
 * residual when non-NULL) and `times` (double [3] or NULL: seconds from
 * submit to admission, admission to completion, submit to completion),
 * releases the ticket and returns its final status (LS_OK, or e.g.
 * LS_ERR_NONFINITE when the optimisation diverged). */
ls_status ls_register_poll(ls_server* sv, uint64_t ticket, ls_reg_result* out, double* times);
ls_status ls_server_get_stats(ls_server* sv, ls_server_stats* out);
/* Finishes every submitted request, then stops the worker and frees the
 * server.  Tickets not yet polled are released. */
ls_status ls_server_destroy(ls_server* sv);

#ifdef __cplusplus
}
#endif
#endif /* LOOPSPLAT_H */

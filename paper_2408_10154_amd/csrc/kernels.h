// Host-side launchers of the gfx950 kernels (defined next to each kernel).
#pragma once

#include "common.h"

namespace ls {

// Error reporting of the C ABI (api.cpp): set the thread's ls_last_error()
// text and return `st`; turn a pending HIP error into LS_ERR_HIP.
ls_status api_fail(ls_status st, const char* msg);
ls_status api_hip_check(const char* what);

void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);

struct ViewOpt;
// live (or NULL: every render) gates each render on its active flag: the
// items of a frozen render project to radius 0, so it has no tile instances.
void launch_project(const JobDev* jobs, const int32_t* blk_off, int R, int nblk, const float* pose, float* rec,
                    int32_t* radius, int32_t* tiles, float* aux, const ViewOpt* live, hipStream_t s);

// One Adam update of a parameter from its gradient, with explicit FMAs so
// that every kernel applying it (k_adam, the fused backward) gives the same
// bits.
__device__ __forceinline__ void adam_update(float& p, float& m, float& v, float g, float lr, float beta1, float beta2,
                                            float eps, float bc1, float bc2) {
  m = __builtin_fmaf(beta1, m, (1.f - beta1) * g);
  v = __builtin_fmaf(beta2, v, (1.f - beta2) * g * g);
  p -= lr * (m * bc1) / (sqrtf(v * bc2) + eps);
}

// Adam state of the fused projection backward: per render (at most
// kAdamRenders) and per parameter array (mean, log_scale, quat, opacity,
// rgb) the moments and the learning rate; bias corrections of the step.
constexpr int kAdamRenders = 16;
struct GaussAdamArgs {
  float* m[kAdamRenders][5];
  float* v[kAdamRenders][5];
  float lr[kAdamRenders][5];
  float beta1, beta2, eps, bc1, bc2;
  // optional pose step in the pose reduction: [R][7] pose and moments (NULL: none)
  float* pose;
  float* pose_m;
  float* pose_v;
  float lr_rot, lr_trans;
};

// adam (or NULL): instead of accumulating the Gaussian gradients into grads,
// apply one Adam step to each Gaussian's parameters (the arrays its render
// job points to) from its gradient; culled items step with zero gradients.
void launch_project_bwd(const JobDev* jobs, const int32_t* blk_off, int R, int nblk, const float* pose,
                        const int32_t* radius, const float* aux, float* g2d, const GradDev* grads, int want_gauss,
                        float* pose_part, int want_pose, float* pose_grad, hipStream_t s,
                        const GaussAdamArgs* adam = nullptr);
void launch_pose_reduce_tiles(const JobDev* jobs, int R, const float* pose, const float* tile_part, float* pose_grad,
                              hipStream_t s);

// tile_bits: bits of the largest tile key (T - 1), which set the tile passes.
void launch_bin_sort(const JobDev* jobs, const int64_t* item_off_d, int R, int64_t M, int T, int tile_bits,
                     const float* rec, const int32_t* radius, const int32_t* tiles, int64_t cap, uint32_t* tile_of,
                     int32_t* item, int32_t* range, int32_t* count, uint32_t* dk0, uint32_t* dv0, uint32_t* dk1,
                     uint32_t* dv1, uint32_t* hist, uint32_t* bsum, uint32_t* tk, uint32_t* tv, hipStream_t s);

// Stable LSD radix sort of n (key, value) pairs on the low `bits` key bits,
// 8 bits per pass (binning.hip); hist holds 256 * sort_blocks(n) words and
// digit_total 256.  The result is in (k0, v0) when the return value is 0,
// else in (k1, v1).
int launch_radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n, int bits,
                            uint32_t* hist, uint32_t* digit_total, hipStream_t s);

// used: 4 rows (one per band) of ustride = used_slots(capacity, T) 64-bit
// words; the forward sets bit l of slot (start / 64) + tile + k of row q when
// some pixel of band q composited list entry start + 64 k + l of the tile
// (chunks a band never walked keep old bits: the backward reads only
// positions below the band's largest n_last).
inline int64_t used_slots(int64_t cap, int T) { return cap / 64 + T + 2; }
void launch_composite_fwd(const JobDev* jobs, const int32_t* tile_off, int R, int T, const float* rec,
                          const int32_t* items, const int32_t* range, const float* bg, float* rgb, float* depth,
                          float* alpha, float* Tf, int32_t* nl, uint64_t* used, int64_t ustride, hipStream_t s);

// Backward compositing (persistent when a launch has many tiles per resident
// block); queues = kTileQueueBytes of zero-initialised workspace (left zeroed
// by every launch; one launch at a time per workspace).
constexpr size_t kTileQueueBytes = 2 * 9 * 128;

// The plain colour + depth L1 of registration (Sec. 3.2), formed per pixel
// by the pose-only backward itself from the forward's images and the targets
// instead of read from a loss kernel's gradient images: on pixels with a
// target depth, sign(rendered - target) per colour channel and for depth,
// times the render's 1 / |Omega| (up_scale); 0 elsewhere.  Targets in the
// batch's image layout, or NULL: each render's own (JobDev.tgt_*).  With
// loss_part, each tile also writes {sum over its pixels in Omega of the L1
// terms (|D - D*| + sum_c |C_c - C*_c|), number of those pixels}.
struct L1Targets {
  const float* pred_rgb;    // forward colour [3][P]; NULL: off
  const float* pred_depth;  // forward depth [P]
  const float* tgt_rgb;
  const float* tgt_depth;
  float* loss_part;         // [T][2], or NULL
};

// Per-render L1 loss from the tile partials: loss[r] = sum / count over the
// render's tiles in a fixed order (0 when the render has no pixel in Omega).
void launch_tile_loss_reduce(const JobDev* jobs, int R, const float* loss_part, float* loss, hipStream_t s);

// used, ustride: the flags the forward wrote for the same bins: the backward
// walks only the entries some pixel of the band composited.
void launch_composite_bwd(const JobDev* jobs, const int32_t* tile_off, int R, int T, const float* rec,
                          const float* aux, const float* pose, const int32_t* items, const int32_t* range,
                          const uint64_t* used, int64_t ustride, const float* bg, const float* Tf, const int32_t* nl,
                          const float* up_rgb,
                          const float* up_depth, const float* up_alpha, const float* up_scale, float* g2d,
                          float* tile_part, int pose_only, void* queues, hipStream_t s,
                          const L1Targets* l1 = nullptr);

// Registration helpers (reg_kernels.hip).
struct ViewOpt {
  float lr_rot, lr_trans;
  int32_t step;    // Adam steps taken so far
  int32_t active;  // 0: frozen (no update)
  float best;      // lowest loss seen (early exit)
  int32_t stall;   // iterations since the loss last improved on best by more than the tolerance
  float resid;     // loss at the pose the view froze at
  int32_t pad;
};
// Adam on one render's 7 pose values (lr_rot for q, lr_trans for t) from its
// gradient g, and on its 2 exposure coefficients when given (lr_expo), bias
// correction from the render's own step count; the gradients are consumed
// (zeroed).  Early exit (exit_patience > 0) freezes a view at its current
// pose (whose loss is the one just computed) instead of stepping once, for
// exit_patience iterations in a row,
//   exit_mode 0: its loss has not improved on its best by more than exit_tol
//                (relative);
//   exit_mode 1: its Adam step would have been small: the largest
//                |m_hat| / (sqrt(v_hat) + eps) over its 7 pose values (the
//                step in units of the learning rate) is below exit_tol.
// Frozen views keep their pose.
struct PoseAdamArgs {
  float* pose;
  float* grad;  // [R][7], zeroed here
  float* m;
  float* v;
  ViewOpt* opt;
  const float* loss;
  float beta1, beta2, eps, exit_tol;
  int exit_patience, exit_mode;
  float* expo;  // exposure coefficients (a, b) per render, or NULL
  float* egrad;
  float* em;
  float* ev;
  float lr_expo;
};

__device__ inline void pose_adam_view(const PoseAdamArgs& a, int r, const float (&g)[7]) {
  ViewOpt o = a.opt[r];
  if (o.active) {
    const int step = o.step + 1;
    const float bc1 = 1.f / (1.f - __powf(a.beta1, (float)step));
    const float bc2 = 1.f / (1.f - __powf(a.beta2, (float)step));
    float mn[7], vn[7], ratio = 0.f;
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      const int i = 7 * r + k;
      mn[k] = a.beta1 * a.m[i] + (1.f - a.beta1) * g[k];
      vn[k] = a.beta2 * a.v[i] + (1.f - a.beta2) * g[k] * g[k];
      ratio = fmaxf(ratio, fabsf(mn[k] * bc1) / (sqrtf(vn[k] * bc2) + a.eps));
    }
    bool step_now = true;
    if (a.exit_patience > 0) {
      const float l = a.loss[r];
      if (a.exit_mode == 1) {
        o.stall = ratio < a.exit_tol ? o.stall + 1 : 0;
        o.best = o.step == 0 ? l : fminf(o.best, l);
      } else if (o.step == 0 || l < o.best * (1.f - a.exit_tol)) {
        o.best = o.step == 0 ? l : fminf(o.best, l);
        o.stall = 0;
      } else {
        o.best = fminf(o.best, l);
        ++o.stall;
      }
      if (o.stall >= a.exit_patience) {
        o.active = 0;
        o.resid = l;
        step_now = false;
      }
    }
    if (step_now) {
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        const int i = 7 * r + k;
        a.m[i] = mn[k];
        a.v[i] = vn[k];
        const float lr = k < 4 ? o.lr_rot : o.lr_trans;
        a.pose[i] -= lr * (mn[k] * bc1) / (sqrtf(vn[k] * bc2) + a.eps);
      }
      if (a.expo) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int i = 2 * r + k;
          const float eg = a.egrad[i];
          const float mi = a.beta1 * a.em[i] + (1.f - a.beta1) * eg;
          const float vi = a.beta2 * a.ev[i] + (1.f - a.beta2) * eg * eg;
          a.em[i] = mi;
          a.ev[i] = vi;
          a.expo[i] -= a.lr_expo * (mi * bc1) / (sqrtf(vi * bc2) + a.eps);
        }
      }
      o.step = step;
    }
    a.opt[r] = o;
  }
#pragma unroll
  for (int k = 0; k < 7; ++k) a.grad[7 * r + k] = 0.f;
  if (a.expo) {
    a.egrad[2 * r] = 0.f;
    a.egrad[2 * r + 1] = 0.f;
  }
}

// sticky[0] |= overflow; sticky[1] keeps the instance count required at the
// first overflow (the pose before any step taken on truncated lists).
__device__ inline void or_flag(const int32_t* count, int32_t* sticky) {
  if (count[1] != 0) {
    if (sticky[0] == 0) sticky[1] = count[2];
    sticky[0] = 1;
  }
}

// Joint registration on the device (one T = T_{P->Q} per pair shared by its
// views, optimised by Adam in double precision).  Per view: its keyframe's
// rotation, translation and unit quaternion, the pair and whether it is a
// keyframe of Q; per pair: T (unnormalised quaternion, translation), its
// moments and its views [first, first + count).
struct JointView {
  double Rc[9], tc[3], qc[4];
  int32_t pair, reverse;
};
struct JointPair {
  double T[7], m[7], v[7];
  int32_t first, count;
};
struct JointAdam {
  double lr_rot, lr_trans, beta1, beta2, eps, bc1, bc2;  // bc = 1 / (1 - beta^step)
};
// pose[r] = the camera-frame correction Delta of view r under its pair's T:
// C^-1 T^-1 C for a keyframe of P, C^-1 T C for one of Q.
void launch_joint_poses(const JointView* views, int R, const JointPair* pairs, float* pose, hipStream_t s);
// One Adam step of every pair's T from its views' pose gradients (chained
// through the Jacobian of T -> Delta by central differences of that smooth
// map in double precision), then the views' new corrections; the pose
// gradients are cleared.
void launch_joint_step(const JointView* views, JointPair* pairs, int npairs, float* pose_grad, float* pose,
                       const JointAdam& a, hipStream_t s);

// One iteration's end in pose-only registration: per render, the tile
// partials reduced to its pose gradient (as launch_pose_reduce_tiles) and
// its Adam step (pose_adam_view) in one launch; render 0 also updates the
// sticky overflow flag from count (as launch_or_flag).
void launch_pose_reduce_adam(const JobDev* jobs, int R, const float* tile_part, const PoseAdamArgs& a,
                             const int32_t* count, int32_t* sticky, hipStream_t s);
void launch_pose_init(float* pose, float* m, float* v, ViewOpt* opt, int R, hipStream_t s);
void launch_or_flag(const int32_t* count, int32_t* sticky, hipStream_t s);
// Per render: fraction of the pixels with a target depth > 0 whose rendered
// alpha is >= 0.5 (part: 2 floats per 1024-pixel block).
void launch_view_coverage(const JobDev* jobs, const int32_t* pblk_off, int R, int npblk, const float* alpha,
                          const float* tgt_depth, float* part, float* coverage, hipStream_t s);
// Per-view exposure coefficients (a, b) [R][2] with their Adam moments and
// gradient, or all null.
struct ExpoState {
  float *expo, *m, *v, *grad;
};
void launch_state_remap(const float* opose, const float* om, const float* ov, const ViewOpt* oopt, float* npose,
                        float* nm, float* nv, float* ngrad, ViewOpt* nopt, const int32_t* map, const ViewOpt* init_opt,
                        int R, hipStream_t s, ExpoState oe = {}, ExpoState ne = {});
void launch_all_finite(const float* a, int64_t n, int32_t* bad, hipStream_t s);

void launch_render_stats(const JobDev* jobs, const int32_t* tile_off, int R, int T, const float* rec,
                         const int32_t* items, const int32_t* range, const int32_t* nl, int64_t* stats, hipStream_t s);

// The loss launchers take optional exposure coefficients (expo [R][2], the
// colour residual then taken on exp(a) C + b) with their block partials
// (epart, 2 floats per 1024-pixel block) and gradients (egrad [R][2]).
void launch_loss_l1(const JobDev* jobs, const int32_t* pblk_off_d, int R, int npblk, const float* pred_rgb,
                    const float* pred_depth, const float* tgt_rgb, const float* tgt_depth, float* g_rgb,
                    float* g_depth, float* part, float* loss, float* scale, hipStream_t s,
                    const float* expo = nullptr, float* epart = nullptr, float* egrad = nullptr);
// Tracking loss with masks; sel = per-render selection workspace
// (kSelWords(R) uint32, zero on first use, left zeroed after each call).
void launch_loss_track(const JobDev* jobs, const int32_t* pblk_off_d, int R, int npblk, const float* pred_rgb,
                       const float* pred_depth, const float* pred_alpha, const float* tgt_rgb, const float* tgt_depth,
                       float lambda_c, float inlier_k, int alpha_power, uint32_t* sel, float* median, float* g_rgb,
                       float* g_depth, float* part, float* loss, float* scale, hipStream_t s,
                       const float* expo = nullptr, float* epart = nullptr, float* egrad = nullptr);
inline int64_t sel_words(int R) { return (int64_t)R * (4 + 2048); }

// Mapping loss (mapping_loss.hip).  SSIM blocks of a W x H render (3 colour
// channels x 32 x 32 tiles); cnt_part: one float per 1024-pixel block;
// map_part: 3 floats per SSIM block + R.
int ssim_blocks(int W, int H);
void launch_loss_mapping(const JobDev* jobs, const int32_t* pblk_off_d, int npblk, const int32_t* sblk_off_d,
                         int nsblk, int R, const float* pred_rgb, const float* pred_depth, const float* tgt_rgb,
                         const float* tgt_depth, float lambda_ssim, float lambda_color, float lambda_depth,
                         float* g_rgb, float* g_depth, float* cnt_part, float* map_part, float* loss, float* scale,
                         hipStream_t s);
// Per render 1 / |Omega| (pixels with a target depth; 0 when none) into inv
// [R]; cnt_part = npblk floats.  Targets as for L1Targets.
void launch_valid_inv(const JobDev* jobs, const int32_t* pblk_off_d, int npblk, int R, const float* tgt_depth,
                      float* cnt_part, float* inv, hipStream_t s);
// Isotropic regulariser; part = kIsotropicBlocks floats.
constexpr int kIsotropicBlocks = LS_ISOTROPIC_WORK_FLOATS;
void launch_loss_isotropic(const float* log_scale, int64_t n, float lambda_reg, float* loss, float* grad, float* part,
                           hipStream_t s);

// Map adjustment (adjust.hip): validated descriptors, any count.
int launch_adjust_submaps(const ls_submap_adjust* subs, int count, hipStream_t s);

// Opacity pruning (prune.hip): up to kPruneArrays SoA arrays [comp][n]
// compacted to [comp][count] by the keep test logit >= tau.
constexpr int kPruneArrays = 16;
struct PruneArrays {
  const float* src[kPruneArrays];
  float* dst[kPruneArrays];
  int comp[kPruneArrays];
  int count;
};
size_t prune_workspace_bytes(int n);
void launch_prune(const float* logit, int n, float tau, const PruneArrays& arr, int32_t* kept, int32_t* count,
                  void* work, hipStream_t s);

// Overlap ratio (overlap.hip).
ls_status overlap_check_args(const float* p_mean, int32_t np, const float* q_mean, int32_t nq, const float* T_pq,
                             float tau, const int32_t* nn_pq, const int32_t* nn_qp, const int32_t* counts);
size_t overlap_workspace_bytes(int np, int nq);
void launch_overlap(const float* p_mean, int np, const float* q_mean, int nq, const float* T, float tau,
                    int32_t* nn_pq, int32_t* nn_qp, int32_t* counts, void* work, hipStream_t s);

void launch_adam(const ls_adam_group* g, int ng, float beta1, float beta2, float eps, float bc1, float bc2,
                 int zero_grad, hipStream_t s);

}  // namespace ls

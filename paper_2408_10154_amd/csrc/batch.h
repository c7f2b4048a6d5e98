// Internal definition of the opaque ls_batch (shared by the C ABI, the
// registration engine and the server).
#pragma once

#include <vector>

#include "kernels.h"

struct ls_batch {
  using JobDev = ls::JobDev;
  using GradDev = ls::GradDev;
  int R = 0;
  int64_t M = 0;
  int T = 0;
  int64_t P = 0;
  int nblk_items = 0;
  int nblk_pix = 0;
  int nblk_ssim = 0;  // mapping-loss SSIM blocks (3 channels x 32x32 tiles per render)
  int tile_bits = 0;  // bits of the largest tile key
  int device = 0;
  std::vector<JobDev> jobs_h;
  std::vector<int64_t> item_off, pix_off;
  std::vector<int32_t> tile_off, blk_off, pblk_off, sblk_off;
  JobDev* jobs_d = nullptr;
  int64_t* item_off_d = nullptr;
  int32_t* tile_off_d = nullptr;
  int32_t* blk_off_d = nullptr;
  int32_t* pblk_off_d = nullptr;
  int32_t* sblk_off_d = nullptr;
  float* loss_part_d = nullptr;
  float* map_part_d = nullptr;   // mapping loss: 3 floats per SSIM block, then 1/|Omega| per render
  uint32_t* sel_d = nullptr;     // median selection workspace (ls::sel_words(R)), kept zeroed
  float* median_d = nullptr;     // [R] median depth error of the last tracking loss
  GradDev* grads_d = nullptr;
  std::vector<GradDev> grads_cached;
  char* dev_base = nullptr;  // one region holding every device table above
  bool external = false;     // the region belongs to the caller (not freed with the batch)
};

namespace ls {
// A batch whose device tables are carved from `mem` (mem_bytes >= its
// batch_tables_bytes, 256-byte aligned; the caller keeps it until
// ls_batch_destroy) with the uploads queued on s, or allocated by the batch
// when mem is NULL (then s may be NULL and the call synchronises).
ls_status batch_create(const ls_render_job* jobs, int32_t R, void* mem, size_t mem_bytes, hipStream_t s,
                       ls_batch** out);
// The same in two steps: the host tables (no device work; sizes and
// ls_batch_query are available), then the device tables.
ls_status batch_create_host(const ls_render_job* jobs, int32_t R, ls_batch** out);
size_t batch_tables_bytes(const ls_batch* b);
ls_status batch_bind(ls_batch* b, void* mem, size_t mem_bytes, hipStream_t s);
// ls_project with every render gated on live[r].active (live NULL: all): a
// frozen registration view contributes no tile instances, so binning,
// compositing and the backward skip it.
ls_status project_views(const ls_batch* b, const float* pose, const ls_projected* out, const ViewOpt* live,
                        hipStream_t s);
// After a pose-only backward: each render's pose gradient from the tile
// partials and its Adam step (a.grad is added to and consumed), and the
// sticky overflow flag updated from count (launch_pose_reduce_adam).
ls_status pose_reduce_adam(const ls_batch* b, const ls_bins* bins, const PoseAdamArgs& a, const int32_t* count,
                           int32_t* sticky, hipStream_t s);
// Per render 1 / |Omega| (pixels with a target depth) into inv [R]; targets in
// the image layout, or NULL: each render's own.  Equals the grad_scale the L1
// loss kernels write.
ls_status batch_valid_inv(const ls_batch* b, const float* tgt_depth, float* inv, hipStream_t s);
// Pose-only ls_render_bwd_tiles whose per-pixel upstream gradient is the
// plain colour + depth L1 of the forward images against the targets (image
// layout, or NULL: each render's own), scaled by scale [R] (batch_valid_inv):
// the same gradient as the L1 loss kernel's, with no loss kernel and no
// gradient images.
ls_status render_bwd_pose_l1(const ls_batch* b, const float* pose, const ls_projected* p, const ls_bins* bins,
                             const ls_image* fwd, const float* tgt_rgb, const float* tgt_depth, const float* scale,
                             hipStream_t s);
// Points every render's loss at its own measurements (device [3][H][W] and
// [H][W]); re-uploads the job table.  Used by engines that do not lay the
// targets out contiguously.
ls_status batch_set_targets(ls_batch* b, const std::vector<const float*>& rgb, const std::vector<const float*>& depth);
// Loss over per-render targets (see batch_set_targets).
ls_status batch_loss_l1(const ls_batch* b, const ls_image* pred, float* loss, float* grad_rgb, float* grad_depth,
                        float* grad_scale, hipStream_t s);
ls_status batch_loss_tracking(const ls_batch* b, const ls_image* pred, const ls_loss_params* prm, float* loss,
                              float* grad_rgb, float* grad_depth, float* grad_scale, hipStream_t s);
// The registration losses with per-render exposure coefficients expo [R][2]
// (colour residual on exp(a) C + b): kind 0 plain L1, 1 tracking loss.  egrad
// [R][2] (or NULL) receives dL/d(a, b); epart holds 2 floats per 1024-pixel
// block.  Targets laid out like the batch's images.
ls_status batch_loss_exposure(const ls_batch* b, int kind, const ls_loss_params* prm, const ls_image* pred,
                              const float* tgt_rgb, const float* tgt_depth, const float* expo, float* epart,
                              float* egrad, float* loss, float* grad_rgb, float* grad_depth, float* grad_scale,
                              hipStream_t s);
}  // namespace ls

// C ABI of libloopsplat.so: argument checking, batch tables, workspace
// layout and kernel sequencing.  See include/loopsplat.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "batch.h"
#include "kernels.h"

using namespace ls;

namespace {

thread_local std::string g_err;

ls_status fail(ls_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
ls_status fail(ls_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

ls_status hip_check(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  return LS_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace



namespace ls {

ls_status api_fail(ls_status st, const char* msg) { return fail(st, "%s", msg); }

ls_status api_hip_check(const char* what) { return hip_check(what); }

ls_status overlap_check_args(const float* p_mean, int32_t np, const float* q_mean, int32_t nq, const float* T_pq,
                             float tau, const int32_t* nn_pq, const int32_t* nn_qp, const int32_t* counts) {
  if (np < 0 || nq < 0) return fail(LS_ERR_INVALID, "negative point count");
  if (!T_pq || !counts || (np > 0 && (!p_mean || !nn_pq)) || (nq > 0 && (!q_mean || !nn_qp)))
    return fail(LS_ERR_INVALID, "NULL arguments");
  for (int k = 0; k < 12; ++k)
    if (!std::isfinite(T_pq[k])) return fail(LS_ERR_INVALID, "non-finite transform");
  if (!(tau > 0.f) || !std::isfinite(tau)) return fail(LS_ERR_INVALID, "tau must be finite and > 0");
  return LS_OK;
}

}  // namespace ls

namespace {

struct Layout {
  size_t dk0, dv0, dk1, dv1, hist, bsum, tk, tv, g2d, tile_part, pose_part, loss_part, used, queues, total;
};

Layout layout_of(const ls_batch* b, int64_t cap) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + std::max<size_t>(bytes, 4));
    return o;
  };
  const int64_t M = b->M;
  const int64_t nbd = sort_blocks(M);
  const int64_t nbt = sort_blocks(cap);
  L.dk0 = take(4 * M);
  L.dv0 = take(4 * M);
  L.dk1 = take(4 * M);
  L.dv1 = take(4 * M);
  // digit histograms; after the depth sort, the first tile pass's histogram
  // followed by the first item of each emission span
  L.hist = take(4 * std::max<int64_t>({(int64_t)(1 << kDepthDigitBits) * nbd,
                                        (int64_t)(1 << kTileDigitBits) * nbt + emit_spans(cap), 256}));
  L.bsum = take(4 * (nbd + 8 + kMaxSortBins + 8));  // block sums, then the digit totals
  L.tk = take(4 * cap);
  L.tv = take(4 * cap);
  L.g2d = take(4 * (size_t)kGrad2D * M);
  L.tile_part = take(4 * (size_t)kPoseAcc * std::max(b->T, 1));
  L.pose_part = take(4 * (size_t)kPoseAcc * std::max(b->nblk_items, 1));
  L.loss_part = take(8 * (size_t)std::max(b->T, 1));  // per tile {L1 sum, pixels in Omega}
  L.used = take(8 * 4 * (size_t)used_slots(cap, b->T));  // per band a row of "used" bits, 64 entries a word
  L.queues = take(kTileQueueBytes);
  L.total = off;
  return L;
}

template <typename T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

ls_status ensure_device(const ls_batch* b) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(LS_ERR_HIP, "hipGetDevice failed");
  if (cur != b->device && hipSetDevice(b->device) != hipSuccess) return fail(LS_ERR_HIP, "hipSetDevice failed");
  return LS_OK;
}

ls_status check_projected(const ls_projected* p, bool need_aux = false) {
  if (!p || !p->rec || !p->radius || !p->tiles) return fail(LS_ERR_INVALID, "ls_projected has NULL members");
  if (reinterpret_cast<uintptr_t>(p->rec) % 16) return fail(LS_ERR_INVALID, "ls_projected.rec must be 16-byte aligned");
  if (need_aux && !p->aux) return fail(LS_ERR_INVALID, "ls_projected.aux is needed by the backward");
  if (p->aux && reinterpret_cast<uintptr_t>(p->aux) % 16)
    return fail(LS_ERR_INVALID, "ls_projected.aux must be 16-byte aligned");
  return LS_OK;
}

ls_status check_bins(const ls_batch* b, const ls_bins* bins) {
  if (!bins || !bins->tile_of || !bins->item || !bins->range || !bins->count || !bins->work)
    return fail(LS_ERR_INVALID, "ls_bins has NULL members");
  if (bins->capacity < 0 || bins->capacity > INT32_MAX)
    return fail(LS_ERR_INVALID, "ls_bins.capacity out of range: %lld", (long long)bins->capacity);
  if (reinterpret_cast<uintptr_t>(bins->work) % 256) return fail(LS_ERR_INVALID, "ls_bins.work must be 256-byte aligned");
  (void)b;
  return LS_OK;
}

}  // namespace

namespace ls {
ls_status batch_set_targets(ls_batch* b, const std::vector<const float*>& rgb, const std::vector<const float*>& depth) {
  if (!b || (int)rgb.size() != b->R || (int)depth.size() != b->R) return fail(LS_ERR_INVALID, "one target per render");
  for (int r = 0; r < b->R; ++r) {
    b->jobs_h[r].tgt_rgb = rgb[r];
    b->jobs_h[r].tgt_depth = depth[r];
  }
  if (hipMemcpy(b->jobs_d, b->jobs_h.data(), sizeof(JobDev) * b->R, hipMemcpyHostToDevice) != hipSuccess)
    return fail(LS_ERR_HIP, "job table upload failed");
  return LS_OK;
}

ls_status batch_loss_l1(const ls_batch* b, const ls_image* pred, float* loss, float* grad_rgb, float* grad_depth,
                        float* grad_scale, hipStream_t s) {
  launch_loss_l1(b->jobs_d, b->pblk_off_d, b->R, b->nblk_pix, pred->rgb, pred->depth, nullptr, nullptr, grad_rgb,
                 grad_depth, b->loss_part_d, loss, grad_scale, s);
  return hip_check("loss over per-render targets");
}

ls_status check_loss_params(const ls_loss_params* prm, const ls_image* pred) {
  if (!prm) return fail(LS_ERR_INVALID, "NULL ls_loss_params");
  if (!(prm->lambda_c >= 0.f && prm->lambda_c <= 1.f)) return fail(LS_ERR_INVALID, "lambda_c must lie in [0, 1]");
  if (!std::isfinite(prm->inlier_k)) return fail(LS_ERR_INVALID, "inlier_k must be finite");
  if (prm->alpha_power < 0 || prm->alpha_power > 8) return fail(LS_ERR_INVALID, "alpha_power must lie in 0..8");
  if (prm->alpha_power > 0 && !pred->alpha) return fail(LS_ERR_INVALID, "the alpha mask needs ls_image.alpha");
  return LS_OK;
}

ls_status batch_loss_exposure(const ls_batch* b, int kind, const ls_loss_params* prm, const ls_image* pred,
                              const float* tgt_rgb, const float* tgt_depth, const float* expo, float* epart,
                              float* egrad, float* loss, float* grad_rgb, float* grad_depth, float* grad_scale,
                              hipStream_t s) {
  if (kind == 1)
    launch_loss_track(b->jobs_d, b->pblk_off_d, b->R, b->nblk_pix, pred->rgb, pred->depth, pred->alpha, tgt_rgb,
                      tgt_depth, prm->lambda_c, prm->inlier_k, prm->alpha_power, b->sel_d, b->median_d, grad_rgb,
                      grad_depth, b->loss_part_d, loss, grad_scale, s, expo, epart, egrad);
  else
    launch_loss_l1(b->jobs_d, b->pblk_off_d, b->R, b->nblk_pix, pred->rgb, pred->depth, tgt_rgb, tgt_depth, grad_rgb,
                   grad_depth, b->loss_part_d, loss, grad_scale, s, expo, epart, egrad);
  return hipGetLastError() == hipSuccess ? LS_OK : LS_ERR_HIP;
}

ls_status batch_loss_tracking(const ls_batch* b, const ls_image* pred, const ls_loss_params* prm, float* loss,
                              float* grad_rgb, float* grad_depth, float* grad_scale, hipStream_t s) {
  launch_loss_track(b->jobs_d, b->pblk_off_d, b->R, b->nblk_pix, pred->rgb, pred->depth, pred->alpha, nullptr, nullptr,
                    prm->lambda_c, prm->inlier_k, prm->alpha_power, b->sel_d, b->median_d, grad_rgb, grad_depth,
                    b->loss_part_d, loss, grad_scale, s);
  return hip_check("tracking loss over per-render targets");
}

// Device tables of a batch, in the order they are carved from one region.
struct BatchTables {
  size_t jobs, item_off, tile_off, blk_off, pblk_off, sblk_off, loss_part, map_part, grads, sel, median, total;
};

static BatchTables batch_tables(const ls_batch* b) {
  BatchTables t{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + std::max<size_t>(bytes, 16));
    return o;
  };
  const size_t R1 = (size_t)b->R + 1;
  t.jobs = take(sizeof(JobDev) * b->R);
  t.item_off = take(8 * R1);
  t.tile_off = take(4 * R1);
  t.blk_off = take(4 * R1);
  t.pblk_off = take(4 * R1);
  t.sblk_off = take(4 * R1);
  t.loss_part = take(8 * (size_t)std::max(b->nblk_pix, 1));
  t.map_part = take(4 * (3 * (size_t)b->nblk_ssim + b->R));
  t.grads = take(sizeof(GradDev) * b->R);
  t.sel = take(4 * (size_t)ls::sel_words(b->R));
  t.median = take(4 * (size_t)b->R);
  t.total = off;
  return t;
}

// Host tables of a batch (offsets, job records); no device work.
static ls_status batch_host(const ls_render_job* jobs, int32_t R, ls_batch** out) {
  *out = nullptr;
  if (!jobs || R < 1) return fail(LS_ERR_INVALID, "need R >= 1 jobs (R = %d)", R);
  auto* b = new ls_batch();
  b->R = R;
  b->item_off.assign(R + 1, 0);
  b->pix_off.assign(R + 1, 0);
  b->tile_off.assign(R + 1, 0);
  b->blk_off.assign(R + 1, 0);
  b->pblk_off.assign(R + 1, 0);
  b->sblk_off.assign(R + 1, 0);
  b->jobs_h.resize(R);
  for (int r = 0; r < R; ++r) {
    const ls_render_job& j = jobs[r];
    const ls_intrinsics& K = j.K;
    if (j.g.n < 0 || K.width <= 0 || K.height <= 0 || !(K.fx > 0.f) || !(K.fy > 0.f) || !std::isfinite(K.cx) ||
        !std::isfinite(K.cy)) {
      delete b;
      return fail(LS_ERR_INVALID, "job %d: bad sizes or intrinsics", r);
    }
    if (j.g.n > 0 && (!j.g.mean || !j.g.log_scale || !j.g.quat || !j.g.opacity_logit || !j.g.rgb)) {
      delete b;
      return fail(LS_ERR_INVALID, "job %d: NULL Gaussian array", r);
    }
    for (int k = 0; k < 12; ++k)
      if (!std::isfinite(j.w2c[k])) {
        delete b;
        return fail(LS_ERR_NONFINITE, "job %d: non-finite w2c", r);
      }
    const int TX = (K.width + kTile - 1) / kTile, TY = (K.height + kTile - 1) / kTile;
    JobDev& d = b->jobs_h[r];
    d.mean = j.g.mean;
    d.log_scale = j.g.log_scale;
    d.quat = j.g.quat;
    d.opac = j.g.opacity_logit;
    d.rgb = j.g.rgb;
    d.fx = K.fx;
    d.fy = K.fy;
    d.cx = K.cx;
    d.cy = K.cy;
    d.n = j.g.n;
    d.W = K.width;
    d.H = K.height;
    d.TX = TX;
    d.TY = TY;
    d.tile_off = b->tile_off[r];
    d.blk_off = b->blk_off[r];
    d.item_off = b->item_off[r];
    d.pix_off = b->pix_off[r];
    std::memcpy(d.w2c, j.w2c, sizeof(d.w2c));
    d.tgt_rgb = nullptr;
    d.tgt_depth = nullptr;
    const int64_t hw = (int64_t)K.width * K.height;
    b->item_off[r + 1] = b->item_off[r] + j.g.n;
    b->pix_off[r + 1] = b->pix_off[r] + hw;
    b->tile_off[r + 1] = b->tile_off[r] + TX * TY;
    b->blk_off[r + 1] = b->blk_off[r] + (j.g.n + 255) / 256;
    b->pblk_off[r + 1] = b->pblk_off[r] + (int32_t)((hw + 1023) / 1024);
    b->sblk_off[r + 1] = b->sblk_off[r] + ls::ssim_blocks(K.width, K.height);
    if (b->item_off[r + 1] > INT32_MAX || b->tile_off[r + 1] < 0) {
      delete b;
      return fail(LS_ERR_INVALID, "batch too large (items or tiles exceed int32)");
    }
  }
  b->M = b->item_off[R];
  b->P = b->pix_off[R];
  b->T = b->tile_off[R];
  b->nblk_items = b->blk_off[R];
  b->nblk_pix = b->pblk_off[R];
  b->nblk_ssim = b->sblk_off[R];
  int bits = 0;
  while (bits < 32 && ((int64_t)1 << bits) < (int64_t)b->T) ++bits;
  b->tile_bits = bits;
  *out = b;
  return LS_OK;
}

ls_status batch_create_host(const ls_render_job* jobs, int32_t R, ls_batch** out) {
  if (!out) return fail(LS_ERR_INVALID, "out is NULL");
  return batch_host(jobs, R, out);
}

size_t batch_tables_bytes(const ls_batch* b) { return batch_tables(b).total; }

ls_status batch_bind(ls_batch* b, void* mem, size_t mem_bytes, hipStream_t s) {
  if (hipGetDevice(&b->device) != hipSuccess) return fail(LS_ERR_HIP, "hipGetDevice failed");
  const BatchTables t = batch_tables(b);
  char* base = nullptr;
  if (mem) {
    if (mem_bytes < t.total || reinterpret_cast<uintptr_t>(mem) % 256)
      return fail(LS_ERR_CAPACITY, "batch tables need %zu bytes at 256-byte alignment", t.total);
    base = static_cast<char*>(mem);
    b->external = true;
  } else {
    void* p = nullptr;
    if (hipMalloc(&p, t.total) != hipSuccess) return fail(LS_ERR_HIP, "hipMalloc of the batch tables failed");
    base = static_cast<char*>(p);
  }
  const int R = b->R;
  b->dev_base = base;
  b->jobs_d = reinterpret_cast<JobDev*>(base + t.jobs);
  b->item_off_d = reinterpret_cast<int64_t*>(base + t.item_off);
  b->tile_off_d = reinterpret_cast<int32_t*>(base + t.tile_off);
  b->blk_off_d = reinterpret_cast<int32_t*>(base + t.blk_off);
  b->pblk_off_d = reinterpret_cast<int32_t*>(base + t.pblk_off);
  b->sblk_off_d = reinterpret_cast<int32_t*>(base + t.sblk_off);
  b->loss_part_d = reinterpret_cast<float*>(base + t.loss_part);
  b->map_part_d = reinterpret_cast<float*>(base + t.map_part);
  b->grads_d = reinterpret_cast<GradDev*>(base + t.grads);
  b->sel_d = reinterpret_cast<uint32_t*>(base + t.sel);
  b->median_d = reinterpret_cast<float*>(base + t.median);
  // the host vectors live as long as the batch, so the copies may stay queued on s
  const bool ok =
      hipMemcpyAsync(b->jobs_d, b->jobs_h.data(), sizeof(JobDev) * R, hipMemcpyHostToDevice, s) == hipSuccess &&
      hipMemcpyAsync(b->item_off_d, b->item_off.data(), 8 * (R + 1), hipMemcpyHostToDevice, s) == hipSuccess &&
      hipMemcpyAsync(b->tile_off_d, b->tile_off.data(), 4 * (R + 1), hipMemcpyHostToDevice, s) == hipSuccess &&
      hipMemcpyAsync(b->blk_off_d, b->blk_off.data(), 4 * (R + 1), hipMemcpyHostToDevice, s) == hipSuccess &&
      hipMemcpyAsync(b->pblk_off_d, b->pblk_off.data(), 4 * (R + 1), hipMemcpyHostToDevice, s) == hipSuccess &&
      hipMemcpyAsync(b->sblk_off_d, b->sblk_off.data(), 4 * (R + 1), hipMemcpyHostToDevice, s) == hipSuccess &&
      hipMemsetAsync(b->sel_d, 0, 4 * (size_t)ls::sel_words(R), s) == hipSuccess &&
      hipMemsetAsync(b->median_d, 0, 4 * (size_t)R, s) == hipSuccess;
  if (!ok || (!mem && hipStreamSynchronize(s) != hipSuccess))
    return fail(LS_ERR_HIP, "upload of the batch tables failed");
  return LS_OK;
}

ls_status batch_create(const ls_render_job* jobs, int32_t R, void* mem, size_t mem_bytes, hipStream_t s,
                       ls_batch** out) {
  ls_batch* b = nullptr;
  ls_status st = batch_create_host(jobs, R, &b);
  if (st) return st;
  if ((st = batch_bind(b, mem, mem_bytes, s))) {
    ls_batch_destroy(b);
    return st;
  }
  *out = b;
  return LS_OK;
}

ls_status batch_valid_inv(const ls_batch* b, const float* tgt_depth, float* inv, hipStream_t s) {
  if (!b || !inv) return fail(LS_ERR_INVALID, "NULL batch or output");
  ls_status st;
  if ((st = ensure_device(b))) return st;
  launch_valid_inv(b->jobs_d, b->pblk_off_d, b->nblk_pix, b->R, tgt_depth, b->loss_part_d, inv, s);
  return hip_check("1 / |Omega| per render");
}

ls_status render_bwd_pose_l1(const ls_batch* b, const float* pose, const ls_projected* p, const ls_bins* bins,
                             const ls_image* fwd, const float* tgt_rgb, const float* tgt_depth, const float* scale,
                             hipStream_t s) {
  if (!b) return fail(LS_ERR_INVALID, "NULL batch");
  ls_status st;
  if ((st = check_projected(p, true)) || (st = check_bins(b, bins)) || (st = ensure_device(b))) return st;
  if (!fwd || !fwd->T_final || !fwd->n_last || !fwd->rgb || !fwd->depth || !scale)
    return fail(LS_ERR_INVALID, "forward images or 1 / |Omega| missing");
  const Layout L = layout_of(b, bins->capacity);
  const float zero[3] = {0.f, 0.f, 0.f};
  const L1Targets l1{fwd->rgb, fwd->depth, tgt_rgb, tgt_depth, nullptr};
  launch_composite_bwd(b->jobs_d, b->tile_off_d, b->R, b->T, p->rec, p->aux, pose, bins->item, bins->range,
                       at<uint64_t>(bins->work, L.used), used_slots(bins->capacity, b->T), zero,
                       fwd->T_final, fwd->n_last, nullptr, nullptr, nullptr, scale, at<float>(bins->work, L.g2d),
                       at<float>(bins->work, L.tile_part), 1, at<char>(bins->work, L.queues), s, &l1);
  return hip_check("pose-only backward with the L1 gradient");
}

ls_status pose_reduce_adam(const ls_batch* b, const ls_bins* bins, const PoseAdamArgs& a, const int32_t* count,
                           int32_t* sticky, hipStream_t s) {
  if (!b) return fail(LS_ERR_INVALID, "NULL batch");
  ls_status st;
  if ((st = check_bins(b, bins)) || (st = ensure_device(b))) return st;
  const Layout L = layout_of(b, bins->capacity);
  launch_pose_reduce_adam(b->jobs_d, b->R, at<float>(bins->work, L.tile_part), a, count, sticky, s);
  return hip_check("pose reduction and Adam step");
}

ls_status project_views(const ls_batch* b, const float* pose, const ls_projected* out, const ViewOpt* live,
                        hipStream_t s) {
  if (!b) return fail(LS_ERR_INVALID, "NULL batch");
  ls_status st;
  if ((st = check_projected(out)) || (st = ensure_device(b))) return st;
  launch_project(b->jobs_d, b->blk_off_d, b->R, b->nblk_items, pose, out->rec, out->radius, out->tiles, out->aux, live,
                 s);
  return hip_check("ls_project");
}
}  // namespace ls

extern "C" {

const char* ls_last_error(void) { return g_err.c_str(); }

int32_t ls_version(void) { return 100; }

int64_t ls_struct_size(const char* name) {
  if (!name) return -1;
  struct Entry { const char* n; size_t s; };
  static const Entry table[] = {
      {"ls_gaussians", sizeof(ls_gaussians)},       {"ls_intrinsics", sizeof(ls_intrinsics)},
      {"ls_render_job", sizeof(ls_render_job)},     {"ls_batch_info", sizeof(ls_batch_info)},
      {"ls_projected", sizeof(ls_projected)},       {"ls_bins", sizeof(ls_bins)},
      {"ls_image", sizeof(ls_image)},               {"ls_image_grad", sizeof(ls_image_grad)},
      {"ls_gaussian_grads", sizeof(ls_gaussian_grads)}, {"ls_adam_group", sizeof(ls_adam_group)},
      {"ls_pair", sizeof(ls_pair)},                 {"ls_reg_params", sizeof(ls_reg_params)},
      {"ls_reg_result", sizeof(ls_reg_result)},     {"ls_server_params", sizeof(ls_server_params)},
      {"ls_server_stats", sizeof(ls_server_stats)}, {"ls_loss_params", sizeof(ls_loss_params)},
      {"ls_mapping_params", sizeof(ls_mapping_params)},
      {"ls_submap_adjust", sizeof(ls_submap_adjust)},
      {"ls_prune_array", sizeof(ls_prune_array)},
      {"ls_adam_array", sizeof(ls_adam_array)},     {"ls_gaussian_adam", sizeof(ls_gaussian_adam)},
      {"ls_pose_adam", sizeof(ls_pose_adam)},
  };
  for (const Entry& e : table)
    if (std::strcmp(e.n, name) == 0) return (int64_t)e.s;
  return -1;
}

ls_status ls_batch_create(const ls_render_job* jobs, int32_t R, ls_batch** out) {
  return ls::batch_create(jobs, R, nullptr, 0, nullptr, out);
}

ls_status ls_batch_destroy(ls_batch* b) {
  if (!b) return LS_OK;
  if (!b->external && b->dev_base) hipFree(b->dev_base);
  delete b;
  return LS_OK;
}

ls_status ls_batch_query(const ls_batch* b, int64_t capacity, ls_batch_info* info) {
  if (!b || !info) return fail(LS_ERR_INVALID, "NULL argument");
  if (capacity < 0 || capacity > INT32_MAX) return fail(LS_ERR_INVALID, "capacity out of range");
  info->renders = b->R;
  info->items = b->M;
  info->tiles = b->T;
  info->pixels = b->P;
  info->workspace_bytes = layout_of(b, capacity).total;
  return LS_OK;
}

ls_status ls_batch_offsets(const ls_batch* b, int64_t* item_off, int64_t* pix_off, int32_t* tile_off) {
  if (!b) return fail(LS_ERR_INVALID, "NULL batch");
  if (item_off) std::copy(b->item_off.begin(), b->item_off.end(), item_off);
  if (pix_off) std::copy(b->pix_off.begin(), b->pix_off.end(), pix_off);
  if (tile_off) std::copy(b->tile_off.begin(), b->tile_off.end(), tile_off);
  return LS_OK;
}

ls_status ls_fill_i32(int32_t* ptr, int64_t count, int32_t value, hipStream_t s) {
  if (count < 0 || (count > 0 && !ptr)) return fail(LS_ERR_INVALID, "bad fill arguments");
  launch_fill_i32(ptr, count, value, s);
  return hip_check("ls_fill_i32");
}

ls_status ls_project(const ls_batch* b, const float* pose, const ls_projected* out, hipStream_t s) {
  return project_views(b, pose, out, nullptr, s);
}

ls_status ls_bin_sort(const ls_batch* b, const ls_projected* p, const ls_bins* bins, hipStream_t s) {
  if (!b) return fail(LS_ERR_INVALID, "NULL batch");
  ls_status st;
  if ((st = check_projected(p)) || (st = check_bins(b, bins)) || (st = ensure_device(b))) return st;
  const Layout L = layout_of(b, bins->capacity);
  void* w = bins->work;
  if (b->M == 0) {
    launch_fill_i32(bins->count, 4, 0, s);
    launch_fill_i32(bins->range, 2 * (int64_t)b->T, 0, s);
    return hip_check("ls_bin_sort");
  }
  launch_bin_sort(b->jobs_d, b->item_off_d, b->R, b->M, b->T, b->tile_bits, p->rec, p->radius, p->tiles,
                  bins->capacity, bins->tile_of, bins->item, bins->range, bins->count, at<uint32_t>(w, L.dk0),
                  at<uint32_t>(w, L.dv0), at<uint32_t>(w, L.dk1), at<uint32_t>(w, L.dv1), at<uint32_t>(w, L.hist),
                  at<uint32_t>(w, L.bsum), at<uint32_t>(w, L.tk), at<uint32_t>(w, L.tv), s);
  return hip_check("ls_bin_sort");
}

ls_status ls_render_fwd(const ls_batch* b, const ls_projected* p, const ls_bins* bins, const float* bg,
                        const ls_image* out, hipStream_t s) {
  if (!b) return fail(LS_ERR_INVALID, "NULL batch");
  ls_status st;
  if ((st = check_projected(p)) || (st = check_bins(b, bins)) || (st = ensure_device(b))) return st;
  if (!out || !out->rgb || !out->depth || !out->alpha || !out->T_final || !out->n_last)
    return fail(LS_ERR_INVALID, "ls_image has NULL members");
  const float zero[3] = {0.f, 0.f, 0.f};
  const Layout L = layout_of(b, bins->capacity);
  launch_composite_fwd(b->jobs_d, b->tile_off_d, b->R, b->T, p->rec, bins->item, bins->range, bg ? bg : zero,
                       out->rgb, out->depth, out->alpha, out->T_final, out->n_last, at<uint64_t>(bins->work, L.used),
                       used_slots(bins->capacity, b->T), s);
  return hip_check("ls_render_fwd");
}

ls_status ls_render_bwd_tiles(const ls_batch* b, const float* pose, const ls_projected* p, const ls_bins* bins,
                              const float* bg, const ls_image* fwd, const ls_image_grad* up, uint32_t flags,
                              hipStream_t s) {
  if (!b) return fail(LS_ERR_INVALID, "NULL batch");
  ls_status st;
  if ((st = check_projected(p, true)) || (st = check_bins(b, bins)) || (st = ensure_device(b))) return st;
  if (!fwd || !fwd->T_final || !fwd->n_last) return fail(LS_ERR_INVALID, "forward state (T_final, n_last) missing");
  if (!up) return fail(LS_ERR_INVALID, "upstream gradients missing");
  const Layout L = layout_of(b, bins->capacity);
  const float zero[3] = {0.f, 0.f, 0.f};
  launch_composite_bwd(b->jobs_d, b->tile_off_d, b->R, b->T, p->rec, p->aux, pose, bins->item, bins->range,
                       at<uint64_t>(bins->work, L.used), used_slots(bins->capacity, b->T),
                       bg ? bg : zero, fwd->T_final, fwd->n_last, up->rgb, up->depth, up->alpha, up->scale,
                       at<float>(bins->work, L.g2d), at<float>(bins->work, L.tile_part),
                       (flags & LS_BWD_POSE_ONLY) ? 1 : 0, at<char>(bins->work, L.queues), s);
  return hip_check("ls_render_bwd_tiles");
}

ls_status ls_render_bwd_tiles_l1(const ls_batch* b, const float* pose, const ls_projected* p, const ls_bins* bins,
                                 const float* bg, const ls_image* fwd, const float* tgt_rgb, const float* tgt_depth,
                                 const float* inv_count, uint32_t flags, hipStream_t s) {
  if (!b) return fail(LS_ERR_INVALID, "NULL batch");
  ls_status st;
  if ((st = check_projected(p, true)) || (st = check_bins(b, bins)) || (st = ensure_device(b))) return st;
  if (!fwd || !fwd->T_final || !fwd->n_last || !fwd->rgb || !fwd->depth)
    return fail(LS_ERR_INVALID, "forward images (rgb, depth, T_final, n_last) missing");
  if (!tgt_rgb || !tgt_depth || !inv_count) return fail(LS_ERR_INVALID, "targets or 1 / |Omega| missing");
  if (flags & ~LS_BWD_POSE_ONLY) return fail(LS_ERR_INVALID, "unknown backward flags");
  const Layout L = layout_of(b, bins->capacity);
  const float zero[3] = {0.f, 0.f, 0.f};
  const L1Targets l1{fwd->rgb, fwd->depth, tgt_rgb, tgt_depth, at<float>(bins->work, L.loss_part)};
  launch_composite_bwd(b->jobs_d, b->tile_off_d, b->R, b->T, p->rec, p->aux, pose, bins->item, bins->range,
                       at<uint64_t>(bins->work, L.used), used_slots(bins->capacity, b->T),
                       bg ? bg : zero, fwd->T_final, fwd->n_last, nullptr, nullptr, nullptr, inv_count,
                       at<float>(bins->work, L.g2d), at<float>(bins->work, L.tile_part),
                       (flags & LS_BWD_POSE_ONLY) ? 1 : 0, at<char>(bins->work, L.queues), s, &l1);
  return hip_check("ls_render_bwd_tiles_l1");
}

ls_status ls_loss_l1_tiles(const ls_batch* b, const ls_bins* bins, float* loss, hipStream_t s) {
  if (!b || !loss) return fail(LS_ERR_INVALID, "NULL batch or loss");
  ls_status st;
  if ((st = check_bins(b, bins)) || (st = ensure_device(b))) return st;
  const Layout L = layout_of(b, bins->capacity);
  launch_tile_loss_reduce(b->jobs_d, b->R, at<float>(bins->work, L.loss_part), loss, s);
  return hip_check("ls_loss_l1_tiles");
}

ls_status ls_render_bwd_project(const ls_batch* b, const float* pose, const ls_projected* p, const ls_bins* bins,
                                const ls_gaussian_grads* grads, float* pose_grad, uint32_t flags, hipStream_t s) {
  if (!b) return fail(LS_ERR_INVALID, "NULL batch");
  ls_status st;
  if ((st = check_projected(p, true)) || (st = check_bins(b, bins)) || (st = ensure_device(b))) return st;
  const Layout L = layout_of(b, bins->capacity);
  if (flags & LS_BWD_POSE_ONLY) {
    if (grads) return fail(LS_ERR_INVALID, "pose-only backward computes no Gaussian gradients");
    if (pose_grad) launch_pose_reduce_tiles(b->jobs_d, b->R, pose, at<float>(bins->work, L.tile_part), pose_grad, s);
    return hip_check("ls_render_bwd_project");
  }
  if (pose_grad && !pose) return fail(LS_ERR_INVALID, "pose_grad needs the pose it is taken at");
  const int want_gauss = grads != nullptr;
  if (want_gauss) {
    std::vector<GradDev> gd(b->R);
    for (int r = 0; r < b->R; ++r) {
      gd[r].mean = grads[r].mean;
      gd[r].log_scale = grads[r].log_scale;
      gd[r].quat = grads[r].quat;
      gd[r].opac = grads[r].opacity_logit;
      gd[r].rgb = grads[r].rgb;
      gd[r].shared = 0;
      gd[r].pad = 0;
    }
    for (int r = 0; r < b->R; ++r)
      for (int q = 0; q < b->R; ++q) {
        if (q == r) continue;
        const float* a[5] = {gd[r].mean, gd[r].log_scale, gd[r].quat, gd[r].opac, gd[r].rgb};
        const float* c[5] = {gd[q].mean, gd[q].log_scale, gd[q].quat, gd[q].opac, gd[q].rgb};
        for (int k = 0; k < 5; ++k)
          if (a[k] && a[k] == c[k]) gd[r].shared = 1;
      }
    const bool same = b->grads_cached.size() == gd.size() &&
                      std::memcmp(b->grads_cached.data(), gd.data(), gd.size() * sizeof(GradDev)) == 0;
    if (!same) {
      if (hipMemcpyAsync(b->grads_d, gd.data(), gd.size() * sizeof(GradDev), hipMemcpyHostToDevice, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return fail(LS_ERR_HIP, "upload of gradient table failed");
      const_cast<ls_batch*>(b)->grads_cached = gd;
    }
  }
  launch_project_bwd(b->jobs_d, b->blk_off_d, b->R, b->nblk_items, pose, p->radius, p->aux,
                     at<float>(bins->work, L.g2d), b->grads_d, want_gauss, at<float>(bins->work, L.pose_part),
                     pose_grad != nullptr, pose_grad, s);
  return hip_check("ls_render_bwd_project");
}

ls_status ls_render_bwd_project_adam(const ls_batch* b, float* pose, const ls_projected* p, const ls_bins* bins,
                                     const ls_gaussian_adam* adam, const ls_pose_adam* pose_adam, int32_t step,
                                     float beta1, float beta2, float eps, float* pose_grad, hipStream_t s) {
  if (!b) return fail(LS_ERR_INVALID, "NULL batch");
  ls_status st;
  if ((st = check_projected(p, true)) || (st = check_bins(b, bins)) || (st = ensure_device(b))) return st;
  if (!adam) return fail(LS_ERR_INVALID, "NULL Adam state");
  if (b->R > LS_ADAM_FUSED_MAX_RENDERS) return fail(LS_ERR_INVALID, "at most %d renders", LS_ADAM_FUSED_MAX_RENDERS);
  if (step < 1) return fail(LS_ERR_INVALID, "Adam step counts from 1");
  if (pose_grad && !pose) return fail(LS_ERR_INVALID, "pose_grad needs the pose it is taken at");
  if (pose_adam && (!pose_grad || !pose_adam->m || !pose_adam->v || !std::isfinite(pose_adam->lr_rot) ||
                    !std::isfinite(pose_adam->lr_trans)))
    return fail(LS_ERR_INVALID, "the pose step needs pose, pose_grad, moments and finite rates");
  if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return fail(LS_ERR_INVALID, "bad Adam constants");
  GaussAdamArgs a{};
  for (int r = 0; r < b->R; ++r) {
    const JobDev& J = b->jobs_h[r];
    const float* par[5] = {J.mean, J.log_scale, J.quat, J.opac, J.rgb};
    const ls_adam_array* arr[5] = {&adam[r].mean, &adam[r].log_scale, &adam[r].quat, &adam[r].opacity_logit,
                                   &adam[r].rgb};
    for (int q = 0; q < 5; ++q) {
      if (J.n > 0 && (!arr[q]->m || !arr[q]->v || !std::isfinite(arr[q]->lr)))
        return fail(LS_ERR_INVALID, "render %d: Adam array %d needs moments and a finite rate", r, q);
      a.m[r][q] = arr[q]->m;
      a.v[r][q] = arr[q]->v;
      a.lr[r][q] = arr[q]->lr;
      for (int o = 0; o < r; ++o) {
        const JobDev& K = b->jobs_h[o];
        const float* other[5] = {K.mean, K.log_scale, K.quat, K.opac, K.rgb};
        for (int u = 0; u < 5; ++u)
          if (J.n > 0 && K.n > 0 && par[q] == other[u])
            return fail(LS_ERR_INVALID, "renders %d and %d share a Gaussian array: use ls_render_bwd_project", o, r);
      }
    }
  }
  a.beta1 = beta1;
  a.beta2 = beta2;
  a.eps = eps;
  a.bc1 = (float)(1.0 / (1.0 - std::pow((double)beta1, step)));
  a.bc2 = (float)(1.0 / (1.0 - std::pow((double)beta2, step)));
  if (pose_adam) {
    a.pose = pose;
    a.pose_m = pose_adam->m;
    a.pose_v = pose_adam->v;
    a.lr_rot = pose_adam->lr_rot;
    a.lr_trans = pose_adam->lr_trans;
  }
  const Layout L = layout_of(b, bins->capacity);
  launch_project_bwd(b->jobs_d, b->blk_off_d, b->R, b->nblk_items, pose, p->radius, p->aux,
                     at<float>(bins->work, L.g2d), nullptr, 1, at<float>(bins->work, L.pose_part),
                     pose_grad != nullptr, pose_grad, s, &a);
  return hip_check("ls_render_bwd_project_adam");
}

ls_status ls_render_bwd(const ls_batch* b, const float* pose, const ls_projected* p, const ls_bins* bins,
                        const float* bg, const ls_image* fwd, const ls_image_grad* up, const ls_gaussian_grads* grads,
                        float* pose_grad, hipStream_t s) {
  if (pose_grad && !pose) return fail(LS_ERR_INVALID, "pose_grad needs the pose it is taken at");
  const uint32_t flags = grads ? 0u : LS_BWD_POSE_ONLY;
  ls_status st = ls_render_bwd_tiles(b, pose, p, bins, bg, fwd, up, flags, s);
  if (st) return st;
  return ls_render_bwd_project(b, pose, p, bins, grads, pose_grad, flags, s);
}

ls_status ls_render_stats(const ls_batch* b, const ls_projected* p, const ls_bins* bins, const ls_image* fwd,
                          int64_t* stats, hipStream_t s) {
  if (!b) return fail(LS_ERR_INVALID, "NULL batch");
  ls_status st;
  if ((st = check_projected(p)) || (st = check_bins(b, bins)) || (st = ensure_device(b))) return st;
  if (!fwd || !fwd->n_last || !stats) return fail(LS_ERR_INVALID, "NULL arguments");
  launch_render_stats(b->jobs_d, b->tile_off_d, b->R, b->T, p->rec, bins->item, bins->range, fwd->n_last, stats, s);
  return hip_check("ls_render_stats");
}

ls_status ls_loss_l1(const ls_batch* b, const ls_image* pred, const float* tgt_rgb, const float* tgt_depth,
                     float* loss, float* grad_rgb, float* grad_depth, float* grad_scale, hipStream_t s) {
  if (!b) return fail(LS_ERR_INVALID, "NULL batch");
  if (!pred || !pred->rgb || !pred->depth || !tgt_rgb || !tgt_depth)
    return fail(LS_ERR_INVALID, "NULL image arguments");
  ls_status st;
  if ((st = ensure_device(b))) return st;
  launch_loss_l1(b->jobs_d, b->pblk_off_d, b->R, b->nblk_pix, pred->rgb, pred->depth, tgt_rgb, tgt_depth, grad_rgb,
                 grad_depth, b->loss_part_d, loss, grad_scale, s);
  return hip_check("ls_loss_l1");
}

ls_status ls_loss_tracking(const ls_batch* b, const ls_image* pred, const float* tgt_rgb, const float* tgt_depth,
                           const ls_loss_params* prm, float* loss, float* median, float* grad_rgb, float* grad_depth,
                           float* grad_scale, hipStream_t s) {
  if (!b) return fail(LS_ERR_INVALID, "NULL batch");
  if (!pred || !pred->rgb || !pred->depth || !tgt_rgb || !tgt_depth)
    return fail(LS_ERR_INVALID, "NULL image arguments");
  ls_status st;
  if ((st = ls::check_loss_params(prm, pred)) || (st = ensure_device(b))) return st;
  launch_loss_track(b->jobs_d, b->pblk_off_d, b->R, b->nblk_pix, pred->rgb, pred->depth, pred->alpha, tgt_rgb,
                    tgt_depth, prm->lambda_c, prm->inlier_k, prm->alpha_power, b->sel_d,
                    median ? median : b->median_d, grad_rgb, grad_depth, b->loss_part_d, loss, grad_scale, s);
  return hip_check("ls_loss_tracking");
}

ls_status ls_loss_mapping(const ls_batch* b, const ls_image* pred, const float* tgt_rgb, const float* tgt_depth,
                          const ls_mapping_params* prm, float* loss, float* grad_rgb, float* grad_depth,
                          float* grad_scale, hipStream_t s) {
  if (!b) return fail(LS_ERR_INVALID, "NULL batch");
  if (!pred || !pred->rgb || !pred->depth || !tgt_rgb || !tgt_depth)
    return fail(LS_ERR_INVALID, "NULL image arguments");
  if (!prm) return fail(LS_ERR_INVALID, "NULL mapping-loss parameters");
  if (!std::isfinite(prm->lambda_color) || !std::isfinite(prm->lambda_depth) || !(prm->lambda_ssim >= 0.f) ||
      !(prm->lambda_ssim <= 1.f))
    return fail(LS_ERR_INVALID, "mapping-loss weights must be finite, lambda_ssim in [0, 1]");
  ls_status st;
  if ((st = ensure_device(b))) return st;
  launch_loss_mapping(b->jobs_d, b->pblk_off_d, b->nblk_pix, b->sblk_off_d, b->nblk_ssim, b->R, pred->rgb,
                      pred->depth, tgt_rgb, tgt_depth, prm->lambda_ssim, prm->lambda_color, prm->lambda_depth,
                      grad_rgb, grad_depth, b->loss_part_d, b->map_part_d, loss, grad_scale, s);
  return hip_check("ls_loss_mapping");
}

ls_status ls_loss_isotropic(const float* log_scale, int64_t n, float lambda_reg, float* loss, float* grad_log_scale,
                            float* work, hipStream_t s) {
  if (n < 0 || n > INT32_MAX) return fail(LS_ERR_INVALID, "n out of range");
  if (!loss || !work || (n > 0 && !log_scale)) return fail(LS_ERR_INVALID, "NULL arguments");
  if (!std::isfinite(lambda_reg)) return fail(LS_ERR_INVALID, "lambda_reg must be finite");
  launch_loss_isotropic(log_scale, n, lambda_reg, loss, grad_log_scale, work, s);
  return hip_check("ls_loss_isotropic");
}

ls_status ls_adjust_submaps(const ls_submap_adjust* subs, int32_t count, hipStream_t s) {
  if (count < 0 || (count > 0 && !subs)) return fail(LS_ERR_INVALID, "bad submap list");
  for (int k = 0; k < count; ++k) {
    const ls_submap_adjust& u = subs[k];
    if (u.n < 0 || u.n_poses < 0) return fail(LS_ERR_INVALID, "submap %d: negative size", k);
    if (u.n > 0 && (!u.mean || !u.quat)) return fail(LS_ERR_INVALID, "submap %d: NULL Gaussian arrays", k);
    for (int i = 0; i < 12; ++i)
      if (!std::isfinite(u.T[i])) return fail(LS_ERR_INVALID, "submap %d: non-finite correction", k);
    double dev = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double d = 0.0;
        for (int r = 0; r < 3; ++r) d += (double)u.T[r * 4 + a] * u.T[r * 4 + b];
        dev = std::max(dev, std::fabs(d - (a == b ? 1.0 : 0.0)));
      }
    const float* R = u.T;
    const double det = (double)R[0] * (R[5] * R[10] - R[6] * R[9]) - (double)R[1] * (R[4] * R[10] - R[6] * R[8]) +
                       (double)R[2] * (R[4] * R[9] - R[5] * R[8]);
    if (dev > 1e-3 || det <= 0.0) return fail(LS_ERR_INVALID, "submap %d: correction is not a rigid motion", k);
  }
  if (count == 0) return LS_OK;
  launch_adjust_submaps(subs, count, s);
  return hip_check("ls_adjust_submaps");
}

size_t ls_overlap_workspace_size(int32_t np, int32_t nq) {
  if (np < 0 || nq < 0) return 0;
  return overlap_workspace_bytes(np, nq);
}

ls_status ls_overlap_ratio(const float* p_mean, int32_t np, const float* q_mean, int32_t nq, const float* T_pq,
                           float tau, int32_t* nn_pq, int32_t* nn_qp, int32_t* counts, void* work, size_t work_bytes,
                           hipStream_t s) {
  const ls_status st = overlap_check_args(p_mean, np, q_mean, nq, T_pq, tau, nn_pq, nn_qp, counts);
  if (st != LS_OK) return st;
  const size_t need = overlap_workspace_bytes(np, nq);
  if (work_bytes < need || (need > 0 && !work))
    return fail(LS_ERR_CAPACITY, "overlap workspace needs %zu bytes", need);
  launch_overlap(p_mean, np, q_mean, nq, T_pq, tau, nn_pq, nn_qp, counts, work, s);
  return hip_check("ls_overlap_ratio");
}

size_t ls_prune_workspace_size(int32_t n) { return n < 0 ? 0 : prune_workspace_bytes(n); }

ls_status ls_prune_gaussians(const float* opacity_logit, int32_t n, float o_thre, const ls_prune_array* arrays,
                             int32_t narrays, int32_t* kept_index, int32_t* count, void* work, size_t work_bytes,
                             hipStream_t s) {
  if (n < 0) return fail(LS_ERR_INVALID, "negative Gaussian count");
  if (!(o_thre > 0.f && o_thre < 1.f)) return fail(LS_ERR_INVALID, "o_thre must lie in (0, 1)");
  if (!count || !work || (n > 0 && (!opacity_logit || !kept_index)))
    return fail(LS_ERR_INVALID, "NULL arguments");
  if (narrays < 0 || narrays > LS_PRUNE_MAX_ARRAYS || (narrays > 0 && !arrays))
    return fail(LS_ERR_INVALID, "0..%d arrays", LS_PRUNE_MAX_ARRAYS);
  PruneArrays arr{};
  arr.count = narrays;
  for (int a = 0; a < narrays; ++a) {
    if (arrays[a].components < 0) return fail(LS_ERR_INVALID, "array %d: negative component count", a);
    if (n > 0 && arrays[a].components > 0 && (!arrays[a].src || !arrays[a].dst))
      return fail(LS_ERR_INVALID, "array %d: NULL pointer", a);
    arr.src[a] = arrays[a].src;
    arr.dst[a] = arrays[a].dst;
    arr.comp[a] = arrays[a].components;
  }
  const size_t need = prune_workspace_bytes(n);
  if (work_bytes < need) return fail(LS_ERR_CAPACITY, "pruning workspace needs %zu bytes", need);
  const float tau = (float)std::log((double)o_thre / (1.0 - (double)o_thre));
  launch_prune(opacity_logit, n, tau, arr, kept_index, count, work, s);
  return hip_check("ls_prune_gaussians");
}

ls_status ls_adam(const ls_adam_group* groups, int32_t ngroups, int32_t step, float beta1, float beta2, float eps,
                  int32_t zero_grad, hipStream_t s) {
  if (!groups || ngroups < 1 || ngroups > 16) return fail(LS_ERR_INVALID, "need 1..16 Adam groups");
  if (step < 1) return fail(LS_ERR_INVALID, "Adam step counts from 1");
  for (int i = 0; i < ngroups; ++i)
    if (groups[i].n < 0 || (groups[i].n > 0 && (!groups[i].param || !groups[i].grad || !groups[i].m || !groups[i].v)))
      return fail(LS_ERR_INVALID, "Adam group %d: bad arguments", i);
  const double bc1 = 1.0 / (1.0 - std::pow((double)beta1, step));
  const double bc2 = 1.0 / (1.0 - std::pow((double)beta2, step));
  launch_adam(groups, ngroups, beta1, beta2, eps, (float)bc1, (float)bc2, zero_grad, s);
  return hip_check("ls_adam");
}

}  // extern "C"

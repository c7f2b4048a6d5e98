// Registration serving loop: admission against a device-byte budget,
// continuous batching of every active pair's views in one launch set per
// iteration, HIP-graph capture of that iteration per active set, retirement
// with host-side Eq. 7 fusion.  See include/loopsplat.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "batch.h"
#include "kernels.h"
#include "register_engine.h"

namespace ls {
namespace {

using Clock = std::chrono::steady_clock;

double seconds_since(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double>(b - a).count();
}

// Grow-only device buffer (contents are not preserved when it grows).
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  ls_status ensure(size_t bytes) {
    bytes = std::max<size_t>(bytes, 256);
    if (bytes <= cap) return LS_OK;
    if (p) hipFree(p);
    p = nullptr;
    cap = 0;
    if (hipMalloc(&p, bytes) != hipSuccess) return LS_ERR_HIP;
    cap = bytes;
    return LS_OK;
  }
  void release() {
    if (p) hipFree(p);
    p = nullptr;
    cap = 0;
  }
  template <typename T>
  T* as(size_t off = 0) const {
    return reinterpret_cast<T*>(static_cast<char*>(p) + off);
  }
};

enum class SlotState { kWaiting, kActive, kDone };

struct Slot {
  uint64_t ticket = 0;
  RegPair rp;
  int views = 0;
  int64_t items = 0, pixels = 0;
  size_t bytes = 0;
  SlotState state = SlotState::kWaiting;
  ls_status status = LS_OK;
  int remaining = 0;
  int iters_done = 0;
  int first_render = -1;  // position of its first view in the current epoch
  float T[12] = {0};
  std::vector<float> per_view, resid, expo;  // expo: (a, b) per view when exposure is on
  Clock::time_point t_submit, t_admit, t_done;
  hipEvent_t ready = nullptr;  // recorded on the producer stream at submit; the worker waits on it
  bool waited = false;
  ~Slot() {
    if (ready) hipEventDestroy(ready);
  }
};

// Device bytes the server allocates per item / pixel / expected instance.
constexpr double kBytesPerItem = 48 + 48 + 8 + 16 + 40 + 8;
constexpr double kBytesPerPixel = 12 + 4 + 4 + 4 + 4 + 12 + 4;
constexpr double kInstancesPerItem = 8.0;
constexpr double kBytesPerInstance = 16 + 8;

size_t estimate_bytes(int64_t items, int64_t pixels) {
  return (size_t)(items * (kBytesPerItem + kInstancesPerItem * kBytesPerInstance) + pixels * kBytesPerPixel) +
         (1u << 20);
}

}  // namespace

class Server {
 public:
  explicit Server(const ls_server_params& p) : prm_(p) {}
  ~Server() { stop(); }

  ls_status start() {
    if (hipGetDevice(&device_) != hipSuccess) return LS_ERR_HIP;
    if (hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&check_stream_, hipStreamNonBlocking) != hipSuccess)
      return LS_ERR_HIP;
    if (small_.ensure(4096) || check_buf_.ensure(256)) return LS_ERR_HIP;
    count_ = small_.as<int32_t>(0);
    sticky_ = small_.as<int32_t>(32);
    worker_ = std::thread([this] { loop(); });
    return LS_OK;
  }

  // Device-side check that every Gaussian parameter of the pair is finite.
  ls_status check_finite(const ls_pair* p, hipEvent_t ready) {
    std::lock_guard<std::mutex> g(check_mu_);
    int cur = -1;
    hipGetDevice(&cur);
    if (cur != device_) hipSetDevice(device_);
    if (ready && hipStreamWaitEvent(check_stream_, ready, 0) != hipSuccess) return LS_ERR_HIP;
    int32_t* flag = check_buf_.as<int32_t>();
    launch_fill_i32(flag, 1, 0, check_stream_);
    for (const ls_gaussians* gs : {&p->P, &p->Q}) {
      const int64_t n = gs->n;
      if (n <= 0) continue;
      launch_all_finite(gs->mean, 3 * n, flag, check_stream_);
      launch_all_finite(gs->log_scale, 3 * n, flag, check_stream_);
      launch_all_finite(gs->quat, 4 * n, flag, check_stream_);
      launch_all_finite(gs->opacity_logit, n, flag, check_stream_);
      launch_all_finite(gs->rgb, 3 * n, flag, check_stream_);
    }
    int32_t h = 1;
    if (hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, check_stream_) != hipSuccess ||
        hipStreamSynchronize(check_stream_) != hipSuccess)
      return LS_ERR_HIP;
    if (cur != device_ && cur >= 0) hipSetDevice(cur);
    return h == 0 ? LS_OK : LS_ERR_NONFINITE;
  }

  ls_status submit(const ls_pair* pair, const ls_reg_params* prm, hipStream_t producer, uint64_t* ticket) {
    ls_status st = validate_pair(pair, prm);
    if (st) return st;
    if (prm->joint || prm->top_k > 0) return LS_ERR_INVALID;  // joint registration, view selection: ls_register_pair only
    {
      std::lock_guard<std::mutex> g(mu_);
      if (!have_betas_) {
        beta1_ = prm->beta1;
        beta2_ = prm->beta2;
        eps_ = prm->adam_eps;
        exit_tol_ = prm->exit_rel_tol;
        exit_patience_ = prm->exit_patience;
        exit_mode_ = prm->exit_mode;
        loss_kind_ = prm->loss_kind;
        track_ = prm->track;
        exposure_ = prm->exposure;
        lr_exposure_ = prm->exposure ? prm->lr_exposure : 0.f;
        fused_l1_ = fused_l1_allowed(*prm);
        have_betas_ = true;
      } else if (prm->beta1 != beta1_ || prm->beta2 != beta2_ || prm->adam_eps != eps_ ||
                 prm->exit_rel_tol != exit_tol_ || prm->exit_patience != exit_patience_ ||
                 prm->exit_mode != exit_mode_ ||
                 prm->loss_kind != loss_kind_ || prm->exposure != exposure_ ||
                 (exposure_ && prm->lr_exposure != lr_exposure_) ||
                 (loss_kind_ == 1 && (prm->track.lambda_c != track_.lambda_c ||
                                      prm->track.inlier_k != track_.inlier_k ||
                                      prm->track.alpha_power != track_.alpha_power))) {
        return LS_ERR_INVALID;
      }
    }
    auto s = std::make_unique<Slot>();
    if (producer) {  // order every read of the pair's buffers after the work queued on the producer
      if (hipEventCreateWithFlags(&s->ready, hipEventDisableTiming) != hipSuccess) return LS_ERR_HIP;
      if (hipEventRecord(s->ready, producer) != hipSuccess) return LS_ERR_HIP;
    }
    if ((st = check_finite(pair, s->ready))) return st;
    s->rp = make_reg_pair(pair, prm);
    s->views = pair->vP + pair->vQ;
    s->items = (int64_t)pair->vP * pair->Q.n + (int64_t)pair->vQ * pair->P.n;
    s->pixels = (int64_t)s->views * pair->K.width * pair->K.height;
    s->bytes = estimate_bytes(s->items, s->pixels);
    if (s->bytes > prm_.hbm_budget_bytes) return LS_ERR_BUDGET;
    s->remaining = prm->iters;
    s->t_submit = Clock::now();
    std::lock_guard<std::mutex> g(mu_);
    s->ticket = ++next_ticket_;
    *ticket = s->ticket;
    waiting_.push_back(s.get());
    slots_[s->ticket] = std::move(s);
    ++stats_.submitted;
    cv_.notify_all();
    return LS_OK;
  }

  ls_status poll(uint64_t ticket, ls_reg_result* out, double* times) {
    std::lock_guard<std::mutex> g(mu_);
    auto it = slots_.find(ticket);
    if (it == slots_.end()) return LS_ERR_INVALID;
    Slot* s = it->second.get();
    if (s->state != SlotState::kDone) return LS_NOT_READY;
    if (out) {
      std::memcpy(out->T_PQ, s->T, sizeof(s->T));
      if (out->per_view_T && !s->per_view.empty()) std::memcpy(out->per_view_T, s->per_view.data(), 4 * s->per_view.size());
      if (out->residual && !s->resid.empty()) std::memcpy(out->residual, s->resid.data(), 4 * s->resid.size());
      if (out->exposure && !s->expo.empty()) std::memcpy(out->exposure, s->expo.data(), 4 * s->expo.size());
      out->status = s->status;
      out->iters_done = s->iters_done;
      out->instances_required = 0;
      out->workspace_required = 0;
    }
    if (times) {
      times[0] = seconds_since(s->t_submit, s->t_admit);
      times[1] = seconds_since(s->t_admit, s->t_done);
      times[2] = seconds_since(s->t_submit, s->t_done);
    }
    const ls_status st = s->status;
    slots_.erase(it);
    return st;
  }

  void get_stats(ls_server_stats* out) {
    std::lock_guard<std::mutex> g(mu_);
    *out = stats_;
    out->active = (int32_t)active_.size();
    out->waiting = (int32_t)waiting_.size();
  }

  void stop() {
    {
      std::lock_guard<std::mutex> g(mu_);
      stopping_ = true;
      cv_.notify_all();
    }
    if (worker_.joinable()) worker_.join();
    if (exec_) hipGraphExecDestroy(exec_);
    exec_ = nullptr;
    if (batch_) ls_batch_destroy(batch_);
    batch_ = nullptr;
    for (DevBuf* b : {&items_, &pixels_, &tiles_, &bins_, &work_, &stateA_, &stateB_, &snap_, &small_, &stage_,
                      &check_buf_, &epart_})
      b->release();
    if (stream_) hipStreamDestroy(stream_);
    if (check_stream_) hipStreamDestroy(check_stream_);
    stream_ = check_stream_ = nullptr;
  }

 private:
  // ---------------------------------------------------------------- worker
  void loop() {
    hipSetDevice(device_);
    for (;;) {
      bool changed = false;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [this] { return stopping_ || !waiting_.empty() || !active_.empty(); });
        if (stopping_ && waiting_.empty() && active_.empty()) return;
        changed = admit_locked();
      }
      if (changed || rebuild_pending_) {
        if (rebuild() != LS_OK) {
          fail_active(LS_ERR_HIP);
          continue;
        }
      }
      if (active_.empty()) continue;
      run_chunk();
    }
  }

  // FIFO admission: the head waits until it fits (no overtaking).
  bool admit_locked() {
    bool changed = false;
    while (!waiting_.empty() && (int)active_.size() < prm_.max_slots) {
      Slot* s = waiting_.front();
      if (active_bytes_ + s->bytes > prm_.hbm_budget_bytes) break;
      if (prm_.max_active_pixels > 0 && !active_.empty() && active_pixels_ + s->pixels > prm_.max_active_pixels) break;
      // the tile lists of one launch set are indexed in int32: hold the head back while the
      // active set's expected instance count would pass that (a pair alone is always admitted)
      if (!active_.empty() && (double)(active_items_ + s->items) * kInstancesPerItem > (double)INT32_MAX) break;
      waiting_.pop_front();
      s->state = SlotState::kActive;
      s->t_admit = Clock::now();
      s->first_render = -1;
      active_.push_back(s);
      active_bytes_ += s->bytes;
      active_pixels_ += s->pixels;
      active_items_ += s->items;
      stats_.peak_bytes = std::max<int64_t>(stats_.peak_bytes, (int64_t)active_bytes_);
      stats_.peak_active = std::max<int32_t>(stats_.peak_active, (int32_t)active_.size());
      changed = true;
    }
    return changed;
  }

  // New batch over the active set; per-view state carried over by a remap.
  ls_status rebuild() {
    rebuild_pending_ = false;
    {
      std::lock_guard<std::mutex> g(mu_);
      ++stats_.epochs;
    }
    if (exec_) hipGraphExecDestroy(exec_);
    exec_ = nullptr;
    if (active_.empty()) return LS_OK;
    for (Slot* s : active_)  // a new pair's buffers are read only after its producer's work
      if (s->ready && !s->waited) {
        if (hipStreamWaitEvent(stream_, s->ready, 0) != hipSuccess) return LS_ERR_HIP;
        s->waited = true;
      }
    std::vector<ls_render_job> jobs;
    std::vector<const float*> trgb, tdep;
    std::vector<int32_t> map;
    std::vector<ViewOpt> init;
    views_.clear();
    for (Slot* s : active_) {
      const ls_pair& pr = s->rp.pair;
      const int64_t hw = (int64_t)pr.K.width * pr.K.height;
      const int prev = s->first_render;
      s->first_render = (int)jobs.size();
      int k = 0;
      for (int dir = 0; dir < 2; ++dir) {
        const int nv = dir == 0 ? pr.vP : pr.vQ;
        for (int i = 0; i < nv; ++i, ++k) {
          View v;
          v.pair = 0;
          v.index = i;
          v.reverse = dir == 1;
          const std::vector<double>& c = dir == 0 ? s->rp.c2wP : s->rp.c2wQ;
          for (int q = 0; q < 12; ++q) v.c2w[q] = c[12 * i + q];
          double w2c[12];
          rigid_inv(v.c2w, w2c);
          ls_render_job j{};
          j.g = dir == 0 ? pr.Q : pr.P;
          j.K = pr.K;
          for (int q = 0; q < 12; ++q) j.w2c[q] = (float)w2c[q];
          jobs.push_back(j);
          views_.push_back(v);
          trgb.push_back((dir == 0 ? pr.rgbP : pr.rgbQ) + 3 * hw * i);
          tdep.push_back((dir == 0 ? pr.depthP : pr.depthQ) + hw * i);
          map.push_back(prev >= 0 ? prev + k : -1);
          init.push_back(ViewOpt{s->rp.prm.lr_rot, s->rp.prm.lr_trans, 0, 1, 0.f, 0, 0.f, 0});
        }
      }
    }
    const int Rold = R_;
    R_ = (int)jobs.size();
    if (batch_) ls_batch_destroy(batch_);
    batch_ = nullptr;
    ls_status st;
    if ((st = ls_batch_create(jobs.data(), R_, &batch_)) || (st = batch_set_targets(batch_, trgb, tdep))) return st;
    ls_batch_info info{};
    ls_batch_query(batch_, 0, &info);
    M_ = info.items;
    P_ = info.pixels;
    T_ = info.tiles;

    // per-view state: old (A) -> new (B), then swap
    const size_t sbytes = state_bytes(R_);
    if ((st = stateB_.ensure(sbytes)) || (st = snap_.ensure(sbytes)) || (st = stage_.ensure(4 * (size_t)R_ + sizeof(ViewOpt) * R_ + 512)))
      return st;
    if (Rold == 0 && (st = stateA_.ensure(sbytes))) return st;
    int32_t* dmap = stage_.as<int32_t>();
    ViewOpt* dinit = stage_.as<ViewOpt>(align(4 * (size_t)R_));
    hipMemcpyAsync(dmap, map.data(), 4 * (size_t)R_, hipMemcpyHostToDevice, stream_);
    hipMemcpyAsync(dinit, init.data(), sizeof(ViewOpt) * R_, hipMemcpyHostToDevice, stream_);
    StatePtrs a = state_ptrs(stateA_, std::max(Rold, 1)), b = state_ptrs(stateB_, R_);
    launch_state_remap(a.pose, a.m, a.v, a.opt, b.pose, b.m, b.v, b.grad, b.opt, dmap, dinit, R_, stream_,
                       ExpoState{a.expo, a.em, a.ev, a.eg}, ExpoState{b.expo, b.em, b.ev, b.eg});
    if ((st = epart_.ensure(8 * (size_t)std::max(batch_->nblk_pix, 1)))) return st;
    if (hipStreamSynchronize(stream_) != hipSuccess) return LS_ERR_HIP;  // host map/init must outlive the copies
    std::swap(stateA_, stateB_);
    // with the fused L1 backward, 1 / |Omega| of every view once per active set
    if (fused_l1_ && (st = batch_valid_inv(batch_, nullptr, state_ptrs(stateA_, R_).scale, stream_))) return st;

    // scratch sized for this active set
    const size_t o_rad = align(48 * (size_t)std::max<int64_t>(M_, 1)), o_til = o_rad + align(4 * M_);
    const size_t o_aux = o_til + align(4 * M_);
    if ((st = items_.ensure(o_aux + align(48 * (size_t)std::max<int64_t>(M_, 1))))) return st;
    proj_.rec = items_.as<float>();
    proj_.radius = items_.as<int32_t>(o_rad);
    proj_.tiles = items_.as<int32_t>(o_til);
    proj_.aux = items_.as<float>(o_aux);
    size_t off = 0;
    auto px = [&](size_t per) { const size_t o = off; off += align(per * P_); return o; };
    const size_t o_rgb = px(12), o_dep = px(4), o_al = px(4), o_T = px(4), o_nl = px(4), o_grgb = px(12),
                 o_gdep = px(4);
    if ((st = pixels_.ensure(off))) return st;
    img_.rgb = pixels_.as<float>(o_rgb);
    img_.depth = pixels_.as<float>(o_dep);
    img_.alpha = pixels_.as<float>(o_al);
    img_.T_final = pixels_.as<float>(o_T);
    img_.n_last = pixels_.as<int32_t>(o_nl);
    g_rgb_ = pixels_.as<float>(o_grgb);
    g_depth_ = pixels_.as<float>(o_gdep);
    if ((st = tiles_.ensure(8 * (size_t)T_ + 256))) return st;
    // tile-instance capacity from the count required at the current poses
    int64_t cap = std::max<int64_t>(4096, (int64_t)std::min<double>(6.0 * M_, (double)INT32_MAX));
    for (int attempt = 0; attempt < 2; ++attempt) {
      if ((st = set_capacity(cap))) return st;
      const StatePtrs s = state_ptrs(stateA_, R_);
      if ((st = ls_project(batch_, s.pose, &proj_, stream_)) || (st = ls_bin_sort(batch_, &proj_, &bins_c_, stream_)))
        return st;
      int32_t hc[4];
      hipMemcpyAsync(hc, count_, 16, hipMemcpyDeviceToHost, stream_);
      if (hipStreamSynchronize(stream_) != hipSuccess) return LS_ERR_HIP;
      const int64_t want = (int64_t)std::min<double>((double)INT32_MAX,
                                                     std::max<double>(1024.0, hc[2] * (double)prm_.instance_headroom));
      cap = want;
      if (hc[1] == 0) break;
    }
    if ((st = set_capacity(cap))) return st;
    if (prm_.use_graphs) return capture();
    return LS_OK;
  }

  struct StatePtrs {
    float *pose, *m, *v, *grad, *loss, *scale;
    ViewOpt* opt;
    float *expo, *em, *ev, *eg;  // exposure coefficients (a, b) per view, their moments and gradient
  };
  static size_t align(size_t x) { return (x + 255) & ~size_t(255); }
  static size_t state_bytes(int R) {
    return 4 * align(28 * (size_t)R) + 2 * align(4 * (size_t)R) + align(sizeof(ViewOpt) * R) + 4 * align(8 * (size_t)R);
  }
  static StatePtrs state_ptrs(const DevBuf& b, int R) {
    StatePtrs s;
    size_t o = 0;
    s.pose = b.as<float>(o); o += align(28 * (size_t)R);
    s.m = b.as<float>(o); o += align(28 * (size_t)R);
    s.v = b.as<float>(o); o += align(28 * (size_t)R);
    s.grad = b.as<float>(o); o += align(28 * (size_t)R);
    s.loss = b.as<float>(o); o += align(4 * (size_t)R);
    s.scale = b.as<float>(o); o += align(4 * (size_t)R);
    s.opt = b.as<ViewOpt>(o); o += align(sizeof(ViewOpt) * R);
    s.expo = b.as<float>(o); o += align(8 * (size_t)R);
    s.em = b.as<float>(o); o += align(8 * (size_t)R);
    s.ev = b.as<float>(o); o += align(8 * (size_t)R);
    s.eg = b.as<float>(o);
    return s;
  }

  ls_status set_capacity(int64_t cap) {
    ls_batch_info info{};
    ls_status st = ls_batch_query(batch_, cap, &info);
    if (st) return st;
    if ((st = bins_.ensure(2 * align(4 * (size_t)cap))) || (st = work_.ensure(info.workspace_bytes))) return st;
    // the image-space gradient accumulator must start at zero
    if (hipMemsetAsync(work_.p, 0, info.workspace_bytes, stream_) != hipSuccess) return LS_ERR_HIP;
    capacity_ = cap;
    bins_c_.capacity = cap;
    bins_c_.tile_of = bins_.as<uint32_t>();
    bins_c_.item = bins_.as<int32_t>(align(4 * (size_t)cap));
    bins_c_.range = tiles_.as<int32_t>();
    bins_c_.count = count_;
    bins_c_.work = work_.p;
    return LS_OK;
  }

  // The loss fixed for this server (plain L1 or the masked tracking loss).
  ls_status view_loss(const StatePtrs& s) {
    if (exposure_)
      return batch_loss_exposure(batch_, loss_kind_, &track_, &img_, nullptr, nullptr, s.expo, epart_.as<float>(), s.eg,
                                 s.loss, g_rgb_, g_depth_, s.scale, stream_);
    if (loss_kind_ == 1)
      return batch_loss_tracking(batch_, &img_, &track_, s.loss, g_rgb_, g_depth_, s.scale, stream_);
    return batch_loss_l1(batch_, &img_, s.loss, g_rgb_, g_depth_, s.scale, stream_);
  }

  // One batched iteration (also the body of the captured graph).
  ls_status iteration() {
    const StatePtrs s = state_ptrs(stateA_, R_);
    const ls_image_grad up{g_rgb_, g_depth_, nullptr, s.scale};
    ls_status st;
    if ((st = project_views(batch_, s.pose, &proj_, s.opt, stream_)) ||
        (st = ls_bin_sort(batch_, &proj_, &bins_c_, stream_)))
      return st;
    if ((st = ls_render_fwd(batch_, &proj_, &bins_c_, nullptr, &img_, stream_))) return st;
    if (fused_l1_)  // the backward forms the L1 gradient itself (no per-iteration loss value)
      st = render_bwd_pose_l1(batch_, s.pose, &proj_, &bins_c_, &img_, nullptr, nullptr, s.scale, stream_);
    else if (!(st = view_loss(s)))
      st = ls_render_bwd_tiles(batch_, s.pose, &proj_, &bins_c_, nullptr, &img_, &up, LS_BWD_POSE_ONLY, stream_);
    if (st) return st;
    // pose gradients, Adam steps and the sticky overflow flag in one launch
    const PoseAdamArgs a{s.pose, s.grad, s.m, s.v, s.opt, s.loss, beta1_, beta2_, eps_, exit_tol_, exit_patience_,
                         exit_mode_, exposure_ ? s.expo : nullptr, s.eg, s.em, s.ev, lr_exposure_};
    return pose_reduce_adam(batch_, &bins_c_, a, count_, sticky_, stream_);
  }

  ls_status capture() {
    if (exec_) hipGraphExecDestroy(exec_);
    exec_ = nullptr;
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal) != hipSuccess) return LS_ERR_HIP;
    const ls_status st = iteration();
    const hipError_t e = hipStreamEndCapture(stream_, &graph);
    if (st || e != hipSuccess) {
      if (graph) hipGraphDestroy(graph);
      return st ? st : LS_ERR_HIP;
    }
    const hipError_t ie = hipGraphInstantiate(&exec_, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    return ie == hipSuccess ? LS_OK : LS_ERR_HIP;
  }

  void run_chunk() {
    int k = prm_.chunk_iters;
    for (Slot* s : active_) k = std::min(k, s->remaining);
    int64_t replays = 0, retries = 0;
    const size_t sbytes = state_bytes(R_);
    for (int attempt = 0;; ++attempt) {
      hipMemcpyAsync(snap_.p, stateA_.p, sbytes, hipMemcpyDeviceToDevice, stream_);
      launch_fill_i32(sticky_, 1, 0, stream_);
      ls_status st = LS_OK;
      for (int i = 0; i < k && !st; ++i) {
        if (exec_) {
          st = hipGraphLaunch(exec_, stream_) == hipSuccess ? LS_OK : LS_ERR_HIP;
          ++replays;
        } else {
          st = iteration();
        }
      }
      int32_t ovf = 0;
      hipMemcpyAsync(&ovf, sticky_, 4, hipMemcpyDeviceToHost, stream_);
      if (hipStreamSynchronize(stream_) != hipSuccess) st = LS_ERR_HIP;
      if (st) {
        fail_active(st);
        return;
      }
      if (!ovf) break;
      // the instance count outgrew the capacity: restore the chunk's start and re-run it larger
      ++retries;
      hipMemcpyAsync(stateA_.p, snap_.p, sbytes, hipMemcpyDeviceToDevice, stream_);
      int32_t need = 0;
      hipMemcpyAsync(&need, count_ + 2, 4, hipMemcpyDeviceToHost, stream_);
      hipStreamSynchronize(stream_);
      const int64_t want = std::min<int64_t>((int64_t)INT32_MAX,
                                             std::max<int64_t>(capacity_ * 2, (int64_t)(need * 1.25) + 1024));
      if (attempt >= 3 || set_capacity(want) ||
          (prm_.use_graphs && capture())) {
        fail_active(LS_ERR_CAPACITY);
        return;
      }
    }
    {
      std::lock_guard<std::mutex> g(mu_);
      stats_.iterations += k;
      stats_.graph_replays += replays;
      stats_.overflow_retries += retries;
    }
    bool any_done = false;
    std::vector<ViewOpt> ho;
    if (exit_patience_ > 0) {  // pairs whose views have all stopped are finished early
      ho.resize(R_);
      hipMemcpyAsync(ho.data(), state_ptrs(stateA_, R_).opt, sizeof(ViewOpt) * R_, hipMemcpyDeviceToHost, stream_);
      if (hipStreamSynchronize(stream_) != hipSuccess) {
        fail_active(LS_ERR_HIP);
        return;
      }
    }
    for (Slot* s : active_) {
      s->remaining -= k;
      s->iters_done += k;
      if (!ho.empty()) {
        bool any_active = false;
        for (int v = 0; v < s->views; ++v) any_active |= ho[s->first_render + v].active != 0;
        if (!any_active) s->remaining = 0;
      }
      any_done |= s->remaining == 0;
    }
    if (any_done) retire();
  }

  // Final forward at the current poses, readback, fusion of finished pairs.
  // The residual of a view is the unmasked L1 there, as in ls_register_pair.
  // An overflow of the residual forward grows the capacity and retries, at
  // most kRetireAttempts times.
  static constexpr int kRetireAttempts = 3;
  void retire(int attempt = 0) {
    const StatePtrs s = state_ptrs(stateA_, R_);
    ls_status st;
    if ((st = ls_project(batch_, s.pose, &proj_, stream_)) || (st = ls_bin_sort(batch_, &proj_, &bins_c_, stream_)) ||
        (st = ls_render_fwd(batch_, &proj_, &bins_c_, nullptr, &img_, stream_)) ||
        (st = exposure_ ? batch_loss_exposure(batch_, 0, nullptr, &img_, nullptr, nullptr, s.expo, nullptr, nullptr,
                                              s.loss, g_rgb_, g_depth_, s.scale, stream_)
                        : batch_loss_l1(batch_, &img_, s.loss, g_rgb_, g_depth_, s.scale, stream_))) {
      fail_active(st);
      return;
    }
    std::vector<float> pose_h(7 * (size_t)R_), loss_h(R_), expo_h(exposure_ ? 2 * (size_t)R_ : 0);
    int32_t hc[4] = {0, 0, 0, 0};
    if (exposure_) hipMemcpyAsync(expo_h.data(), s.expo, 8 * (size_t)R_, hipMemcpyDeviceToHost, stream_);
    hipMemcpyAsync(pose_h.data(), s.pose, 28 * (size_t)R_, hipMemcpyDeviceToHost, stream_);
    hipMemcpyAsync(loss_h.data(), s.loss, 4 * (size_t)R_, hipMemcpyDeviceToHost, stream_);
    hipMemcpyAsync(hc, count_, 16, hipMemcpyDeviceToHost, stream_);
    if (hipStreamSynchronize(stream_) != hipSuccess) {
      fail_active(LS_ERR_HIP);
      return;
    }
    if (hc[1]) {  // residual forward overflowed: grow and redo the residuals
      {
        std::lock_guard<std::mutex> g(mu_);
        ++stats_.overflow_retries;
      }
      const int64_t want = std::min<int64_t>((int64_t)INT32_MAX, (int64_t)(hc[2] * 1.25) + 4096);
      if (attempt + 1 >= kRetireAttempts || want <= capacity_ || set_capacity(want) ||
          (prm_.use_graphs && capture())) {
        fail_active(LS_ERR_CAPACITY);
        return;
      }
      retire(attempt + 1);
      return;
    }
    std::vector<Slot*> keep;
    std::lock_guard<std::mutex> g(mu_);
    for (Slot* sl : active_) {
      if (sl->remaining > 0) {
        keep.push_back(sl);
        continue;
      }
      finish_slot(sl, pose_h, loss_h, expo_h);
      active_bytes_ -= sl->bytes;
      active_pixels_ -= sl->pixels;
      active_items_ -= sl->items;
    }
    active_.swap(keep);
    rebuild_pending_ = true;
    cv_.notify_all();
  }

  void finish_slot(Slot* sl, const std::vector<float>& pose_h, const std::vector<float>& loss_h,
                   const std::vector<float>& expo_h) {
    const int n = sl->views, r0 = sl->first_render;
    if (!expo_h.empty()) sl->expo.assign(expo_h.begin() + 2 * (size_t)r0, expo_h.begin() + 2 * (size_t)(r0 + n));
    std::vector<double> est(12 * (size_t)n), res(n);
    std::vector<int32_t> rev(n);
    sl->per_view.assign(12 * (size_t)n, 0.f);
    sl->resid.assign(n, 0.f);
    ls_status st = LS_OK;
    for (int k = 0; k < n && !st; ++k) {
      const View& v = views_[r0 + k];
      for (int q = 0; q < 7; ++q)
        if (!std::isfinite(pose_h[7 * (size_t)(r0 + k) + q])) st = LS_ERR_NONFINITE;
      if (!std::isfinite(loss_h[r0 + k])) st = LS_ERR_NONFINITE;
      if (st) break;
      view_estimate(v.c2w, &pose_h[7 * (size_t)(r0 + k)], &est[12 * (size_t)k]);
      res[k] = loss_h[r0 + k];
      rev[k] = v.reverse ? 1 : 0;
      for (int q = 0; q < 12; ++q) sl->per_view[12 * (size_t)k + q] = (float)est[12 * (size_t)k + q];
      sl->resid[k] = loss_h[r0 + k];
    }
    double T[12];
    if (!st) st = fuse_estimates(est.data(), res.data(), rev.data(), n, T);
    if (!st)
      for (int q = 0; q < 12; ++q) sl->T[q] = (float)T[q];
    sl->status = st;
    sl->state = SlotState::kDone;
    sl->t_done = Clock::now();
    if (st) ++stats_.failed; else ++stats_.completed;
  }

  void fail_active(ls_status st) {
    std::lock_guard<std::mutex> g(mu_);
    for (Slot* sl : active_) {
      sl->status = st;
      sl->state = SlotState::kDone;
      sl->t_done = Clock::now();
      ++stats_.failed;
      active_bytes_ -= sl->bytes;
      active_pixels_ -= sl->pixels;
      active_items_ -= sl->items;
    }
    active_.clear();
    R_ = 0;
    rebuild_pending_ = true;
    cv_.notify_all();
  }

  ls_server_params prm_;
  int device_ = 0;
  hipStream_t stream_ = nullptr, check_stream_ = nullptr;
  std::mutex check_mu_;
  DevBuf check_buf_;
  bool have_betas_ = false;
  float beta1_ = 0.9f, beta2_ = 0.999f, eps_ = 1e-8f, exit_tol_ = 0.f;
  int32_t exit_patience_ = 0, exit_mode_ = 0;
  bool fused_l1_ = false;  // iterations take render_bwd_pose_l1 (set with the first request's settings)
  int32_t loss_kind_ = 0;
  ls_loss_params track_{};
  int32_t exposure_ = 0;  // exposure coefficients on (fixed by the first request, like the loss)
  float lr_exposure_ = 0.f;
  DevBuf epart_;           // exposure-gradient block partials of the active set
  std::thread worker_;
  std::mutex mu_;
  std::condition_variable cv_;
  bool stopping_ = false;
  uint64_t next_ticket_ = 0;
  std::map<uint64_t, std::unique_ptr<Slot>> slots_;
  std::deque<Slot*> waiting_;
  std::vector<Slot*> active_;
  size_t active_bytes_ = 0;
  int64_t active_pixels_ = 0;
  int64_t active_items_ = 0;  // rendered Gaussians per iteration of the active set
  ls_server_stats stats_{};
  bool rebuild_pending_ = false;

  // epoch state (worker thread only)
  ls_batch* batch_ = nullptr;
  int R_ = 0, T_ = 0;
  int64_t M_ = 0, P_ = 0, capacity_ = 0;
  std::vector<View> views_;
  DevBuf items_, pixels_, tiles_, bins_, work_, stateA_, stateB_, snap_, small_, stage_;
  ls_projected proj_{};
  ls_bins bins_c_{};
  ls_image img_{};
  float *g_rgb_ = nullptr, *g_depth_ = nullptr;
  int32_t *count_ = nullptr, *sticky_ = nullptr;
  hipGraphExec_t exec_ = nullptr;
};

}  // namespace ls

struct ls_server {
  std::unique_ptr<ls::Server> impl;
};

extern "C" {

ls_status ls_server_create(const ls_server_params* prm, ls_server** out) {
  if (!prm || !out) return LS_ERR_INVALID;
  *out = nullptr;
  if (prm->max_slots < 1 || prm->chunk_iters < 1 || !(prm->instance_headroom >= 0.25f) || prm->hbm_budget_bytes == 0 ||
      prm->max_active_pixels < 0)
    return LS_ERR_INVALID;
  auto* s = new ls_server();
  s->impl = std::make_unique<ls::Server>(*prm);
  const ls_status st = s->impl->start();
  if (st) {
    delete s;
    return st;
  }
  *out = s;
  return LS_OK;
}

ls_status ls_register_submit(ls_server* sv, const ls_pair* pair, const ls_reg_params* prm, hipStream_t producer,
                             uint64_t* ticket) {
  if (!sv || !ticket) return LS_ERR_INVALID;
  return sv->impl->submit(pair, prm, producer, ticket);
}

ls_status ls_register_poll(ls_server* sv, uint64_t ticket, ls_reg_result* out, double* times) {
  if (!sv) return LS_ERR_INVALID;
  return sv->impl->poll(ticket, out, times);
}

ls_status ls_server_get_stats(ls_server* sv, ls_server_stats* out) {
  if (!sv || !out) return LS_ERR_INVALID;
  sv->impl->get_stats(out);
  return LS_OK;
}

ls_status ls_server_destroy(ls_server* sv) {
  if (!sv) return LS_OK;
  sv->impl->stop();
  delete sv;
  return LS_OK;
}

}  // extern "C"

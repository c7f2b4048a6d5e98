// 3DGS registration as keyframe localisation (Sec. 3.2) on top of the
// rasterizer calls: every keyframe of P localised in Q and every keyframe of
// Q in P, all views of all pairs of an engine in one launch set per Adam
// iteration, then the Eq. 7 fusion on the host in double precision.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <vector>

#include "batch.h"
#include "kernels.h"
#include "register_engine.h"

namespace ls {

// ------------------------------------------------------------------ host math

void rot_of_quat(const double* q, double* R) {
  const double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

// 3x4 rigid transforms, row-major [R | t].
void rigid_inv(const double* A, double* out) {
  double o[12];
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) o[i * 4 + j] = A[j * 4 + i];
    o[i * 4 + 3] = -(A[0 * 4 + i] * A[3] + A[1 * 4 + i] * A[7] + A[2 * 4 + i] * A[11]);
  }
  std::memcpy(out, o, sizeof(o));
}

void rigid_mul(const double* A, const double* B, double* out) {
  double o[12];
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) o[i * 4 + j] = A[i * 4 + 0] * B[0 * 4 + j] + A[i * 4 + 1] * B[1 * 4 + j] + A[i * 4 + 2] * B[2 * 4 + j];
    o[i * 4 + 3] = A[i * 4 + 0] * B[3] + A[i * 4 + 1] * B[7] + A[i * 4 + 2] * B[11] + A[i * 4 + 3];
  }
  std::memcpy(out, o, sizeof(o));
}

// Unit quaternion of a rotation (row-major), largest-diagonal branch.
static void quat_of_rot(const double* R, double* q) {
  const double tr = R[0] + R[4] + R[8];
  if (tr > 0.0) {
    const double S = std::sqrt(tr + 1.0) * 2.0;
    q[0] = 0.25 * S; q[1] = (R[7] - R[5]) / S; q[2] = (R[2] - R[6]) / S; q[3] = (R[3] - R[1]) / S;
  } else if (R[0] > R[4] && R[0] > R[8]) {
    const double S = std::sqrt(1.0 + R[0] - R[4] - R[8]) * 2.0;
    q[0] = (R[7] - R[5]) / S; q[1] = 0.25 * S; q[2] = (R[1] + R[3]) / S; q[3] = (R[2] + R[6]) / S;
  } else if (R[4] > R[8]) {
    const double S = std::sqrt(1.0 + R[4] - R[0] - R[8]) * 2.0;
    q[0] = (R[2] - R[6]) / S; q[1] = (R[1] + R[3]) / S; q[2] = 0.25 * S; q[3] = (R[5] + R[7]) / S;
  } else {
    const double S = std::sqrt(1.0 + R[8] - R[0] - R[4]) * 2.0;
    q[0] = (R[3] - R[1]) / S; q[1] = (R[2] + R[6]) / S; q[2] = (R[5] + R[7]) / S; q[3] = 0.25 * S;
  }
  const double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; ++k) q[k] /= n;
}

// E = C Delta^-1 C^-1 for a keyframe c2w C and its optimised correction Delta.
void view_estimate(const double* c2w, const float* pose7, double* E) {
  const double q[4] = {pose7[0], pose7[1], pose7[2], pose7[3]};
  double D[12];
  double R[9];
  rot_of_quat(q, R);
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) D[i * 4 + j] = R[i * 3 + j];
    D[i * 4 + 3] = pose7[4 + i];
  }
  double Di[12], Ci[12], tmp[12];
  rigid_inv(D, Di);
  rigid_inv(c2w, Ci);
  rigid_mul(c2w, Di, tmp);
  rigid_mul(tmp, Ci, E);
}

// Eigenvector of the largest eigenvalue of a symmetric 4x4 (cyclic Jacobi).
static void top_eigvec4(double A[4][4], double* out) {
  double V[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0;
    for (int p = 0; p < 4; ++p)
      for (int q = p + 1; q < 4; ++q) off += A[p][q] * A[p][q];
    if (off < 1e-30) break;
    for (int p = 0; p < 4; ++p)
      for (int q = p + 1; q < 4; ++q) {
        if (std::fabs(A[p][q]) < 1e-300) continue;
        const double theta = (A[q][q] - A[p][p]) / (2 * A[p][q]);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1));
        const double c = 1 / std::sqrt(t * t + 1), s = t * c;
        for (int k = 0; k < 4; ++k) {  // A <- J^T A J
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 4; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 4; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
  int best = 0;
  for (int k = 1; k < 4; ++k)
    if (A[k][k] > A[best][best]) best = k;
  for (int k = 0; k < 4; ++k) out[k] = V[k][best];
}

int fuse_estimates(const double* est, const double* resid, const int32_t* rev, int n, double* out) {
  double M[9] = {0}, ts[3] = {0}, wsum = 0;
  for (int i = 0; i < n; ++i) {
    double e[12];
    if (rev[i]) rigid_inv(est + 12 * i, e); else std::memcpy(e, est + 12 * i, sizeof(e));
    const double w = 1.0 / std::max(resid[i], 1e-12);
    if (!std::isfinite(w)) return LS_ERR_NONFINITE;
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c) M[r * 3 + c] += w * e[r * 4 + c];
      ts[r] += w * e[r * 4 + 3];
    }
    wsum += w;
  }
  // argmax_R tr(R^T M) over SO(3): q maximising q^T N q (N quadratic form of tr(R(q)^T M))
  double N[4][4] = {
      {M[0] + M[4] + M[8], M[7] - M[5], M[2] - M[6], M[3] - M[1]},
      {M[7] - M[5], M[0] - M[4] - M[8], M[1] + M[3], M[2] + M[6]},
      {M[2] - M[6], M[1] + M[3], -M[0] + M[4] - M[8], M[5] + M[7]},
      {M[3] - M[1], M[2] + M[6], M[5] + M[7], -M[0] - M[4] + M[8]},
  };
  double q[4];
  top_eigvec4(N, q);
  double R[9];
  rot_of_quat(q, R);
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) out[r * 4 + c] = R[r * 3 + c];
    out[r * 4 + 3] = ts[r] / wsum;
  }
  for (int k = 0; k < 12; ++k)
    if (!std::isfinite(out[k])) return LS_ERR_NONFINITE;
  return LS_OK;
}

// ------------------------------------------------------------------ engine

RegEngine::~RegEngine() { release(); }

void RegEngine::release() {
  if (batch) ls_batch_destroy(batch);
  batch = nullptr;
}

// Host side of an engine: one render job per view (a keyframe of one submap
// rendering the other), the host batch tables and the workspace layout.
ls_status RegEngine::prepare(const std::vector<RegPair>& pairs_in) {
  release();
  pairs = pairs_in;
  std::vector<ls_render_job> jobs;
  first_view.assign(pairs.size() + 1, 0);
  views.clear();
  for (size_t p = 0; p < pairs.size(); ++p) {
    const ls_pair& pr = pairs[p].pair;
    first_view[p] = (int)jobs.size();
    for (int dir = 0; dir < 2; ++dir) {
      const int nv = dir == 0 ? pr.vP : pr.vQ;
      const std::vector<int>& sel = pairs[p].sel[dir];
      const int nsel = sel.empty() ? nv : (int)sel.size();
      for (int k = 0; k < nsel; ++k) {
        const int i = sel.empty() ? k : sel[k];
        View v;
        v.pair = (int)p;
        v.reverse = dir == 1;
        v.index = i;
        for (int k = 0; k < 12; ++k) v.c2w[k] = (dir == 0 ? pairs[p].c2wP : pairs[p].c2wQ)[12 * i + k];
        double w2c[12];
        rigid_inv(v.c2w, w2c);
        ls_render_job j{};
        j.g = dir == 0 ? pr.Q : pr.P;  // a keyframe of one submap renders the other
        j.K = pr.K;
        for (int k = 0; k < 12; ++k) j.w2c[k] = (float)w2c[k];
        jobs.push_back(j);
        views.push_back(v);
      }
    }
  }
  first_view[pairs.size()] = (int)jobs.size();
  R = (int)jobs.size();
  ls_status st = batch_create_host(jobs.data(), R, &batch);
  if (st) return st;
  ls_batch_info info{};
  ls_batch_query(batch, 0, &info);
  M = info.items;
  P = info.pixels;
  T = info.tiles;
  pix_off.assign(R + 1, 0);
  ls_batch_offsets(batch, nullptr, pix_off.data(), nullptr);
  return LS_OK;
}

// Workspace layout for an instance capacity: the batch's device tables, the
// per-item / per-pixel / per-view arena, the two instance arrays and the bins
// workspace, each piece 256-byte aligned.
RegEngine::Layout RegEngine::layout(int64_t cap) const {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off = (off + std::max<size_t>(bytes, 4) + 255) & ~size_t(255); return o; };
  L.tables = take(batch_tables_bytes(batch));
  L.rec = take(48 * (size_t)std::max<int64_t>(M, 1));
  L.rad = take(4 * M);
  L.til = take(4 * M);
  L.aux = take(48 * (size_t)std::max<int64_t>(M, 1));
  L.rgb = take(12 * P);
  L.dep = take(4 * P);
  L.alp = take(4 * P);
  L.Tf = take(4 * P);
  L.nl = take(4 * P);
  L.trgb = take(12 * P);
  L.tdep = take(4 * P);
  L.grgb = take(12 * P);
  L.gdep = take(4 * P);
  L.scale = take(4 * R);
  L.loss = take(4 * R);
  L.pose = take(28 * R);
  L.pg = take(28 * R);
  L.m = take(28 * R);
  L.v = take(28 * R);
  L.opt = take(sizeof(ViewOpt) * R);
  L.range = take(8 * (size_t)T);
  L.count = take(16);
  L.sticky = take(8);
  L.expo = pairs[0].prm.exposure ? take(4 * (8 * (size_t)R + 2 * (size_t)batch->nblk_pix)) : 0;
  L.joint = pairs[0].prm.joint ? take(sizeof(JointView) * (size_t)R + sizeof(JointPair) * pairs.size()) : 0;
  L.zero_end = off;  // everything above starts at zero
  L.tile_of = take(4 * (size_t)cap);
  L.item = take(4 * (size_t)cap);
  ls_batch_info info{};
  ls_batch_query(batch, cap, &info);
  L.work = take(info.workspace_bytes);
  L.total = off;
  return L;
}

size_t RegEngine::workspace_bytes(int64_t cap) const { return layout(cap).total; }

// Device side: carves the caller's workspace, uploads the tables, copies the
// keyframe targets, clears the state and starts every view at identity.
ls_status RegEngine::bind(void* work, size_t work_bytes, int64_t cap, hipStream_t s) {
  const Layout L = layout(cap);
  if (!work || work_bytes < L.total || reinterpret_cast<uintptr_t>(work) % 256) return LS_ERR_CAPACITY;
  char* a = static_cast<char*>(work);
  ls_status st = batch_bind(batch, a + L.tables, L.rec - L.tables, s);
  if (st) return st;
  proj.rec = reinterpret_cast<float*>(a + L.rec);
  proj.radius = reinterpret_cast<int32_t*>(a + L.rad);
  proj.tiles = reinterpret_cast<int32_t*>(a + L.til);
  proj.aux = reinterpret_cast<float*>(a + L.aux);
  img.rgb = reinterpret_cast<float*>(a + L.rgb);
  img.depth = reinterpret_cast<float*>(a + L.dep);
  img.alpha = reinterpret_cast<float*>(a + L.alp);
  img.T_final = reinterpret_cast<float*>(a + L.Tf);
  img.n_last = reinterpret_cast<int32_t*>(a + L.nl);
  tgt_rgb = reinterpret_cast<float*>(a + L.trgb);
  tgt_depth = reinterpret_cast<float*>(a + L.tdep);
  g_rgb = reinterpret_cast<float*>(a + L.grgb);
  g_depth = reinterpret_cast<float*>(a + L.gdep);
  scale = reinterpret_cast<float*>(a + L.scale);
  loss = reinterpret_cast<float*>(a + L.loss);
  pose = reinterpret_cast<float*>(a + L.pose);
  pose_grad = reinterpret_cast<float*>(a + L.pg);
  adam_m = reinterpret_cast<float*>(a + L.m);
  adam_v = reinterpret_cast<float*>(a + L.v);
  opt = reinterpret_cast<ViewOpt*>(a + L.opt);
  range = reinterpret_cast<int32_t*>(a + L.range);
  count = reinterpret_cast<int32_t*>(a + L.count);
  sticky = reinterpret_cast<int32_t*>(a + L.sticky);
  if (pairs[0].prm.exposure) {
    expo = reinterpret_cast<float*>(a + L.expo);
    expo_grad = expo + 2 * R;
    expo_m = expo + 4 * R;
    expo_v = expo + 6 * R;
    expo_part = expo + 8 * R;
  }
  bins.capacity = cap;
  bins.tile_of = reinterpret_cast<uint32_t*>(a + L.tile_of);
  bins.item = reinterpret_cast<int32_t*>(a + L.item);
  bins.range = range;
  bins.count = count;
  bins.work = a + L.work;
  capacity = cap;
  // the state (a = b = 0 and their moments included) and the bins workspace start at zero
  if (hipMemsetAsync(a + L.rec, 0, L.zero_end - L.rec, s) != hipSuccess ||
      hipMemsetAsync(a + L.work, 0, L.total - L.work, s) != hipSuccess)
    return LS_ERR_HIP;

  // targets: each view's measurements, laid out like the batch's images
  for (int r = 0; r < R; ++r) {
    const View& v = views[r];
    const ls_pair& pr = pairs[v.pair].pair;
    const int64_t hw = (int64_t)pr.K.width * pr.K.height;
    const float* srgb = (v.reverse ? pr.rgbQ : pr.rgbP) + 3 * hw * v.index;
    const float* sdep = (v.reverse ? pr.depthQ : pr.depthP) + hw * v.index;
    if (hipMemcpyAsync(tgt_rgb + 3 * pix_off[r], srgb, 12 * hw, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(tgt_depth + pix_off[r], sdep, 4 * hw, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return LS_ERR_HIP;
  }
  std::vector<ViewOpt> ho(R);
  for (int r = 0; r < R; ++r) {
    const ls_reg_params& pm = pairs[views[r].pair].prm;
    ho[r] = ViewOpt{pm.lr_rot, pm.lr_trans, 0, 1, 0.f, 0, 0.f, 0};
  }
  if (hipMemcpyAsync(opt, ho.data(), sizeof(ViewOpt) * R, hipMemcpyHostToDevice, s) != hipSuccess) return LS_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return LS_ERR_HIP;
  launch_pose_init(pose, adam_m, adam_v, opt, R, s);
  fused_l1 = fused_l1_allowed(pairs[0].prm);
  if (fused_l1 && (st = batch_valid_inv(batch, tgt_depth, scale, s))) return st;  // constant over the iterations
  joint_step = 0;
  joint_T.assign(7 * pairs.size(), 0.0);
  if (pairs[0].prm.joint) {  // T = identity, zero moments; each view's rotation as a unit quaternion
    jviews = reinterpret_cast<JointView*>(a + L.joint);
    jpairs = reinterpret_cast<JointPair*>(a + L.joint + sizeof(JointView) * (size_t)R);
    jviews_h.assign(R, JointView{});
    jpairs_h.assign(pairs.size(), JointPair{});
    for (int r = 0; r < R; ++r) {
      JointView& jv = jviews_h[r];
      for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) jv.Rc[i * 3 + j] = views[r].c2w[i * 4 + j];
        jv.tc[i] = views[r].c2w[i * 4 + 3];
      }
      quat_of_rot(jv.Rc, jv.qc);
      jv.pair = views[r].pair;
      jv.reverse = views[r].reverse ? 1 : 0;
    }
    for (size_t p = 0; p < pairs.size(); ++p) {
      jpairs_h[p].T[0] = 1.0;
      jpairs_h[p].first = first_view[p];
      jpairs_h[p].count = first_view[p + 1] - first_view[p];
    }
    if (hipMemcpyAsync(jviews, jviews_h.data(), sizeof(JointView) * R, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(jpairs, jpairs_h.data(), sizeof(JointPair) * pairs.size(), hipMemcpyHostToDevice, s) !=
            hipSuccess || hipStreamSynchronize(s) != hipSuccess)
      return LS_ERR_HIP;
    launch_joint_poses(jviews, R, jpairs, pose, s);
  }
  return hip_ok();
}

ls_status RegEngine::coverage(hipStream_t s, std::vector<float>& cov) {
  ls_status st;
  if ((st = ls_render_fwd(batch, &proj, &bins, nullptr, &img, s))) return st;
  launch_view_coverage(batch->jobs_d, batch->pblk_off_d, R, batch->nblk_pix, img.alpha, tgt_depth, g_rgb, loss, s);
  cov.resize(R);
  if (hipMemcpyAsync(cov.data(), loss, 4 * (size_t)R, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return LS_ERR_HIP;
  return hip_ok();
}

// Bins every view at its current pose and reads the instance count back:
// {kept, overflow, required, 0}.
ls_status RegEngine::measure(hipStream_t s, int32_t* hc) {
  ls_status st;
  if ((st = ls_project(batch, pose, &proj, s)) || (st = ls_bin_sort(batch, &proj, &bins, s))) return st;
  if (hipMemcpyAsync(hc, count, 16, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return LS_ERR_HIP;
  return LS_OK;
}

ls_status RegEngine::step(hipStream_t s) {
  ls_status st;
  const ls_image_grad up{g_rgb, g_depth, nullptr, scale};
  // views frozen by the early exit are not rendered (the final forward
  // renders every view)
  if ((st = project_views(batch, pose, &proj, opt, s)) || (st = ls_bin_sort(batch, &proj, &bins, s))) return st;
  if ((st = ls_render_fwd(batch, &proj, &bins, nullptr, &img, s))) return st;
  if (fused_l1)  // the backward forms the L1 gradient itself; no per-iteration loss value
    st = render_bwd_pose_l1(batch, pose, &proj, &bins, &img, tgt_rgb, tgt_depth, scale, s);
  else if (!(st = view_loss(s)))
    st = ls_render_bwd_tiles(batch, pose, &proj, &bins, nullptr, &img, &up, LS_BWD_POSE_ONLY, s);
  if (st) return st;
  // pose gradients, Adam steps and the sticky overflow flag in one launch
  const ls_reg_params& pm = pairs[0].prm;
  const PoseAdamArgs a{pose, pose_grad, adam_m, adam_v, opt, loss, pm.beta1, pm.beta2, pm.adam_eps, pm.exit_rel_tol,
                       pm.exit_patience, pm.exit_mode, expo, expo_grad, expo_m, expo_v, pm.lr_exposure};
  if ((st = pose_reduce_adam(batch, &bins, a, count, sticky, s))) return st;
  return hip_ok();
}

// One joint iteration: the views' pose gradients from the pose-only
// backward, then on the device every pair's Adam step of T (chained through
// the Jacobian of T -> Delta) and the views' new corrections.  No host
// synchronisation.
ls_status RegEngine::step_joint(hipStream_t s) {
  ls_status st;
  const ls_image_grad up{g_rgb, g_depth, nullptr, scale};
  if ((st = ls_project(batch, pose, &proj, s)) || (st = ls_bin_sort(batch, &proj, &bins, s))) return st;
  launch_or_flag(count, sticky, s);
  if ((st = ls_render_fwd(batch, &proj, &bins, nullptr, &img, s)) || (st = view_loss(s)) ||
      (st = ls_render_bwd_tiles(batch, pose, &proj, &bins, nullptr, &img, &up, LS_BWD_POSE_ONLY, s)) ||
      (st = ls_render_bwd_project(batch, pose, &proj, &bins, nullptr, pose_grad, LS_BWD_POSE_ONLY, s)))
    return st;
  ++joint_step;
  const ls_reg_params& pm = pairs[0].prm;
  const JointAdam ja{pm.lr_rot, pm.lr_trans, pm.beta1, pm.beta2, pm.adam_eps,
                     1.0 / (1.0 - std::pow((double)pm.beta1, joint_step)),
                     1.0 / (1.0 - std::pow((double)pm.beta2, joint_step))};
  launch_joint_step(jviews, jpairs, (int)pairs.size(), pose_grad, pose, ja, s);
  return hip_ok();
}

ls_status RegEngine::read_joint_T(hipStream_t s) {
  std::vector<JointPair> h(pairs.size());
  if (hipMemcpyAsync(h.data(), jpairs, sizeof(JointPair) * pairs.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return LS_ERR_HIP;
  for (size_t p = 0; p < pairs.size(); ++p)
    for (int k = 0; k < 7; ++k) joint_T[7 * p + k] = h[p].T[k];
  return LS_OK;
}

// Residual of each view at its final pose: the unmasked colour + depth L1,
// whichever loss drove the optimisation (it rates how well the moved view
// explains its whole observation; a masked loss would rate a view that
// drifted off the other submap best).
ls_status RegEngine::final_forward(hipStream_t s) {
  ls_status st;
  if ((st = ls_project(batch, pose, &proj, s)) || (st = ls_bin_sort(batch, &proj, &bins, s))) return st;
  launch_or_flag(count, sticky, s);
  if ((st = ls_render_fwd(batch, &proj, &bins, nullptr, &img, s))) return st;
  if (expo)  // the residual sees the view's fitted exposure
    st = batch_loss_exposure(batch, 0, nullptr, &img, tgt_rgb, tgt_depth, expo, nullptr, nullptr, loss, g_rgb,
                             g_depth, scale, s);
  else
    st = ls_loss_l1(batch, &img, tgt_rgb, tgt_depth, loss, g_rgb, g_depth, scale, s);
  if (st) return st;
  return hip_ok();
}

ls_status RegEngine::view_loss(hipStream_t s) {
  const ls_reg_params& pm = pairs[0].prm;
  if (expo)
    return batch_loss_exposure(batch, pm.loss_kind, &pm.track, &img, tgt_rgb, tgt_depth, expo, expo_part, expo_grad,
                               loss, g_rgb, g_depth, scale, s);
  if (pm.loss_kind == 1)
    return ls_loss_tracking(batch, &img, tgt_rgb, tgt_depth, &pm.track, loss, nullptr, g_rgb, g_depth, scale, s);
  return ls_loss_l1(batch, &img, tgt_rgb, tgt_depth, loss, g_rgb, g_depth, scale, s);
}

ls_status RegEngine::readback(std::vector<float>& pose_h, std::vector<float>& loss_h, int32_t* overflow,
                              hipStream_t s) {
  pose_h.resize(7 * R);
  loss_h.resize(R);
  if (hipMemcpyAsync(pose_h.data(), pose, 28 * R, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(loss_h.data(), loss, 4 * R, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(overflow, sticky, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return LS_ERR_HIP;
  return LS_OK;
}

ls_status RegEngine::hip_ok() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LS_OK : LS_ERR_HIP;
}

ls_status RegEngine::fuse_pair(int p, const std::vector<float>& pose_h, const std::vector<float>& loss_h,
                               ls_reg_result* out) {
  const int v0 = first_view[p], v1 = first_view[p + 1];
  const int n = v1 - v0;
  const int vp = pairs[p].pair.vP, vall = vp + pairs[p].pair.vQ;
  if (out->per_view_T) std::fill(out->per_view_T, out->per_view_T + 12 * (size_t)vall, 0.f);
  if (out->residual) std::fill(out->residual, out->residual + vall, -1.f);  // views not kept
  std::vector<double> est(12 * n), res(n);
  std::vector<int32_t> rev(n);
  for (int k = 0; k < n; ++k) {
    const View& v = views[v0 + k];
    const int slot = (v.reverse ? vp : 0) + v.index;  // the keyframe's position among all of the pair's
    for (int q = 0; q < 7; ++q)
      if (!std::isfinite(pose_h[7 * (v0 + k) + q])) return LS_ERR_NONFINITE;
    if (!std::isfinite(loss_h[v0 + k])) return LS_ERR_NONFINITE;
    view_estimate(v.c2w, &pose_h[7 * (v0 + k)], &est[12 * k]);
    res[k] = loss_h[v0 + k];
    rev[k] = v.reverse ? 1 : 0;
    if (out->per_view_T)
      for (int q = 0; q < 12; ++q) out->per_view_T[12 * slot + q] = (float)est[12 * k + q];
    if (out->residual) out->residual[slot] = loss_h[v0 + k];
  }
  double T[12];
  const int st = fuse_estimates(est.data(), res.data(), rev.data(), n, T);
  if (st) return st;
  for (int q = 0; q < 12; ++q) out->T_PQ[q] = (float)T[q];
  return LS_OK;
}

ls_status RegEngine::read_exposure(int p, ls_reg_result* out, hipStream_t s) {
  if (!out->exposure || !expo) return LS_OK;
  const int v0 = first_view[p], n = first_view[p + 1] - v0;
  std::vector<float> h(2 * (size_t)n);
  if (hipMemcpyAsync(h.data(), expo + 2 * v0, 8 * (size_t)n, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return LS_ERR_HIP;
  const int vp = pairs[p].pair.vP;
  std::fill(out->exposure, out->exposure + 2 * (size_t)(vp + pairs[p].pair.vQ), 0.f);
  for (int k = 0; k < n; ++k) {
    const View& v = views[v0 + k];
    const int slot = (v.reverse ? vp : 0) + v.index;
    out->exposure[2 * slot] = h[2 * k];
    out->exposure[2 * slot + 1] = h[2 * k + 1];
  }
  return LS_OK;
}

bool fused_l1_allowed(const ls_reg_params& pm) {
  const char* e = std::getenv("LS_FUSED_L1");
  if (e && e[0] == '0' && e[1] == '\0') return false;
  return pm.loss_kind == 0 && !pm.exposure && !pm.joint && !(pm.exit_patience > 0 && pm.exit_mode == 0);
}

ls_status validate_pair(const ls_pair* p, const ls_reg_params* prm) {
  if (!p || !prm) return LS_ERR_INVALID;
  if (p->vP < 0 || p->vQ < 0 || p->vP + p->vQ < 1) return LS_ERR_INVALID;
  if (p->K.width <= 0 || p->K.height <= 0 || !(p->K.fx > 0) || !(p->K.fy > 0)) return LS_ERR_INVALID;
  if (p->vP > 0 && (!p->rgbP || !p->depthP || !p->c2wP || p->Q.n < 0)) return LS_ERR_INVALID;
  if (p->vQ > 0 && (!p->rgbQ || !p->depthQ || !p->c2wQ || p->P.n < 0)) return LS_ERR_INVALID;
  if (prm->iters < 1 || !(prm->lr_rot >= 0) || !(prm->lr_trans >= 0) || !(prm->beta1 >= 0 && prm->beta1 < 1) ||
      !(prm->beta2 >= 0 && prm->beta2 < 1) || !(prm->adam_eps > 0) || !(prm->exit_rel_tol >= 0) ||
      prm->exit_patience < 0 || prm->loss_kind < 0 || prm->loss_kind > 1 || prm->exposure < 0 ||
      prm->exposure > 1 || (prm->exposure && !(prm->lr_exposure >= 0.f && std::isfinite(prm->lr_exposure))) ||
      prm->joint < 0 || prm->joint > 1 || (prm->joint && (prm->exposure || prm->exit_patience > 0)) ||
      prm->top_k < 0 || prm->exit_mode < 0 || prm->exit_mode > 1)
    return LS_ERR_INVALID;
  if (prm->loss_kind == 1 && (!(prm->track.lambda_c >= 0.f && prm->track.lambda_c <= 1.f) ||
                              !std::isfinite(prm->track.inlier_k) || prm->track.alpha_power < 0 ||
                              prm->track.alpha_power > 8))
    return LS_ERR_INVALID;
  for (int i = 0; i < 12 * p->vP; ++i)
    if (!std::isfinite(p->c2wP[i])) return LS_ERR_NONFINITE;
  for (int i = 0; i < 12 * p->vQ; ++i)
    if (!std::isfinite(p->c2wQ[i])) return LS_ERR_NONFINITE;
  return LS_OK;
}

RegPair make_reg_pair(const ls_pair* p, const ls_reg_params* prm) {
  RegPair rp;
  rp.pair = *p;
  rp.prm = *prm;
  rp.c2wP.assign(p->c2wP ? p->c2wP : nullptr, p->c2wP ? p->c2wP + 12 * p->vP : nullptr);
  rp.c2wQ.assign(p->c2wQ ? p->c2wQ : nullptr, p->c2wQ ? p->c2wQ + 12 * p->vQ : nullptr);
  rp.pair.c2wP = nullptr;  // host copies above are used from here on
  rp.pair.c2wQ = nullptr;
  return rp;
}

}  // namespace ls

using namespace ls;

extern "C" {

ls_status ls_fuse_estimates(const double* est, const double* resid, const int32_t* reverse, int32_t n, double* out) {
  if (!est || !resid || !reverse || !out || n < 1) return LS_ERR_INVALID;
  return fuse_estimates(est, resid, reverse, n, out);
}

ls_status ls_register_workspace_size(const ls_pair* pair, const ls_reg_params* prm, int64_t capacity,
                                     size_t* bytes) {
  if (!bytes || capacity < 0 || capacity > INT32_MAX) return LS_ERR_INVALID;
  *bytes = 0;
  ls_status st = validate_pair(pair, prm);
  if (st) return st;
  RegEngine e;
  if ((st = e.prepare({make_reg_pair(pair, prm)}))) return st;
  *bytes = e.workspace_bytes(capacity);
  return LS_OK;
}

ls_status ls_register_pair(const ls_pair* pair, const ls_reg_params* prm, void* work, size_t work_bytes,
                           int64_t capacity, ls_reg_result* out, hipStream_t s) {
  if (!out) return LS_ERR_INVALID;
  out->status = LS_ERR_INVALID;
  out->iters_done = 0;
  out->instances_required = 0;
  out->workspace_required = 0;
  if (capacity < 0 || capacity > INT32_MAX) return LS_ERR_INVALID;
  ls_status st = validate_pair(pair, prm);
  out->status = st;
  if (st) return st;
  auto finish = [&](ls_status code) {
    out->status = code;
    return code;
  };
  RegPair rp = make_reg_pair(pair, prm);
  auto engine = std::make_unique<RegEngine>();
  if ((st = engine->prepare({rp}))) return finish(st);
  out->workspace_required = (int64_t)engine->workspace_bytes(capacity);
  if (!work || work_bytes < (size_t)out->workspace_required || reinterpret_cast<uintptr_t>(work) % 256)
    return finish(LS_ERR_CAPACITY);
  if ((st = engine->bind(work, work_bytes, capacity, s))) return finish(st);
  int32_t hc[4];
  if ((st = engine->measure(s, hc))) return finish(st);
  if (hc[1]) {  // the lists at the starting poses do not fit
    out->instances_required = hc[2];
    return finish(LS_ERR_CAPACITY);
  }
  const int k = prm->top_k;
  if (k > 0 && (pair->vP > k || pair->vQ > k)) {
    // top-k views per direction by co-visibility at the starting poses, then
    // a fresh engine over those views only (its workspace fits in the same one)
    std::vector<float> cov;
    if ((st = engine->coverage(s, cov))) return finish(st);
    for (int dir = 0; dir < 2; ++dir) {
      const int nv = dir == 0 ? pair->vP : pair->vQ, r0 = dir == 0 ? 0 : pair->vP;
      std::vector<int> order(nv);
      for (int i = 0; i < nv; ++i) order[i] = i;
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cov[r0 + a] > cov[r0 + b]; });
      order.resize(std::min(nv, k));
      std::sort(order.begin(), order.end());
      rp.sel[dir] = order;
    }
    engine = std::make_unique<RegEngine>();
    if ((st = engine->prepare({rp})) || (st = engine->bind(work, work_bytes, capacity, s)) ||
        (st = engine->measure(s, hc)))
      return finish(st);
    if (hc[1]) {
      out->instances_required = hc[2];
      return finish(LS_ERR_CAPACITY);
    }
  }
  RegEngine& e = *engine;
  int done = 0;
  constexpr int kCheckEvery = 16;  // early exit: poll the views' active flags this often
  if (prm->joint) {
    for (; done < prm->iters; ++done)
      if ((st = e.step_joint(s))) return finish(st);
    if ((st = e.read_joint_T(s))) return finish(st);  // the last step left the final T's corrections in pose
  }
  while (done < prm->iters) {
    const int k = prm->exit_patience > 0 ? std::min(kCheckEvery, prm->iters - done) : prm->iters - done;
    for (int it = 0; it < k; ++it)
      if ((st = e.step(s))) return finish(st);
    done += k;
    if (prm->exit_patience > 0 && done < prm->iters) {
      std::vector<ViewOpt> ho(e.R);
      if (hipMemcpyAsync(ho.data(), e.opt, sizeof(ViewOpt) * e.R, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return finish(LS_ERR_HIP);
      bool any = false;
      for (const ViewOpt& o : ho) any |= o.active != 0;
      if (!any) break;
    }
  }
  std::vector<float> ph, lh;
  int32_t ovf[2] = {0, 0};
  if ((st = e.final_forward(s)) || (st = e.readback(ph, lh, ovf, s))) return finish(st);
  if (ovf[0]) {  // the instance count outgrew the capacity during the optimisation
    out->instances_required = ovf[1];
    return finish(LS_ERR_CAPACITY);
  }
  st = e.fuse_pair(0, ph, lh, out);
  if (!st) st = e.read_exposure(0, out, s);
  if (!st && prm->joint) {  // the shared T is the estimate (no fusion)
    double T[12], Rm[9];
    rot_of_quat(&e.joint_T[0], Rm);
    for (int i = 0; i < 3; ++i) {
      for (int j = 0; j < 3; ++j) T[i * 4 + j] = Rm[i * 3 + j];
      T[i * 4 + 3] = e.joint_T[4 + i];
    }
    for (int q = 0; q < 12; ++q) out->T_PQ[q] = (float)T[q];
  }
  if (prm->joint) {
    out->iters_done = e.joint_step;
    return finish(st);
  }
  std::vector<ViewOpt> ho(e.R);
  if (hipMemcpyAsync(ho.data(), e.opt, sizeof(ViewOpt) * e.R, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return finish(LS_ERR_HIP);
  int steps = 0;
  for (const ViewOpt& o : ho) steps = std::max(steps, o.step);
  out->iters_done = steps;
  return finish(st);
}

}  // extern "C"

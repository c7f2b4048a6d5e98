// Per-view pose optimiser kernels for registration (Sec. 3.2): identity
// initialisation and an Adam step whose step counters live on the device, so
// an iteration can be captured once in a graph and replayed.
#include "kernels.h"

#include <algorithm>

namespace ls {

__global__ void k_pose_init(float* __restrict__ pose, float* __restrict__ m, float* __restrict__ v,
                            ViewOpt* __restrict__ opt, int R) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 7 * R) return;
  pose[i] = (i % 7) == 0 ? 1.f : 0.f;
  m[i] = 0.f;
  v[i] = 0.f;
  if (i < R) {
    opt[i].step = 0;
    opt[i].active = 1;
    opt[i].stall = 0;
    opt[i].best = 0.f;
    opt[i].resid = 0.f;
  }
}

// sticky[0] |= overflow; sticky[1] keeps the instance count required at the
// first overflow (the pose before any step taken on truncated lists).
__global__ void k_or_flag(const int32_t* __restrict__ count, int32_t* __restrict__ sticky) {
  if (threadIdx.x == 0) or_flag(count, sticky);
}

// ---------------------------------------------------------------- joint mode

__device__ __forceinline__ void quat_mul_d(const double* a, const double* b, double* o) {
  o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

// Delta (7 values: unit quaternion, translation) of one view under T.
__device__ void joint_delta_d(const double* T7, const JointView& jv, double* d7) {
  const double n = sqrt(T7[0] * T7[0] + T7[1] * T7[1] + T7[2] * T7[2] + T7[3] * T7[3]);
  const double w = T7[0] / n, x = T7[1] / n, y = T7[2] / n, z = T7[3] / n;
  const double q[4] = {w, x, y, z}, qi[4] = {w, -x, -y, -z};
  const double Rt[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z),     2 * (x * z + w * y),
                        2 * (x * y + w * z),     1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                        2 * (x * z - w * y),     2 * (y * z + w * x),     1 - 2 * (x * x + y * y)};
  const double qci[4] = {jv.qc[0], -jv.qc[1], -jv.qc[2], -jv.qc[3]};
  double tmp[4];
  quat_mul_d(qci, jv.reverse ? q : qi, tmp);
  quat_mul_d(tmp, jv.qc, d7);
  double v[3];
  for (int i = 0; i < 3; ++i) {
    if (jv.reverse)  // Rt tc + t - tc
      v[i] = Rt[i * 3 + 0] * jv.tc[0] + Rt[i * 3 + 1] * jv.tc[1] + Rt[i * 3 + 2] * jv.tc[2] + T7[4 + i] - jv.tc[i];
    else  // Rt^T (tc - t) - tc
      v[i] = Rt[0 * 3 + i] * (jv.tc[0] - T7[4]) + Rt[1 * 3 + i] * (jv.tc[1] - T7[5]) +
             Rt[2 * 3 + i] * (jv.tc[2] - T7[6]) - jv.tc[i];
  }
  for (int i = 0; i < 3; ++i) d7[4 + i] = jv.Rc[0 * 3 + i] * v[0] + jv.Rc[1 * 3 + i] * v[1] + jv.Rc[2 * 3 + i] * v[2];
}

__global__ void k_joint_poses(const JointView* __restrict__ views, int R, const JointPair* __restrict__ pairs,
                              float* __restrict__ pose) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  double d[7];
  joint_delta_d(pairs[views[r].pair].T, views[r], d);
  for (int k = 0; k < 7; ++k) pose[7 * r + k] = (float)d[k];
}

constexpr int kJointChunk = 32;  // views per round of the gradient (kJointChunk x 7 tasks <= block)

// One block per pair.  Rounds of up to kJointChunk views: task (view, k)
// forms sum_i dDelta_i/dT_k g_i by central differences (h = 1e-7); threads
// 0..6 add the round's tasks of their k in view order.  Thread k then takes
// the Adam step of T_k; the pose gradients are cleared and each view gets its
// correction under the new T.
__global__ __launch_bounds__(256) void k_joint_step(const JointView* __restrict__ views, JointPair* __restrict__ pairs,
                                                    float* __restrict__ pose_grad, float* __restrict__ pose,
                                                    JointAdam a) {
  __shared__ double part[kJointChunk][7];
  __shared__ double Tn[7];
  JointPair& P = pairs[blockIdx.x];
  const int first = P.first, count = P.count;
  double T[7];
  for (int k = 0; k < 7; ++k) T[k] = P.T[k];
  double g = 0.0;  // thread k < 7: dL/dT_k
  for (int v0 = 0; v0 < count; v0 += kJointChunk) {
    const int nv = min(kJointChunk, count - v0);
    for (int t = threadIdx.x; t < 7 * nv; t += blockDim.x) {
      const int v = t / 7, k = t - 7 * v, r = first + v0 + v;
      constexpr double h = 1e-7;
      double Tp[7], Tm[7], dp[7], dm[7];
      for (int i = 0; i < 7; ++i) Tp[i] = Tm[i] = T[i];
      Tp[k] += h;
      Tm[k] -= h;
      joint_delta_d(Tp, views[r], dp);
      joint_delta_d(Tm, views[r], dm);
      double c = 0.0;
      for (int i = 0; i < 7; ++i) c += (dp[i] - dm[i]) / (2 * h) * (double)pose_grad[7 * r + i];
      part[v][k] = c;
    }
    __syncthreads();
    if (threadIdx.x < 7)
      for (int v = 0; v < nv; ++v) g += part[v][threadIdx.x];
    __syncthreads();
  }
  if (threadIdx.x < 7) {
    const int k = threadIdx.x;
    double m = P.m[k], v = P.v[k];
    m = a.beta1 * m + (1.0 - a.beta1) * g;
    v = a.beta2 * v + (1.0 - a.beta2) * g * g;
    const double lr = k < 4 ? a.lr_rot : a.lr_trans;
    const double t = T[k] - lr * (m * a.bc1) / (sqrt(v * a.bc2) + a.eps);
    P.m[k] = m;
    P.v[k] = v;
    P.T[k] = t;
    Tn[k] = t;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 7 * count; i += blockDim.x) pose_grad[7 * first + i] = 0.f;
  for (int v = threadIdx.x; v < count; v += blockDim.x) {
    const int r = first + v;
    double d[7];
    joint_delta_d(Tn, views[r], d);
    for (int k = 0; k < 7; ++k) pose[7 * r + k] = (float)d[k];
  }
}

void launch_joint_poses(const JointView* views, int R, const JointPair* pairs, float* pose, hipStream_t s) {
  if (R > 0) hipLaunchKernelGGL(k_joint_poses, dim3((R + 63) / 64), dim3(64), 0, s, views, R, pairs, pose);
}

void launch_joint_step(const JointView* views, JointPair* pairs, int npairs, float* pose_grad, float* pose,
                       const JointAdam& a, hipStream_t s) {
  if (npairs > 0) hipLaunchKernelGGL(k_joint_step, dim3(npairs), dim3(256), 0, s, views, pairs, pose_grad, pose, a);
}

void launch_pose_init(float* pose, float* m, float* v, ViewOpt* opt, int R, hipStream_t s) {
  const int n = 7 * R;
  hipLaunchKernelGGL(k_pose_init, dim3((n + 255) / 256), dim3(256), 0, s, pose, m, v, opt, R);
}

// View co-visibility for the top-k selection of registration views: per
// 1024-pixel block, the pixels with a measured depth and, of those, the ones
// the other submap covers (rendered alpha >= 0.5); then per render, in a
// fixed order, covered / measured (0 when nothing is measured).
__global__ __launch_bounds__(256) void k_view_cover(const JobDev* __restrict__ jobs, const int32_t* __restrict__ pblk_off,
                                                    int R, const float* __restrict__ alpha,
                                                    const float* __restrict__ tgt_depth, float* __restrict__ part) {
  const int r = find_segment<int32_t>(pblk_off, R, (int32_t)blockIdx.x);
  const JobDev& J = jobs[r];
  const int64_t hw = (int64_t)J.W * J.H;
  const int64_t b0 = (int64_t)(blockIdx.x - pblk_off[r]) * 1024;
  float valid = 0.f, cover = 0.f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t p = b0 + (int64_t)k * 256 + threadIdx.x;
    if (p < hw && tgt_depth[J.pix_off + p] > 0.f) {
      valid += 1.f;
      cover += alpha[J.pix_off + p] >= 0.5f ? 1.f : 0.f;
    }
  }
  valid = wave_sum(valid);
  cover = wave_sum(cover);
  __shared__ float ws[2][4];
  if ((threadIdx.x & 63) == 0) {
    ws[0][threadIdx.x >> 6] = valid;
    ws[1][threadIdx.x >> 6] = cover;
  }
  __syncthreads();
  if (threadIdx.x < 2) part[2 * blockIdx.x + threadIdx.x] = (ws[threadIdx.x][0] + ws[threadIdx.x][1]) +
                                                             (ws[threadIdx.x][2] + ws[threadIdx.x][3]);
}

__global__ void k_view_cover_reduce(const int32_t* __restrict__ pblk_off, int R, const float* __restrict__ part,
                                    float* __restrict__ coverage) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  float v = 0.f, c = 0.f;
  for (int b = pblk_off[r]; b < pblk_off[r + 1]; ++b) {
    v += part[2 * b];
    c += part[2 * b + 1];
  }
  coverage[r] = v > 0.f ? c / v : 0.f;
}

void launch_view_coverage(const JobDev* jobs, const int32_t* pblk_off, int R, int npblk, const float* alpha,
                          const float* tgt_depth, float* part, float* coverage, hipStream_t s) {
  if (npblk > 0)
    hipLaunchKernelGGL(k_view_cover, dim3(npblk), dim3(256), 0, s, jobs, pblk_off, R, alpha, tgt_depth, part);
  hipLaunchKernelGGL(k_view_cover_reduce, dim3((R + 63) / 64), dim3(64), 0, s, pblk_off, R, (const float*)part,
                     coverage);
}

void launch_or_flag(const int32_t* count, int32_t* sticky, hipStream_t s) {
  hipLaunchKernelGGL(k_or_flag, dim3(1), dim3(64), 0, s, count, sticky);
}

}  // namespace ls

namespace ls {

// New epoch's per-view state from the previous epoch's: views that continue
// (map[r] >= 0) keep pose, Adam moments and step; new views start at the
// identity with the settings in init_opt.
__global__ void k_state_remap(const float* __restrict__ opose, const float* __restrict__ om,
                              const float* __restrict__ ov, const ViewOpt* __restrict__ oopt,
                              float* __restrict__ npose, float* __restrict__ nm, float* __restrict__ nv,
                              float* __restrict__ ngrad, ViewOpt* __restrict__ nopt, const int32_t* __restrict__ map,
                              const ViewOpt* __restrict__ init_opt, int R, ExpoState oe, ExpoState ne) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int o = map[r];
  for (int k = 0; k < 7; ++k) {
    npose[7 * r + k] = o >= 0 ? opose[7 * o + k] : (k == 0 ? 1.f : 0.f);
    nm[7 * r + k] = o >= 0 ? om[7 * o + k] : 0.f;
    nv[7 * r + k] = o >= 0 ? ov[7 * o + k] : 0.f;
    ngrad[7 * r + k] = 0.f;  // the backward accumulates into it; Adam consumes it
  }
  if (ne.expo) {  // exposure coefficients (a, b) and their moments; new views start at 0
    for (int k = 0; k < 2; ++k) {
      ne.expo[2 * r + k] = o >= 0 ? oe.expo[2 * o + k] : 0.f;
      ne.m[2 * r + k] = o >= 0 ? oe.m[2 * o + k] : 0.f;
      ne.v[2 * r + k] = o >= 0 ? oe.v[2 * o + k] : 0.f;
      ne.grad[2 * r + k] = 0.f;
    }
  }
  nopt[r] = o >= 0 ? oopt[o] : init_opt[r];
}

__global__ void k_all_finite(const float* __restrict__ a, int64_t n, int32_t* __restrict__ bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(a[i])) { *bad = 1; return; }
}

void launch_state_remap(const float* opose, const float* om, const float* ov, const ViewOpt* oopt, float* npose,
                        float* nm, float* nv, float* ngrad, ViewOpt* nopt, const int32_t* map, const ViewOpt* init_opt,
                        int R, hipStream_t s, ExpoState oe, ExpoState ne) {
  if (R > 0)
    hipLaunchKernelGGL(k_state_remap, dim3((R + 127) / 128), dim3(128), 0, s, opose, om, ov, oopt, npose, nm, nv,
                       ngrad, nopt, map, init_opt, R, oe, ne);
}

void launch_all_finite(const float* a, int64_t n, int32_t* bad, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_all_finite, dim3((unsigned)blocks), dim3(256), 0, s, a, n, bad);
}

}  // namespace ls

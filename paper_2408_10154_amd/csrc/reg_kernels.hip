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

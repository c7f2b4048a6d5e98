// Globally consistent map adjustment (Sec. 3.3, Eq. 8): after pose-graph
// optimisation every submap's Gaussian means, Gaussian orientations and
// keyframe poses are moved by that submap's rigid correction T_c = [R_c|t_c],
// in place, for many submaps per launch.  Means map to R_c mu + t_c; the
// covariance R_c Sigma R_c^T is R(q_c q) S^2 R(q_c q)^T, so only the
// quaternion changes (scales, opacity and colour stay); camera-to-world
// keyframe poses are left-multiplied, T_j <- T_c T_j.
#include <algorithm>
#include <cmath>

#include "kernels.h"

namespace ls {

constexpr int kAdjustPerLaunch = 32;  // submaps per launch (the table travels as a kernel argument)

struct AdjustDesc {
  float* mean;  // [3][n]
  float* quat;  // [4][n] (w, x, y, z)
  float* c2w;   // [n_poses][12] row-major 3x4, or null
  int32_t n, n_poses;
  float R[9], t[3], q[4];  // R_c (row-major), t_c, and the unit quaternion of R_c
};

struct AdjustArgs {
  AdjustDesc d[kAdjustPerLaunch];
  int32_t blk_off[kAdjustPerLaunch + 1];
  int32_t count;
};
static_assert(sizeof(AdjustArgs) <= 4096, "kernel arguments are limited to 4 KB");

// Each thread moves kAdjustItems Gaussians of one submap (block-strided, so
// every load instruction of a wave stays coalesced; all loads are issued
// before the first store) and, in the submap's first blocks, one keyframe
// pose.  Blocks never straddle submaps.
constexpr int kAdjustItems = 4;

__global__ __launch_bounds__(256) void k_adjust(AdjustArgs a) {
  const int s = find_segment<int32_t>(a.blk_off, a.count, (int32_t)blockIdx.x);
  const AdjustDesc& D = a.d[s];
  const int64_t blk = blockIdx.x - a.blk_off[s];
  const int64_t n = D.n;
  const float* R = D.R;
  float v[kAdjustItems][7];
#pragma unroll
  for (int j = 0; j < kAdjustItems; ++j) {
    const int64_t i = (blk * kAdjustItems + j) * kBlock + threadIdx.x;
    if (i < n) {
      v[j][0] = D.mean[i];
      v[j][1] = D.mean[n + i];
      v[j][2] = D.mean[2 * n + i];
      v[j][3] = D.quat[i];
      v[j][4] = D.quat[n + i];
      v[j][5] = D.quat[2 * n + i];
      v[j][6] = D.quat[3 * n + i];
    }
  }
  const float w1 = D.q[0], x1 = D.q[1], y1 = D.q[2], z1 = D.q[3];
#pragma unroll
  for (int j = 0; j < kAdjustItems; ++j) {
    const int64_t i = (blk * kAdjustItems + j) * kBlock + threadIdx.x;
    if (i < n) {
      const float x = v[j][0], y = v[j][1], z = v[j][2];
      D.mean[i] = R[0] * x + R[1] * y + R[2] * z + D.t[0];
      D.mean[n + i] = R[3] * x + R[4] * y + R[5] * z + D.t[1];
      D.mean[2 * n + i] = R[6] * x + R[7] * y + R[8] * z + D.t[2];
      const float w2 = v[j][3], x2 = v[j][4], y2 = v[j][5], z2 = v[j][6];
      // Hamilton product q_c q: R(q_c q) = R(q_c) R(q)
      D.quat[i] = w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2;
      D.quat[n + i] = w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2;
      D.quat[2 * n + i] = w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2;
      D.quat[3 * n + i] = w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2;
    }
  }
  const int64_t ip = blk * kBlock + threadIdx.x;
  if (D.c2w && ip < D.n_poses) {
    float* P = D.c2w + 12 * ip;
    float o[12];
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 4; ++c)
        o[r * 4 + c] = R[r * 3 + 0] * P[c] + R[r * 3 + 1] * P[4 + c] + R[r * 3 + 2] * P[8 + c];
      o[r * 4 + 3] += D.t[r];
    }
    for (int k = 0; k < 12; ++k) P[k] = o[k];
  }
}

// Unit quaternion (w, x, y, z) of a rotation matrix (row-major), by the
// largest of the four diagonal combinations (Shepperd's method).
static void rotation_to_quat(const double* R, double* q) {
  const double tr = R[0] + R[4] + R[8];
  if (tr > 0.0) {
    const double S = std::sqrt(tr + 1.0) * 2.0;
    q[0] = 0.25 * S;
    q[1] = (R[7] - R[5]) / S;
    q[2] = (R[2] - R[6]) / S;
    q[3] = (R[3] - R[1]) / S;
  } else if (R[0] > R[4] && R[0] > R[8]) {
    const double S = std::sqrt(1.0 + R[0] - R[4] - R[8]) * 2.0;
    q[0] = (R[7] - R[5]) / S;
    q[1] = 0.25 * S;
    q[2] = (R[1] + R[3]) / S;
    q[3] = (R[2] + R[6]) / S;
  } else if (R[4] > R[8]) {
    const double S = std::sqrt(1.0 + R[4] - R[0] - R[8]) * 2.0;
    q[0] = (R[2] - R[6]) / S;
    q[1] = (R[1] + R[3]) / S;
    q[2] = 0.25 * S;
    q[3] = (R[5] + R[7]) / S;
  } else {
    const double S = std::sqrt(1.0 + R[8] - R[0] - R[4]) * 2.0;
    q[0] = (R[3] - R[1]) / S;
    q[1] = (R[2] + R[6]) / S;
    q[2] = (R[5] + R[7]) / S;
    q[3] = 0.25 * S;
  }
  const double nrm = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; ++k) q[k] /= nrm;
}

int launch_adjust_submaps(const ls_submap_adjust* subs, int count, hipStream_t s) {
  for (int c0 = 0; c0 < count; c0 += kAdjustPerLaunch) {
    AdjustArgs a{};
    a.count = std::min(kAdjustPerLaunch, count - c0);
    a.blk_off[0] = 0;
    for (int k = 0; k < a.count; ++k) {
      const ls_submap_adjust& u = subs[c0 + k];
      AdjustDesc& d = a.d[k];
      d.mean = u.mean;
      d.quat = u.quat;
      d.c2w = u.c2w;
      d.n = u.n;
      d.n_poses = u.c2w ? u.n_poses : 0;
      double Rd[9], q[4];
      for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) {
          d.R[r * 3 + c] = u.T[r * 4 + c];
          Rd[r * 3 + c] = u.T[r * 4 + c];
        }
        d.t[r] = u.T[r * 4 + 3];
      }
      rotation_to_quat(Rd, q);
      for (int k2 = 0; k2 < 4; ++k2) d.q[k2] = (float)q[k2];
      const int64_t per = (int64_t)kBlock * kAdjustItems;
      const int64_t nb = std::max<int64_t>(std::max<int64_t>((d.n + per - 1) / per, (d.n_poses + kBlock - 1) / kBlock), 1);
      a.blk_off[k + 1] = a.blk_off[k] + (int32_t)nb;
    }
    for (int k = a.count + 1; k <= kAdjustPerLaunch; ++k) a.blk_off[k] = a.blk_off[a.count];
    hipLaunchKernelGGL(k_adjust, dim3(a.blk_off[a.count]), dim3(kBlock), 0, s, a);
  }
  return 0;
}

}  // namespace ls

// EWA projection of 3D Gaussians (forward) and its backward, gfx950.
//
// One thread per item; blocks never straddle two renders (each render owns
// ceil(n / 256) blocks starting at blk_off), so the per-render pose-gradient
// partials of the backward can be reduced in a fixed order.
#include "kernels.h"

namespace ls {

__global__ __launch_bounds__(256) void k_project(const JobDev* __restrict__ jobs, const int32_t* __restrict__ blk_off,
                                                 int R, const float* __restrict__ pose, float4* __restrict__ rec,
                                                 int32_t* __restrict__ radius_out, int32_t* __restrict__ tiles_out,
                                                 float4* __restrict__ aux, const ViewOpt* __restrict__ live) {
  const int r = find_segment<int32_t>(blk_off, R, (int32_t)blockIdx.x);
  const JobDev& J = jobs[r];
  const int g = (blockIdx.x - J.blk_off) * 256 + threadIdx.x;
  if (g >= J.n) return;
  const int64_t item = J.item_off + g;
  const int n = J.n;

  float W[9], t[3];
  camera_of(J, pose ? pose + 7 * r : nullptr, W, t);

  const float mx = J.mean[g], my = J.mean[n + g], mz = J.mean[2 * n + g];
  const float px = W[0] * mx + W[1] * my + W[2] * mz + t[0];
  const float py = W[3] * mx + W[4] * my + W[5] * mz + t[1];
  const float pz = W[6] * mx + W[7] * my + W[8] * mz + t[2];

  float4* out = rec + item * 3;
  int rad = 0, ntiles = 0;
  float4 o0 = make_float4(0.f, 0.f, 0.f, 0.f), o1 = o0, o2 = o0;
  float4 x0 = make_float4(px, py, pz, 0.f), x1 = make_float4(0.f, 0.f, 0.f, 0.f), x2 = x1;
  if (pz > LS_NEAR_Z && (!live || live[r].active)) {
    // Sigma = M M^T, M = R(q) diag(s)
    float Rq[9];
    quat_to_rot(J.quat[g], J.quat[n + g], J.quat[2 * n + g], J.quat[3 * n + g], Rq);
    const float s0 = __expf(J.log_scale[g]), s1 = __expf(J.log_scale[n + g]), s2 = __expf(J.log_scale[2 * n + g]);
    float M[9];
    for (int i = 0; i < 3; ++i) { M[i * 3 + 0] = Rq[i * 3 + 0] * s0; M[i * 3 + 1] = Rq[i * 3 + 1] * s1; M[i * 3 + 2] = Rq[i * 3 + 2] * s2; }
    // V = W M ; Sigma_c = V V^T
    float V[9];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) V[i * 3 + k] = W[i * 3 + 0] * M[0 * 3 + k] + W[i * 3 + 1] * M[1 * 3 + k] + W[i * 3 + 2] * M[2 * 3 + k];
    // J rows: J0 = (fx/z, 0, -fx x/z^2), J1 = (0, fy/z, -fy y/z^2); U = J V (2x3)
    const float iz = 1.0f / pz;
    const float j00 = J.fx * iz, j02 = -J.fx * px * iz * iz;
    const float j11 = J.fy * iz, j12 = -J.fy * py * iz * iz;
    float U0[3], U1[3];
    for (int k = 0; k < 3; ++k) { U0[k] = j00 * V[k] + j02 * V[6 + k]; U1[k] = j11 * V[3 + k] + j12 * V[6 + k]; }
    // camera-space covariance V V^T (kept for the pose backward)
    const float sxx = V[0] * V[0] + V[1] * V[1] + V[2] * V[2], sxy = V[0] * V[3] + V[1] * V[4] + V[2] * V[5];
    const float sxz = V[0] * V[6] + V[1] * V[7] + V[2] * V[8], syy = V[3] * V[3] + V[4] * V[4] + V[5] * V[5];
    const float syz = V[3] * V[6] + V[4] * V[7] + V[5] * V[8], szz = V[6] * V[6] + V[7] * V[7] + V[8] * V[8];
    x0.w = sxx;
    x1 = make_float4(sxy, sxz, syy, syz);
    x2 = make_float4(szz, 0.f, 0.f, 0.f);
    const float a = U0[0] * U0[0] + U0[1] * U0[1] + U0[2] * U0[2] + LS_EPS_2D;
    const float b = U0[0] * U1[0] + U0[1] * U1[1] + U0[2] * U1[2];
    const float c = U1[0] * U1[0] + U1[1] * U1[1] + U1[2] * U1[2] + LS_EPS_2D;
    const float det = a * c - b * b;
    if (det > 0.f) {
      const float mid = 0.5f * (a + c);
      const float hd = 0.5f * (a - c);
      const float lam = mid + sqrtf(hd * hd + b * b);
      rad = (int)ceilf(3.0f * sqrtf(lam));
      const float u = J.fx * px * iz + J.cx;
      const float v = J.fy * py * iz + J.cy;
      const Rect rc = tile_rect(u, v, rad, J.TX, J.TY);
      ntiles = max(rc.x1 - rc.x0, 0) * max(rc.y1 - rc.y0, 0);
      if (ntiles == 0) rad = 0;
      if (rad > 0) {
        const float idet = 1.0f / det;
        const float op = 1.0f / (1.0f + __expf(-J.opac[g]));
        o0 = make_float4(u, v, c * idet, -b * idet);
        o1 = make_float4(a * idet, op, pz, 0.f);
        o2 = make_float4(J.rgb[g], J.rgb[n + g], J.rgb[2 * n + g], 0.f);
      }
    }
  }
  if (rad == 0) ntiles = 0;
  radius_out[item] = rad;
  tiles_out[item] = ntiles;
  if (rad == 0) return;  // nothing reads a culled item's record or aux (most items of a registration view)
  out[0] = o0;
  out[1] = o1;
  out[2] = o2;
  if (aux) {
    aux[item * 3 + 0] = x0;
    aux[item * 3 + 1] = x1;
    aux[item * 3 + 2] = x2;
  }
}

// d R(q/|q|) / d(q) contracted with G (row-major dL/dR): returns dL/dq for the
// unnormalised quaternion.
__device__ __forceinline__ void rot_backward(float w, float x, float y, float z, const float* G, float* dq) {
  const float n2 = w * w + x * x + y * y + z * z;
  const float inv = rsqrtf(n2);
  const float qw = w * inv, qx = x * inv, qy = y * inv, qz = z * inv;
  // dL/dq_hat
  const float gw = 2.f * (-qz * G[1] + qy * G[2] + qz * G[3] - qx * G[5] - qy * G[6] + qx * G[7]);
  const float gx = 2.f * (qy * G[1] + qz * G[2] + qy * G[3] - 2.f * qx * G[4] - qw * G[5] + qz * G[6] + qw * G[7] -
                          2.f * qx * G[8]);
  const float gy = 2.f * (-2.f * qy * G[0] + qx * G[1] + qw * G[2] + qx * G[3] + qz * G[5] - qw * G[6] + qz * G[7] -
                          2.f * qy * G[8]);
  const float gz = 2.f * (-2.f * qz * G[0] - qw * G[1] + qx * G[2] + qw * G[3] - 2.f * qz * G[4] + qy * G[5] +
                          qx * G[6] + qy * G[7]);
  const float dot = qw * gw + qx * gx + qy * gy + qz * gz;
  dq[0] = (gw - qw * dot) * inv;
  dq[1] = (gx - qx * dot) * inv;
  dq[2] = (gy - qy * dot) * inv;
  dq[3] = (gz - qz * dot) * inv;
}

__device__ __forceinline__ void store_grad(float* p, float v, bool shared) {
  if (shared) atomic_add_f32(p, v); else *p += v;
}

// Chains image-space gradients (du dv dA dB dC dop dz dr dg db, accumulated
// per item over its tiles) to the Gaussian parameters and to the per-render
// pose correction, and clears the accumulator for the next backward.
template <bool kAdam>
__global__ __launch_bounds__(256) void k_project_bwd(const JobDev* __restrict__ jobs, const int32_t* __restrict__ blk_off,
                                                     int R, const float* __restrict__ pose,
                                                     const int32_t* __restrict__ radius, const float4* __restrict__ aux,
                                                     float* __restrict__ g2d, const GradDev* __restrict__ grads,
                                                     int want_gauss, float* __restrict__ pose_part, int want_pose,
                                                     GaussAdamArgs adam) {
  const int r = find_segment<int32_t>(blk_off, R, (int32_t)blockIdx.x);
  const JobDev& J = jobs[r];
  const int g = (blockIdx.x - J.blk_off) * 256 + threadIdx.x;
  const int n = J.n;
  float acc[kPoseAcc];
#pragma unroll
  for (int k = 0; k < kPoseAcc; ++k) acc[k] = 0.f;

  // fused Adam: the 14 gradient values of this Gaussian (mean 0-2,
  // log_scale 3-5, quat 6-9, opacity 10, rgb 11-13; zero for a culled one,
  // whose moments still decay and which still moves) are gathered first and
  // stepped together after the chain, every load before any store
  float* const params[5] = {const_cast<float*>(J.mean), const_cast<float*>(J.log_scale), const_cast<float*>(J.quat),
                            const_cast<float*>(J.opac), const_cast<float*>(J.rgb)};
  constexpr int kSlot0[5] = {0, 3, 6, 10, 11};
  float gv[14];
#pragma unroll
  for (int j = 0; j < 14; ++j) gv[j] = 0.f;

  const int64_t item = J.item_off + g;
  if (g < n && radius[item] > 0) {
    float* gp = g2d + item * kGrad2D;
    float gi[kGrad2D];
#pragma unroll
    for (int q = 0; q < kGrad2D; ++q) {
      gi[q] = gp[q];
      gp[q] = 0.f;  // leave the accumulator cleared for the next backward
    }
    const float4 a0 = aux[item * 3 + 0], a1 = aux[item * 3 + 1], a2 = aux[item * 3 + 2];
    const float p[3] = {a0.x, a0.y, a0.z};
    const float s6[6] = {a0.w, a1.x, a1.y, a1.z, a1.w, a2.x};
    float Sc[9];
    sym3(s6, Sc);
    const float g6[6] = {gi[0], gi[1], gi[2], gi[3], gi[4], gi[6]};
    float dp[3], G[9];
    camera_space_grads(p, Sc, J.fx, J.fy, g6, dp, G);
    const float* pr = pose ? pose + 7 * r : nullptr;

    if (want_gauss) {
      float W[9], t[3];
      camera_of(J, pr, W, t);
      const GradDev GD = kAdam ? GradDev{params[0], params[1], params[2], params[3], params[4], 0, 0} : grads[r];
      const bool sh = GD.shared != 0;
      // gradient of component k of array q: accumulated, or kept for the Adam step
      auto emit = [&](int q, int k, float* base, float val) {
        if (kAdam) gv[kSlot0[q] + k] = val;
        else store_grad(base + (int64_t)k * n + g, val, sh);
      };
      if (GD.mean) {
        for (int k = 0; k < 3; ++k)
          emit(0, k, GD.mean, W[0 * 3 + k] * dp[0] + W[1 * 3 + k] * dp[1] + W[2 * 3 + k] * dp[2]);
      }
      if (GD.log_scale || GD.quat) {
        const float qw0 = J.quat[g], qx0 = J.quat[n + g], qy0 = J.quat[2 * n + g], qz0 = J.quat[3 * n + g];
        float Rq[9];
        quat_to_rot(qw0, qx0, qy0, qz0, Rq);
        const float s[3] = {__expf(J.log_scale[g]), __expf(J.log_scale[n + g]), __expf(J.log_scale[2 * n + g])};
        float M[9];
        for (int i = 0; i < 3; ++i)
          for (int k = 0; k < 3; ++k) M[i * 3 + k] = Rq[i * 3 + k] * s[k];
        // dL/dSigma = W^T G W ; dL/dM = 2 dL/dSigma M
        float GW[9];
        for (int i = 0; i < 3; ++i)
          for (int k = 0; k < 3; ++k) GW[i * 3 + k] = G[i * 3 + 0] * W[0 * 3 + k] + G[i * 3 + 1] * W[1 * 3 + k] + G[i * 3 + 2] * W[2 * 3 + k];
        float GS[9];
        for (int i = 0; i < 3; ++i)
          for (int k = 0; k < 3; ++k) GS[i * 3 + k] = W[0 * 3 + i] * GW[0 * 3 + k] + W[1 * 3 + i] * GW[1 * 3 + k] + W[2 * 3 + i] * GW[2 * 3 + k];
        float GM[9];
        for (int i = 0; i < 3; ++i)
          for (int k = 0; k < 3; ++k) GM[i * 3 + k] = 2.f * (GS[i * 3 + 0] * M[0 * 3 + k] + GS[i * 3 + 1] * M[1 * 3 + k] + GS[i * 3 + 2] * M[2 * 3 + k]);
        if (GD.log_scale) {
          for (int k = 0; k < 3; ++k)
            emit(1, k, GD.log_scale, s[k] * (GM[0 * 3 + k] * Rq[0 * 3 + k] + GM[1 * 3 + k] * Rq[1 * 3 + k] + GM[2 * 3 + k] * Rq[2 * 3 + k]));
        }
        if (GD.quat) {
          float GR[9];
          for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) GR[i * 3 + k] = GM[i * 3 + k] * s[k];
          float dq[4];
          rot_backward(qw0, qx0, qy0, qz0, GR, dq);
          for (int k = 0; k < 4; ++k) emit(2, k, GD.quat, dq[k]);
        }
      }
      if (GD.opac) {
        const float op = 1.0f / (1.0f + __expf(-J.opac[g]));
        emit(3, 0, GD.opac, gi[5] * op * (1.f - op));
      }
      if (GD.rgb) {
        for (int k = 0; k < 3; ++k) emit(4, k, GD.rgb, gi[7 + k]);
      }
    }
    if (want_pose && pr != nullptr) {
      float Rd[9];
      quat_to_rot(pr[0], pr[1], pr[2], pr[3], Rd);
      pose_contrib(p, Sc, Rd, pr + 4, dp, G, acc);
    }
  }
  if (kAdam && g < n) {
    float pv[14], mv[14], vv[14];
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
      for (int k = 0; k < (q == 2 ? 4 : q == 3 ? 1 : 3); ++k) {
        const int j2 = kSlot0[q] + k;
        const int64_t idx = (int64_t)k * n + g;
        pv[j2] = params[q][idx];
        mv[j2] = adam.m[r][q][idx];
        vv[j2] = adam.v[r][q][idx];
      }
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
      for (int k = 0; k < (q == 2 ? 4 : q == 3 ? 1 : 3); ++k) {
        const int j2 = kSlot0[q] + k;
        const int64_t idx = (int64_t)k * n + g;
        adam_update(pv[j2], mv[j2], vv[j2], gv[j2], adam.lr[r][q], adam.beta1, adam.beta2, adam.eps, adam.bc1,
                    adam.bc2);
        params[q][idx] = pv[j2];
        adam.m[r][q][idx] = mv[j2];
        adam.v[r][q][idx] = vv[j2];
      }
  }
  if (want_pose) {
    // fixed-order block reduction: wave sums, then the 4 waves in order
    __shared__ float part[4][kPoseAcc];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < kPoseAcc; ++k) {
      const float s = wave_sum(acc[k]);
      if (lane == 0) part[w][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < kPoseAcc) {
      const int k = threadIdx.x;
      pose_part[(int64_t)blockIdx.x * kPoseAcc + k] = (part[0][k] + part[1][k]) + (part[2][k] + part[3][k]);
    }
  }
}

// Per render: sum the partials in order (per 256-item block of the render,
// or per tile when by_tile is set), chain dL/dR_d to the quaternion,
// accumulate into pose_grad [R][7].  One wave per render.
// With step.pose_m set, each render's pose then takes one Adam step from the
// accumulated gradient (as ls_adam over pose_grad), which is consumed.
constexpr int kPoseSumThreads = 256;

// Sum of the kPoseAcc-float rows part[first .. first + nb) over a block of
// kPoseSumThreads threads in a fixed order: strided per-thread sums (each
// row three 16-byte loads, four rows in flight per thread), wave sums, then
// the four waves in order.  Thread 0 returns the totals.
__device__ __forceinline__ void block_pose_sum(const float* __restrict__ part, int first, int nb,
                                               float (&acc)[kPoseAcc]) {
  static_assert(kPoseAcc == 12, "a row is three float4");
  __shared__ float ws[kPoseSumThreads / 64][kPoseAcc];
  const float4* p4 = reinterpret_cast<const float4*>(part);
#pragma unroll
  for (int k = 0; k < kPoseAcc; ++k) acc[k] = 0.f;
  auto add = [&](const float4* row) {
    const float4 x = row[0], y = row[1], z = row[2];
    acc[0] += x.x; acc[1] += x.y; acc[2] += x.z; acc[3] += x.w;
    acc[4] += y.x; acc[5] += y.y; acc[6] += y.z; acc[7] += y.w;
    acc[8] += z.x; acc[9] += z.y; acc[10] += z.z; acc[11] += z.w;
  };
#pragma unroll 4
  for (int b = threadIdx.x; b < nb; b += kPoseSumThreads) add(p4 + 3 * (int64_t)(first + b));
#pragma unroll
  for (int k = 0; k < kPoseAcc; ++k) acc[k] = wave_sum(acc[k]);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < kPoseAcc; ++k) ws[w][k] = acc[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < kPoseAcc; ++k) acc[k] = (ws[0][k] + ws[1][k]) + (ws[2][k] + ws[3][k]);
}

__global__ __launch_bounds__(kPoseSumThreads) void k_pose_reduce(const JobDev* __restrict__ jobs, int R,
                                                                 const float* __restrict__ pose,
                                                                 const float* __restrict__ pose_part,
                                                                 float* __restrict__ pose_grad, int by_tile,
                                                                 GaussAdamArgs step) {
  const int r = blockIdx.x;
  if (r >= R) return;
  const JobDev& J = jobs[r];
  const int first = by_tile ? J.tile_off : J.blk_off;
  const int nb = by_tile ? J.TX * J.TY : (J.n + 255) / 256;
  float acc[kPoseAcc];
  block_pose_sum(pose_part, first, nb, acc);
  if (threadIdx.x == 0) {
    const float* pr = pose + 7 * r;
    float dq[4];
    rot_backward(pr[0], pr[1], pr[2], pr[3], acc, dq);
    float* out = pose_grad + 7 * r;
    for (int k = 0; k < 4; ++k) out[k] += dq[k];
    for (int k = 0; k < 3; ++k) out[4 + k] += acc[9 + k];
    if (step.pose_m) {
      for (int k = 0; k < 7; ++k) {
        const int i = 7 * r + k;
        float p = step.pose[i], m = step.pose_m[i], v = step.pose_v[i];
        adam_update(p, m, v, out[k], k < 4 ? step.lr_rot : step.lr_trans, step.beta1, step.beta2, step.eps, step.bc1,
                    step.bc2);
        step.pose[i] = p;
        step.pose_m[i] = m;
        step.pose_v[i] = v;
        out[k] = 0.f;
      }
    }
  }
}

}  // namespace ls

namespace ls {
void launch_project(const JobDev* jobs, const int32_t* blk_off, int R, int nblk, const float* pose, float* rec,
                    int32_t* radius, int32_t* tiles, float* aux, const ViewOpt* live, hipStream_t s) {
  if (nblk > 0)
    hipLaunchKernelGGL(k_project, dim3(nblk), dim3(256), 0, s, jobs, blk_off, R, pose, reinterpret_cast<float4*>(rec),
                       radius, tiles, reinterpret_cast<float4*>(aux), live);
}
void launch_project_bwd(const JobDev* jobs, const int32_t* blk_off, int R, int nblk, const float* pose,
                        const int32_t* radius, const float* aux, float* g2d, const GradDev* grads, int want_gauss,
                        float* pose_part, int want_pose, float* pose_grad, hipStream_t s, const GaussAdamArgs* adam) {
  if (nblk > 0) {
    if (adam)
      hipLaunchKernelGGL(k_project_bwd<true>, dim3(nblk), dim3(256), 0, s, jobs, blk_off, R, pose, radius,
                         reinterpret_cast<const float4*>(aux), g2d, grads, 1, pose_part, want_pose, *adam);
    else
      hipLaunchKernelGGL(k_project_bwd<false>, dim3(nblk), dim3(256), 0, s, jobs, blk_off, R, pose, radius,
                         reinterpret_cast<const float4*>(aux), g2d, grads, want_gauss, pose_part, want_pose,
                         GaussAdamArgs{});
  }
  if (want_pose)
    hipLaunchKernelGGL(k_pose_reduce, dim3(R), dim3(kPoseSumThreads), 0, s, jobs, R, pose, (const float*)pose_part,
                       pose_grad, 0, adam ? *adam : GaussAdamArgs{});
}

// Pose reduction by tile partials (as k_pose_reduce with by_tile) followed
// by the render's Adam step; block 0 also folds the overflow count into the
// sticky flag.
__global__ __launch_bounds__(kPoseSumThreads) void k_pose_reduce_adam(const JobDev* __restrict__ jobs, int R,
                                                                      const float* __restrict__ tile_part,
                                                                      PoseAdamArgs a,
                                                                      const int32_t* __restrict__ count,
                                                                      int32_t* __restrict__ sticky) {
  const int r = blockIdx.x;
  if (r >= R) return;
  const JobDev& J = jobs[r];
  float acc[kPoseAcc];
  block_pose_sum(tile_part, J.tile_off, J.TX * J.TY, acc);
  if (threadIdx.x == 0) {
    const float* pr = a.pose + 7 * r;
    float dq[4], g[7];
    rot_backward(pr[0], pr[1], pr[2], pr[3], acc, dq);
    for (int k = 0; k < 4; ++k) g[k] = a.grad[7 * r + k] + dq[k];
    for (int k = 0; k < 3; ++k) g[4 + k] = a.grad[7 * r + 4 + k] + acc[9 + k];
    pose_adam_view(a, r, g);
    if (r == 0 && count) or_flag(count, sticky);
  }
}

void launch_pose_reduce_adam(const JobDev* jobs, int R, const float* tile_part, const PoseAdamArgs& a,
                             const int32_t* count, int32_t* sticky, hipStream_t s) {
  if (R > 0)
    hipLaunchKernelGGL(k_pose_reduce_adam, dim3(R), dim3(kPoseSumThreads), 0, s, jobs, R, tile_part, a, count, sticky);
}

void launch_pose_reduce_tiles(const JobDev* jobs, int R, const float* pose, const float* tile_part, float* pose_grad,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_pose_reduce, dim3(R), dim3(kPoseSumThreads), 0, s, jobs, R, pose, tile_part, pose_grad, 1,
                     GaussAdamArgs{});
}
}  // namespace ls

// Per-view pose optimiser kernels for registration (Sec. 3.2): identity
// initialisation and an Adam step whose step counters live on the device, so
// an iteration can be captured once in a graph and replayed.
#include "kernels.h"

namespace ls {

__global__ void k_pose_init(float* __restrict__ pose, float* __restrict__ m, float* __restrict__ v,
                            ViewOpt* __restrict__ opt, int R) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 7 * R) return;
  pose[i] = (i % 7) == 0 ? 1.f : 0.f;
  m[i] = 0.f;
  v[i] = 0.f;
  if (i < R) opt[i].step = 0;
}

// One thread per render: Adam on its 7 pose values (lr_rot for q, lr_trans
// for t), bias correction from the render's own step count; the gradient is
// consumed (zeroed).  Frozen renders keep their pose and clear the gradient.
__global__ void k_pose_adam(float* __restrict__ pose, float* __restrict__ grad, float* __restrict__ m,
                            float* __restrict__ v, ViewOpt* __restrict__ opt, int R, float beta1, float beta2,
                            float eps) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  ViewOpt o = opt[r];
  if (o.active) {
    const int step = o.step + 1;
    const float bc1 = 1.f / (1.f - __powf(beta1, (float)step));
    const float bc2 = 1.f / (1.f - __powf(beta2, (float)step));
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      const int i = 7 * r + k;
      const float g = grad[i];
      const float mi = beta1 * m[i] + (1.f - beta1) * g;
      const float vi = beta2 * v[i] + (1.f - beta2) * g * g;
      m[i] = mi;
      v[i] = vi;
      const float lr = k < 4 ? o.lr_rot : o.lr_trans;
      pose[i] -= lr * (mi * bc1) / (sqrtf(vi * bc2) + eps);
    }
    opt[r].step = step;
  }
#pragma unroll
  for (int k = 0; k < 7; ++k) grad[7 * r + k] = 0.f;
}

__global__ void k_or_flag(const int32_t* __restrict__ count, int32_t* __restrict__ sticky) {
  if (threadIdx.x == 0 && count[1] != 0) *sticky = 1;
}

void launch_pose_init(float* pose, float* m, float* v, ViewOpt* opt, int R, hipStream_t s) {
  const int n = 7 * R;
  hipLaunchKernelGGL(k_pose_init, dim3((n + 255) / 256), dim3(256), 0, s, pose, m, v, opt, R);
}

void launch_pose_adam(float* pose, float* grad, float* m, float* v, ViewOpt* opt, int R, float beta1, float beta2,
                      float eps, hipStream_t s) {
  hipLaunchKernelGGL(k_pose_adam, dim3((R + 255) / 256), dim3(256), 0, s, pose, grad, m, v, opt, R, beta1, beta2,
                     eps);
}

void launch_or_flag(const int32_t* count, int32_t* sticky, hipStream_t s) {
  hipLaunchKernelGGL(k_or_flag, dim3(1), dim3(64), 0, s, count, sticky);
}

}  // namespace ls

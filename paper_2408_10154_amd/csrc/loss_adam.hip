// L1 registration/tracking loss with its image gradients, and fused Adam.
#include "common.h"

#include <algorithm>

namespace ls {

constexpr int kLossPix = 4;  // pixels per thread
constexpr int kLossBlockPix = 256 * kLossPix;

// Per block of 1024 pixels (blocks never straddle renders): writes sign
// gradients on valid pixels and the block's (sum |residual|, valid count).
__global__ __launch_bounds__(256) void k_loss_l1(const JobDev* __restrict__ jobs, const int32_t* __restrict__ pblk_off,
                                                 int R, const float* __restrict__ pred_rgb,
                                                 const float* __restrict__ pred_depth,
                                                 const float* __restrict__ tgt_rgb,
                                                 const float* __restrict__ tgt_depth, float* __restrict__ g_rgb,
                                                 float* __restrict__ g_depth, float* __restrict__ part) {
  const int r = find_segment<int32_t>(pblk_off, R, (int32_t)blockIdx.x);
  const JobDev& J = jobs[r];
  const int64_t hw = (int64_t)J.W * J.H;
  const int64_t b0 = (int64_t)(blockIdx.x - pblk_off[r]) * kLossBlockPix;
  float s = 0.f, cnt = 0.f;
  for (int k = 0; k < kLossPix; ++k) {
    const int64_t p = b0 + (int64_t)k * 256 + threadIdx.x;
    if (p >= hw) break;
    const int64_t pi = J.pix_off + p;
    const int64_t ci = 3 * J.pix_off + p;
    const float* trgb = tgt_rgb ? tgt_rgb + ci : J.tgt_rgb + p;  // per-render targets when not batch-laid-out
    const float td = tgt_depth ? tgt_depth[pi] : J.tgt_depth[p];
    const bool valid = td > 0.f;
    float l = 0.f;
    const float dd = pred_depth[pi] - td;
    l += fabsf(dd);
    if (g_depth) g_depth[pi] = valid ? (dd > 0.f ? 1.f : (dd < 0.f ? -1.f : 0.f)) : 0.f;
    for (int ch = 0; ch < 3; ++ch) {
      const float dc = pred_rgb[ci + ch * hw] - trgb[ch * hw];
      l += fabsf(dc);
      if (g_rgb) g_rgb[ci + ch * hw] = valid ? (dc > 0.f ? 1.f : (dc < 0.f ? -1.f : 0.f)) : 0.f;
    }
    if (valid) { s += l; cnt += 1.f; }
  }
  s = wave_sum(s);
  cnt = wave_sum(cnt);
  __shared__ float ws[4][2];
  if ((threadIdx.x & 63) == 0) { ws[threadIdx.x >> 6][0] = s; ws[threadIdx.x >> 6][1] = cnt; }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int q = threadIdx.x;
    part[2 * (int64_t)blockIdx.x + q] = (ws[0][q] + ws[1][q]) + (ws[2][q] + ws[3][q]);
  }
}

// One wave per render: ordered sum of the block partials.
__global__ void k_loss_reduce(const int32_t* __restrict__ pblk_off, int R, const float* __restrict__ part,
                              float* __restrict__ loss, float* __restrict__ scale) {
  const int r = blockIdx.x;
  if (r >= R) return;
  float s = 0.f, c = 0.f;
  for (int b = pblk_off[r] + threadIdx.x; b < pblk_off[r + 1]; b += 64) {
    s += part[2 * (int64_t)b];
    c += part[2 * (int64_t)b + 1];
  }
  s = wave_sum(s);
  c = wave_sum(c);
  if (threadIdx.x == 0) {
    if (loss) loss[r] = c > 0.f ? s / c : 0.f;
    if (scale) scale[r] = c > 0.f ? 1.f / c : 0.f;
  }
}

struct AdamArgs {
  float* param[16];
  float* grad[16];
  float* m[16];
  float* v[16];
  int64_t n[16];
  float lr[16];
};

__global__ __launch_bounds__(256) void k_adam(AdamArgs a, float beta1, float beta2, float eps, float bc1, float bc2,
                                              int zero_grad) {
  const int gidx = blockIdx.y;
  const int64_t n = a.n[gidx];
  float* __restrict__ p = a.param[gidx];
  float* __restrict__ g = a.grad[gidx];
  float* __restrict__ m = a.m[gidx];
  float* __restrict__ v = a.v[gidx];
  const float lr = a.lr[gidx];
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * bc1) / (sqrtf(vi * bc2) + eps);
    if (zero_grad) g[i] = 0.f;
  }
}

}  // namespace ls

namespace ls {
void launch_loss_l1(const JobDev* jobs, const int32_t* pblk_off_d, int R, int npblk, const float* pred_rgb,
                    const float* pred_depth, const float* tgt_rgb, const float* tgt_depth, float* g_rgb,
                    float* g_depth, float* part, float* loss, float* scale, hipStream_t s) {
  if (npblk > 0)
    hipLaunchKernelGGL(k_loss_l1, dim3(npblk), dim3(256), 0, s, jobs, pblk_off_d, R, pred_rgb, pred_depth, tgt_rgb,
                       tgt_depth, g_rgb, g_depth, part);
  hipLaunchKernelGGL(k_loss_reduce, dim3(R), dim3(64), 0, s, pblk_off_d, R, (const float*)part, loss, scale);
}

void launch_adam(const ls_adam_group* g, int ng, float beta1, float beta2, float eps, float bc1, float bc2,
                 int zero_grad, hipStream_t s) {
  AdamArgs a{};
  int64_t maxn = 0;
  for (int i = 0; i < ng; ++i) {
    a.param[i] = g[i].param;
    a.grad[i] = g[i].grad;
    a.m[i] = g[i].m;
    a.v[i] = g[i].v;
    a.n[i] = g[i].n;
    a.lr[i] = g[i].lr;
    maxn = std::max(maxn, g[i].n);
  }
  if (maxn == 0) return;
  const int64_t bx = std::min<int64_t>((maxn + 255) / 256, 2048);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)bx, ng), dim3(256), 0, s, a, beta1, beta2, eps, bc1, bc2, zero_grad);
}
}  // namespace ls

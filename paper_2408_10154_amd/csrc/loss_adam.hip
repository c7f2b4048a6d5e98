// L1 registration/tracking loss with its image gradients, and fused Adam.
#include "common.h"
#include "kernels.h"

#include <algorithm>

namespace ls {

constexpr int kLossPix = 4;  // pixels per thread
constexpr int kLossBlockPix = 256 * kLossPix;

// Per-render exposure coefficients (a, b) of the rendered colour, C' =
// exp(a) C + b (registration with exposure compensation); identity without.
struct Exposure {
  float gain, offset;
  bool on;
};
__device__ __forceinline__ Exposure exposure_of(const float* expo, int r) {
  Exposure e{1.f, 0.f, expo != nullptr};
  if (e.on) {
    e.gain = expf(expo[2 * r]);
    e.offset = expo[2 * r + 1];
  }
  return e;
}

// Block sums of the exposure-gradient terms (sum g' e^a C and sum g' over
// the block's pixels and channels, g' = dL/dC' before the 1/|Omega| scale).
__device__ __forceinline__ void exposure_partials(float sa, float sb, float* epart) {
  sa = wave_sum(sa);
  sb = wave_sum(sb);
  __shared__ float we[4][2];
  if ((threadIdx.x & 63) == 0) { we[threadIdx.x >> 6][0] = sa; we[threadIdx.x >> 6][1] = sb; }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int q = threadIdx.x;
    epart[2 * (int64_t)blockIdx.x + q] = (we[0][q] + we[1][q]) + (we[2][q] + we[3][q]);
  }
}

// One pixel's inputs to the loss kernels.
struct PixIn {
  float td, pd, al, pc[3], tc[3];
};

// Loads every pixel of the thread (kLossPix, 256 apart) before any is used,
// so the thread waits for memory once; pixels past the image read as zero.
// Targets come batch-laid-out (tgt_* non-null) or per render from the job.
__device__ __forceinline__ void load_pixels(const JobDev& J, int64_t hw, int64_t b0, const float* __restrict__ pred_rgb,
                                            const float* __restrict__ pred_depth,
                                            const float* __restrict__ pred_alpha,
                                            const float* __restrict__ tgt_rgb,
                                            const float* __restrict__ tgt_depth, PixIn (&in)[kLossPix]) {
#pragma unroll
  for (int k = 0; k < kLossPix; ++k) {
    const int64_t p = b0 + (int64_t)k * 256 + threadIdx.x;
    PixIn v{0.f, 0.f, 0.f, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    if (p < hw) {
      const int64_t pi = J.pix_off + p;
      const int64_t ci = 3 * J.pix_off + p;
      const float* trgb = tgt_rgb ? tgt_rgb + ci : J.tgt_rgb + p;
      v.td = tgt_depth ? tgt_depth[pi] : J.tgt_depth[p];
      v.pd = pred_depth[pi];
      if (pred_alpha) v.al = pred_alpha[pi];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        v.pc[ch] = pred_rgb[ci + ch * hw];
        v.tc[ch] = trgb[ch * hw];
      }
    }
    in[k] = v;
  }
}

// Per block of 1024 pixels (blocks never straddle renders): writes sign
// gradients on valid pixels and the block's (sum |residual|, valid count);
// with exposure coefficients the colour residual is taken on exp(a) C + b,
// the colour gradient carries the factor exp(a) and epart receives the
// block's exposure-gradient terms.
__global__ __launch_bounds__(256) void k_loss_l1(const JobDev* __restrict__ jobs, const int32_t* __restrict__ pblk_off,
                                                 int R, const float* __restrict__ pred_rgb,
                                                 const float* __restrict__ pred_depth,
                                                 const float* __restrict__ tgt_rgb,
                                                 const float* __restrict__ tgt_depth, float* __restrict__ g_rgb,
                                                 float* __restrict__ g_depth, float* __restrict__ part,
                                                 const float* __restrict__ expo, float* __restrict__ epart) {
  const int r = find_segment<int32_t>(pblk_off, R, (int32_t)blockIdx.x);
  const JobDev& J = jobs[r];
  const int64_t hw = (int64_t)J.W * J.H;
  const int64_t b0 = (int64_t)(blockIdx.x - pblk_off[r]) * kLossBlockPix;
  const Exposure ex = exposure_of(expo, r);
  float s = 0.f, cnt = 0.f, sa = 0.f, sb = 0.f;
  PixIn in[kLossPix];
  load_pixels(J, hw, b0, pred_rgb, pred_depth, nullptr, tgt_rgb, tgt_depth, in);
#pragma unroll
  for (int k = 0; k < kLossPix; ++k) {
    const int64_t p = b0 + (int64_t)k * 256 + threadIdx.x;
    if (p >= hw) continue;
    const int64_t pi = J.pix_off + p;
    const int64_t ci = 3 * J.pix_off + p;
    const float td = in[k].td;
    const bool valid = td > 0.f;
    float l = 0.f;
    const float dd = in[k].pd - td;
    l += fabsf(dd);
    if (g_depth) g_depth[pi] = valid ? (dd > 0.f ? 1.f : (dd < 0.f ? -1.f : 0.f)) : 0.f;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float pc = in[k].pc[ch];
      const float dc = (ex.on ? ex.gain * pc + ex.offset : pc) - in[k].tc[ch];
      l += fabsf(dc);
      const float sg = dc > 0.f ? 1.f : (dc < 0.f ? -1.f : 0.f);
      if (g_rgb) g_rgb[ci + ch * hw] = valid ? (ex.on ? ex.gain * sg : sg) : 0.f;
      if (valid && ex.on) {
        sa += sg * ex.gain * pc;
        sb += sg;
      }
    }
    if (valid) { s += l; cnt += 1.f; }
  }
  if (epart) exposure_partials(sa, sb, epart);
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

// One wave per render: ordered sum of the block partials; with exposure
// partials, also dL/d(a, b) = (1/|Omega|) (sum g' e^a C, sum g').
__global__ void k_loss_reduce(const int32_t* __restrict__ pblk_off, int R, const float* __restrict__ part,
                              float* __restrict__ loss, float* __restrict__ scale, const float* __restrict__ epart,
                              float* __restrict__ egrad) {
  const int r = blockIdx.x;
  if (r >= R) return;
  float s = 0.f, c = 0.f, sa = 0.f, sb = 0.f;
  for (int b = pblk_off[r] + threadIdx.x; b < pblk_off[r + 1]; b += 64) {
    s += part[2 * (int64_t)b];
    c += part[2 * (int64_t)b + 1];
    if (epart) {
      sa += epart[2 * (int64_t)b];
      sb += epart[2 * (int64_t)b + 1];
    }
  }
  s = wave_sum(s);
  c = wave_sum(c);
  if (epart) {
    sa = wave_sum(sa);
    sb = wave_sum(sb);
  }
  if (threadIdx.x == 0) {
    const float inv = c > 0.f ? 1.f / c : 0.f;
    if (loss) loss[r] = c > 0.f ? s / c : 0.f;
    if (scale) scale[r] = inv;
    if (egrad) {
      egrad[2 * r] = sa * inv;
      egrad[2 * r + 1] = sb * inv;
    }
  }
}

// Per-render L1 loss from the per-tile partials {sum, count} that the
// compositing backward wrote with L1 targets: one 256-thread block per render,
// strided per-thread sums, wave sums, then the four waves in order.
__global__ __launch_bounds__(256) void k_tile_loss_reduce(const JobDev* __restrict__ jobs, int R,
                                                          const float* __restrict__ part, float* __restrict__ loss) {
  __shared__ float ws[2][4];
  const int r = blockIdx.x;
  if (r >= R) return;
  const JobDev& J = jobs[r];
  const int first = J.tile_off, nt = J.TX * J.TY;
  const float2* p2 = reinterpret_cast<const float2*>(part);
  float s = 0.f, c = 0.f;
#pragma unroll 4
  for (int t = threadIdx.x; t < nt; t += 256) {
    const float2 v = p2[first + t];
    s += v.x;
    c += v.y;
  }
  s = wave_sum(s);
  c = wave_sum(c);
  if ((threadIdx.x & 63) == 0) {
    ws[0][threadIdx.x >> 6] = s;
    ws[1][threadIdx.x >> 6] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const float ts = (ws[0][0] + ws[0][1]) + (ws[0][2] + ws[0][3]);
    const float tc = (ws[1][0] + ws[1][1]) + (ws[1][2] + ws[1][3]);
    loss[r] = tc > 0.f ? ts / tc : 0.f;
  }
}

// ---------------------------------------------------------------------------
// Tracking loss with masks (Eq. 2 and the supplement's tracking-loss
// details).  The inlier mask needs, per render, the median of the depth
// error e = |D - D*| over pixels with D* > 0.  It is found exactly by radix
// selection on the bit patterns of the non-negative FP32 errors (their
// unsigned order is their numeric order): three passes over 11, 11 and 10
// bits, each a histogram of the errors that match the digits fixed so far,
// followed by a one-block-per-render pass that picks the digit holding the
// element of rank floor((n-1)/2) and re-zeroes the histogram for the next
// pass (no memset, so the sequence can be captured in a graph).

constexpr int kSelBins = 2048;

struct SelState {
  uint32_t prefix, mask, k, n;
};

__device__ __forceinline__ int sel_shift(int pass) { return pass == 0 ? 21 : (pass == 1 ? 10 : 0); }
__device__ __forceinline__ int sel_bins(int pass) { return pass == 2 ? 1024 : 2048; }

__device__ __forceinline__ float depth_error(float d, float t) { return fabsf(d - t); }

__global__ __launch_bounds__(256) void k_err_hist(const JobDev* __restrict__ jobs, const int32_t* __restrict__ pblk_off,
                                                  int R, const float* __restrict__ pred_depth,
                                                  const float* __restrict__ tgt_depth,
                                                  const SelState* __restrict__ state, uint32_t* __restrict__ hist,
                                                  int pass) {
  __shared__ uint32_t h[kSelBins];
  const int r = find_segment<int32_t>(pblk_off, R, (int32_t)blockIdx.x);
  const JobDev& J = jobs[r];
  const int64_t hw = (int64_t)J.W * J.H;
  const int64_t b0 = (int64_t)(blockIdx.x - pblk_off[r]) * kLossBlockPix;
  const int shift = sel_shift(pass), nb = sel_bins(pass);
  const uint32_t prefix = pass ? state[r].prefix : 0u, mask = pass ? state[r].mask : 0u;
  // every pixel of the thread is loaded before any is counted (one wait for
  // memory, overlapping the histogram clear)
  float td[kLossPix], pd[kLossPix];
#pragma unroll
  for (int k = 0; k < kLossPix; ++k) {
    const int64_t p = b0 + (int64_t)k * 256 + threadIdx.x;
    const bool in = p < hw;
    td[k] = in ? (tgt_depth ? tgt_depth[J.pix_off + p] : J.tgt_depth[p]) : 0.f;
    pd[k] = in ? pred_depth[J.pix_off + p] : 0.f;
  }
  for (int i = threadIdx.x; i < nb; i += 256) h[i] = 0u;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kLossPix; ++k) {
    if (!(td[k] > 0.f)) continue;  // out-of-image pixels carry td = 0
    const uint32_t bits = __float_as_uint(depth_error(pd[k], td[k]));
    if ((bits & mask) == prefix) atomicAdd(&h[(bits >> shift) & (uint32_t)(nb - 1)], 1u);
  }
  __syncthreads();
  uint32_t* __restrict__ g = hist + (int64_t)r * kSelBins;
  for (int i = threadIdx.x; i < nb; i += 256)
    if (h[i]) atomicAdd(&g[i], h[i]);
}

// One block per render: locate the digit of the rank-k element, fold it
// into the prefix, clear the histogram; after the last pass write the median.
__global__ __launch_bounds__(256) void k_err_select(int R, SelState* __restrict__ state, uint32_t* __restrict__ hist,
                                                    float* __restrict__ median, int pass) {
  const int r = blockIdx.x;
  if (r >= R) return;
  const int shift = sel_shift(pass), nb = sel_bins(pass);
  const int per = nb / 256;  // 8 or 4 bins per thread
  uint32_t* __restrict__ g = hist + (int64_t)r * kSelBins;
  uint32_t c[8];
  uint32_t mine = 0;
  for (int j = 0; j < per; ++j) {
    c[j] = g[threadIdx.x * per + j];
    mine += c[j];
  }
  // block-wide exclusive scan of the per-thread sums
  __shared__ uint32_t wsum[4];
  __shared__ uint32_t total_s;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t incl = mine;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  uint32_t before = incl - mine;
  for (int w = 0; w < wv; ++w) before += wsum[w];
  if (threadIdx.x == 0) total_s = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  __syncthreads();
  SelState st = state[r];
  if (pass == 0) {
    st.prefix = 0u;
    st.mask = 0u;
    st.n = total_s;
    st.k = total_s ? (total_s - 1u) / 2u : 0u;
  }
  __syncthreads();
  if (st.n && st.k >= before && st.k < before + mine) {
    uint32_t cum = before;
    for (int j = 0; j < per; ++j) {
      if (st.k < cum + c[j]) {
        const uint32_t digit = (uint32_t)(threadIdx.x * per + j);
        SelState o = st;
        o.prefix |= digit << shift;
        o.mask |= (uint32_t)(nb - 1) << shift;
        o.k -= cum;
        state[r] = o;
        if (pass == 2) median[r] = __uint_as_float(o.prefix);
        break;
      }
      cum += c[j];
    }
  }
  if (!st.n && threadIdx.x == 0) {
    state[r] = st;
    if (pass == 2) median[r] = 0.f;
  }
  for (int j = 0; j < per; ++j) g[threadIdx.x * per + j] = 0u;
}

// Per block of 1024 pixels: the masked, weighted L1 of Eq. 2 with its
// gradient w.r.t. the rendered colour and depth (the alpha weight is a
// constant), and the block's (sum, valid count) partials.
__global__ __launch_bounds__(256) void k_loss_track(const JobDev* __restrict__ jobs,
                                                    const int32_t* __restrict__ pblk_off, int R,
                                                    const float* __restrict__ pred_rgb,
                                                    const float* __restrict__ pred_depth,
                                                    const float* __restrict__ pred_alpha,
                                                    const float* __restrict__ tgt_rgb,
                                                    const float* __restrict__ tgt_depth,
                                                    const float* __restrict__ median, float lambda_c, float inlier_k,
                                                    int alpha_power, float* __restrict__ g_rgb,
                                                    float* __restrict__ g_depth, float* __restrict__ part,
                                                    const float* __restrict__ expo, float* __restrict__ epart) {
  const int r = find_segment<int32_t>(pblk_off, R, (int32_t)blockIdx.x);
  const JobDev& J = jobs[r];
  const int64_t hw = (int64_t)J.W * J.H;
  const int64_t b0 = (int64_t)(blockIdx.x - pblk_off[r]) * kLossBlockPix;
  const float thr = inlier_k > 0.f ? inlier_k * median[r] : 0.f;
  const Exposure ex = exposure_of(expo, r);
  float s = 0.f, cnt = 0.f, sa = 0.f, sb = 0.f;
  PixIn in[kLossPix];
  load_pixels(J, hw, b0, pred_rgb, pred_depth, alpha_power > 0 ? pred_alpha : nullptr, tgt_rgb, tgt_depth, in);
#pragma unroll
  for (int k = 0; k < kLossPix; ++k) {
    const int64_t p = b0 + (int64_t)k * 256 + threadIdx.x;
    if (p >= hw) continue;
    const int64_t pi = J.pix_off + p;
    const int64_t ci = 3 * J.pix_off + p;
    const float td = in[k].td;
    const bool valid = td > 0.f;
    const float dd = in[k].pd - td;
    float w = 0.f;
    if (valid && (inlier_k <= 0.f || depth_error(in[k].pd, td) <= thr)) {
      w = 1.f;
      if (alpha_power > 0) {
        const float a = in[k].al;
        for (int e = 0; e < alpha_power; ++e) w *= a;
      }
    }
    const float wc = w * lambda_c, wd = w * (1.f - lambda_c);
    float lc = 0.f;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float pc = in[k].pc[ch];
      const float dc = (ex.on ? ex.gain * pc + ex.offset : pc) - in[k].tc[ch];
      lc += fabsf(dc);
      const float gc = dc > 0.f ? wc : (dc < 0.f ? -wc : 0.f);
      if (g_rgb) g_rgb[ci + ch * hw] = ex.on ? ex.gain * gc : gc;
      if (ex.on) {
        sa += gc * ex.gain * pc;
        sb += gc;
      }
    }
    if (g_depth) g_depth[pi] = dd > 0.f ? wd : (dd < 0.f ? -wd : 0.f);
    if (valid) {
      s += wc * lc + wd * fabsf(dd);
      cnt += 1.f;
    }
  }
  if (epart) exposure_partials(sa, sb, epart);
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
    float pi = p[i], mi = m[i], vi = v[i];
    adam_update(pi, mi, vi, g[i], lr, beta1, beta2, eps, bc1, bc2);
    p[i] = pi;
    m[i] = mi;
    v[i] = vi;
    if (zero_grad) g[i] = 0.f;
  }
}

}  // namespace ls

namespace ls {
void launch_loss_l1(const JobDev* jobs, const int32_t* pblk_off_d, int R, int npblk, const float* pred_rgb,
                    const float* pred_depth, const float* tgt_rgb, const float* tgt_depth, float* g_rgb,
                    float* g_depth, float* part, float* loss, float* scale, hipStream_t s, const float* expo,
                    float* epart, float* egrad) {
  if (npblk > 0)
    hipLaunchKernelGGL(k_loss_l1, dim3(npblk), dim3(256), 0, s, jobs, pblk_off_d, R, pred_rgb, pred_depth, tgt_rgb,
                       tgt_depth, g_rgb, g_depth, part, expo, epart);
  hipLaunchKernelGGL(k_loss_reduce, dim3(R), dim3(64), 0, s, pblk_off_d, R, (const float*)part, loss, scale,
                     (const float*)epart, egrad);
}

void launch_loss_track(const JobDev* jobs, const int32_t* pblk_off_d, int R, int npblk, const float* pred_rgb,
                       const float* pred_depth, const float* pred_alpha, const float* tgt_rgb, const float* tgt_depth,
                       float lambda_c, float inlier_k, int alpha_power, uint32_t* sel, float* median, float* g_rgb,
                       float* g_depth, float* part, float* loss, float* scale, hipStream_t s, const float* expo,
                       float* epart, float* egrad) {
  SelState* st = reinterpret_cast<SelState*>(sel);
  uint32_t* hist = sel + 4 * (int64_t)R;
  if (inlier_k > 0.f) {
    for (int pass = 0; pass < 3; ++pass) {
      if (npblk > 0)
        hipLaunchKernelGGL(k_err_hist, dim3(npblk), dim3(256), 0, s, jobs, pblk_off_d, R, pred_depth, tgt_depth,
                           (const SelState*)st, hist, pass);
      hipLaunchKernelGGL(k_err_select, dim3(R), dim3(256), 0, s, R, st, hist, median, pass);
    }
  }
  if (npblk > 0)
    hipLaunchKernelGGL(k_loss_track, dim3(npblk), dim3(256), 0, s, jobs, pblk_off_d, R, pred_rgb, pred_depth,
                       pred_alpha, tgt_rgb, tgt_depth, (const float*)median, lambda_c, inlier_k, alpha_power, g_rgb,
                       g_depth, part, expo, epart);
  hipLaunchKernelGGL(k_loss_reduce, dim3(R), dim3(64), 0, s, pblk_off_d, R, (const float*)part, loss, scale,
                     (const float*)epart, egrad);
}

void launch_tile_loss_reduce(const JobDev* jobs, int R, const float* loss_part, float* loss, hipStream_t s) {
  if (R > 0) hipLaunchKernelGGL(k_tile_loss_reduce, dim3(R), dim3(256), 0, s, jobs, R, loss_part, loss);
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

// Submap-update (mapping) loss of Sec. 3.1, Eq. 3-5: the colour term mixing
// L1 and SSIM (Eq. 4), the L1 depth term, and the isotropic regulariser on
// the Gaussian scales (Eq. 5), each with its gradient.
//
// SSIM is the windowed index with an 11 x 11 Gaussian window (sigma 1.5,
// weights summing to 1), zero padding outside the image, C1 = 0.01^2 and
// C2 = 0.03^2, per colour channel, averaged over channels and pixels.  Its
// gradient follows from the three partial derivatives of the per-pixel index
// with respect to the x-side windowed moments (mu_x, E[x^2], E[xy]):
//   dS/dx(q) = sum_p w(p - q) (A_p + 2 x_q B_p + y_q C_p)
// i.e. the same window applied to the maps A, B, C (the window is symmetric).
#include <algorithm>
#include <cmath>

#include "kernels.h"

namespace ls {

constexpr int kSsimR = 5;                    // window radius: 11 taps
constexpr int kSsimTaps = 2 * kSsimR + 1;
constexpr int kSsimT = 32;                   // output tile side
constexpr int kSsimM = kSsimT + 2 * kSsimR;  // 42: side of the region whose SSIM terms reach the tile
constexpr int kSsimI = kSsimT + 4 * kSsimR;  // 52: side of the input region those terms read
constexpr int kSsimIn = kSsimI * kSsimI;     // 2704
constexpr int kSsimLoadPer = (kSsimIn + kBlock - 1) / kBlock;  // 11 input values per thread
constexpr int kSsimRowMom = kSsimI * kSsimM; // 2184: row-filtered moments per map
constexpr int kSsimMom = kSsimM * kSsimM;    // 1764: SSIM terms per map
constexpr int kSsimRowD = kSsimM * kSsimT;   // 1344: row-filtered derivatives per map
// Each filter pass gives a work item a strip of consecutive outputs along the
// filter direction, so an input is read from LDS once per strip rather than
// once per tap.
constexpr int kRowStrip = 6;                         // moment row pass: 52 rows x 7 strips
constexpr int kRowStrips = kSsimM / kRowStrip;
constexpr int kColStrip = 7;                         // moment column pass: 42 columns x 6 strips
constexpr int kColStrips = kSsimM / kColStrip;
constexpr int kDRowStrip = 8;                        // derivative row pass: 42 rows x 4 strips
constexpr int kDRowStrips = kSsimT / kDRowStrip;
constexpr int kOutStrip = kSsimT * kSsimT / kBlock;  // derivative column pass: 32 columns x 8 strips of 4
static_assert(kSsimM % kRowStrip == 0 && kSsimM % kColStrip == 0 && kSsimT % kDRowStrip == 0, "whole strips");
static_assert(kSsimM * kColStrips <= kBlock, "one column strip per thread");
static_assert(kSsimT * (kSsimT / kOutStrip) == kBlock, "one output strip per thread");
constexpr float kSsimC1 = 0.01f * 0.01f;
constexpr float kSsimC2 = 0.03f * 0.03f;
static_assert(3 * kSsimRowD <= 2 * kSsimIn, "row-filtered derivatives fit the input buffer");
static_assert(3 * kSsimMom <= 5 * kSsimRowMom, "derivative maps fit the moment buffer");

struct SsimWindow {
  float w[kSsimTaps];
};

// Pixels with a target depth, per 1024-pixel block (blocks never straddle
// renders).
__global__ __launch_bounds__(256) void k_valid_count(const JobDev* __restrict__ jobs,
                                                     const int32_t* __restrict__ pblk_off, int R,
                                                     const float* __restrict__ tgt_depth, float* __restrict__ part) {
  const int r = find_segment<int32_t>(pblk_off, R, (int32_t)blockIdx.x);
  const JobDev& J = jobs[r];
  const int64_t hw = (int64_t)J.W * J.H;
  const int64_t b0 = (int64_t)(blockIdx.x - pblk_off[r]) * 1024;
  float cnt = 0.f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t p = b0 + (int64_t)k * 256 + threadIdx.x;
    if (p < hw) {
      const float td = tgt_depth ? tgt_depth[J.pix_off + p] : J.tgt_depth[p];
      cnt += td > 0.f ? 1.f : 0.f;
    }
  }
  cnt = wave_sum(cnt);
  __shared__ float ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// Block-wide sum of one value per thread (256 threads), fixed order; the
// total is returned to thread 0.
__device__ __forceinline__ float block_sum(float v, float* ws) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  return (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// One block per render: 1 / |Omega| (0 when no pixel has a target depth).
__global__ __launch_bounds__(256) void k_valid_inv(const int32_t* __restrict__ pblk_off, int R,
                                                   const float* __restrict__ part, float* __restrict__ inv) {
  __shared__ float ws[4];
  const int r = blockIdx.x;
  float c = 0.f;
  for (int b = pblk_off[r] + threadIdx.x; b < pblk_off[r + 1]; b += kBlock) c += part[b];
  c = block_sum(c, ws);
  if (threadIdx.x == 0) inv[r] = c > 0.f ? 1.f / c : 0.f;
}

// One block per (render, colour channel, 32 x 32 output tile).  The block
// stages the 52 x 52 input region of both images in LDS, filters the five
// windowed moments separably (rows, then columns) over the 42 x 42 region
// whose SSIM terms reach the tile, forms the index and its derivative maps
// A, B, C there (zero outside the image), filters those back onto the tile
// and writes the weighted colour gradient; channel-0 blocks also handle the
// depth term.  Partials per block: (sum of SSIM over the tile, L1 colour
// sum and L1 depth sum over its pixels with a target depth).
__global__ __launch_bounds__(256) void k_loss_ssim(const JobDev* __restrict__ jobs,
                                                   const int32_t* __restrict__ sblk_off, int R, int nblk,
                                                   const float* __restrict__ pred_rgb,
                                                   const float* __restrict__ pred_depth,
                                                   const float* __restrict__ tgt_rgb,
                                                   const float* __restrict__ tgt_depth,
                                                   const float* __restrict__ inv_valid, SsimWindow win,
                                                   float lambda_ssim, float lambda_color, float lambda_depth,
                                                   float* __restrict__ g_rgb, float* __restrict__ g_depth,
                                                   float* __restrict__ part) {
  __shared__ float sA[2 * kSsimIn];      // x, y inputs; later the row-filtered derivative maps
  __shared__ float sB[5 * kSsimRowMom];  // row-filtered moments; later the derivative maps
  const int blk = xcd_remap(blockIdx.x, nblk);
  if (blk >= nblk) return;
  const int r = find_segment<int32_t>(sblk_off, R, (int32_t)blk);
  const JobDev& J = jobs[r];
  const int W = J.W, H = J.H;
  const int tx = (W + kSsimT - 1) / kSsimT, ty = (H + kSsimT - 1) / kSsimT;
  const int local = blk - sblk_off[r];
  const int ch = local / (tx * ty);
  const int t = local - ch * tx * ty;
  const int x0 = (t % tx) * kSsimT, y0 = (t / tx) * kSsimT;
  const int64_t hw = (int64_t)W * H;
  const float* __restrict__ X = pred_rgb + 3 * J.pix_off + ch * hw;
  const float* __restrict__ Y = (tgt_rgb ? tgt_rgb + 3 * J.pix_off : J.tgt_rgb) + ch * hw;

  float* sx = sA;
  float* sy = sA + kSsimIn;
  {
    // every load of the input region is issued before the first is used
    float xv[kSsimLoadPer], yv[kSsimLoadPer];
#pragma unroll
    for (int j = 0; j < kSsimLoadPer; ++j) {
      const int i = threadIdx.x + kBlock * j;
      const int rr = i / kSsimI, cc = i - rr * kSsimI;
      const int gy = y0 - 2 * kSsimR + rr, gx = x0 - 2 * kSsimR + cc;
      xv[j] = 0.f;
      yv[j] = 0.f;
      if (i < kSsimIn && gx >= 0 && gx < W && gy >= 0 && gy < H) {
        const int64_t p = (int64_t)gy * W + gx;
        xv[j] = X[p];
        yv[j] = Y[p];
      }
    }
#pragma unroll
    for (int j = 0; j < kSsimLoadPer; ++j) {
      const int i = threadIdx.x + kBlock * j;
      if (i < kSsimIn) {
        sx[i] = xv[j];
        sy[i] = yv[j];
      }
    }
  }
  __syncthreads();

  // this thread's output strip (column ocol, rows o0 .. o0 + kOutStrip - 1):
  // centre values from LDS, depths issued now and used at the end
  const int ocol = threadIdx.x % kSsimT, o0 = (threadIdx.x / kSsimT) * kOutStrip;
  float xq[kOutStrip], yq[kOutStrip], tq[kOutStrip], dq[kOutStrip];
#pragma unroll
  for (int q = 0; q < kOutStrip; ++q) {
    const int li = (o0 + q + 2 * kSsimR) * kSsimI + ocol + 2 * kSsimR;
    xq[q] = sx[li];
    yq[q] = sy[li];
    const int gy = y0 + o0 + q, gx = x0 + ocol;
    tq[q] = dq[q] = 0.f;
    if (gx < W && gy < H) {
      const int64_t p = (int64_t)gy * W + gx;
      tq[q] = tgt_depth ? tgt_depth[J.pix_off + p] : J.tgt_depth[p];
      if (ch == 0) dq[q] = pred_depth[J.pix_off + p];
    }
  }

  // row pass: the five moments of each input row at the 42 moment columns,
  // kRowStrip consecutive columns per work item (each input read once)
  for (int it = threadIdx.x; it < kSsimI * kRowStrips; it += kBlock) {
    const int rr = it / kRowStrips, c0 = (it - rr * kRowStrips) * kRowStrip;
    const float* xr = sx + rr * kSsimI + c0;
    const float* yr = sy + rr * kSsimI + c0;
    float a[kRowStrip], b[kRowStrip], c[kRowStrip], d[kRowStrip], e[kRowStrip];
#pragma unroll
    for (int o = 0; o < kRowStrip; ++o) a[o] = b[o] = c[o] = d[o] = e[o] = 0.f;
#pragma unroll
    for (int k = 0; k < kRowStrip + 2 * kSsimR; ++k) {
      const float xv = xr[k], yv = yr[k];
      const float xx = xv * xv, yy = yv * yv, xy = xv * yv;
#pragma unroll
      for (int o = 0; o < kRowStrip; ++o) {
        const int tap = k - o;
        if (tap >= 0 && tap < kSsimTaps) {
          const float w = win.w[tap];
          a[o] += w * xv;
          b[o] += w * yv;
          c[o] += w * xx;
          d[o] += w * yy;
          e[o] += w * xy;
        }
      }
    }
    float* out = sB + rr * kSsimM + c0;
#pragma unroll
    for (int o = 0; o < kRowStrip; ++o) {
      out[o] = a[o];
      out[kSsimRowMom + o] = b[o];
      out[2 * kSsimRowMom + o] = c[o];
      out[3 * kSsimRowMom + o] = d[o];
      out[4 * kSsimRowMom + o] = e[o];
    }
  }
  __syncthreads();

  // column pass, SSIM index and its derivative maps on the 42 x 42 region:
  // one strip of kColStrip rows of one moment column per thread
  float dA[kColStrip], dB[kColStrip], dC[kColStrip];
  float ssum = 0.f;
  const int mc = threadIdx.x % kSsimM, r0 = (threadIdx.x / kSsimM) * kColStrip;
  const bool col_item = threadIdx.x < kSsimM * kColStrips;
#pragma unroll
  for (int q = 0; q < kColStrip; ++q) dA[q] = dB[q] = dC[q] = 0.f;
  if (col_item) {
    float mx[kColStrip], my[kColStrip], exx[kColStrip], eyy[kColStrip], exy[kColStrip];
#pragma unroll
    for (int q = 0; q < kColStrip; ++q) mx[q] = my[q] = exx[q] = eyy[q] = exy[q] = 0.f;
#pragma unroll
    for (int k = 0; k < kColStrip + 2 * kSsimR; ++k) {
      const int o = (r0 + k) * kSsimM + mc;
      const float v0 = sB[o], v1 = sB[kSsimRowMom + o], v2 = sB[2 * kSsimRowMom + o];
      const float v3 = sB[3 * kSsimRowMom + o], v4 = sB[4 * kSsimRowMom + o];
#pragma unroll
      for (int q = 0; q < kColStrip; ++q) {
        const int tap = k - q;
        if (tap >= 0 && tap < kSsimTaps) {
          const float w = win.w[tap];
          mx[q] += w * v0;
          my[q] += w * v1;
          exx[q] += w * v2;
          eyy[q] += w * v3;
          exy[q] += w * v4;
        }
      }
    }
    const int gx = x0 - kSsimR + mc;
#pragma unroll
    for (int q = 0; q < kColStrip; ++q) {
      const int mr = r0 + q;
      const int gy = y0 - kSsimR + mr;
      if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
        const float vx = exx[q] - mx[q] * mx[q], vy = eyy[q] - my[q] * my[q], cxy = exy[q] - mx[q] * my[q];
        const float n1 = 2.f * mx[q] * my[q] + kSsimC1, n2 = 2.f * cxy + kSsimC2;
        const float i1 = 1.f / (mx[q] * mx[q] + my[q] * my[q] + kSsimC1), i2 = 1.f / (vx + vy + kSsimC2);
        const float sv = n1 * n2 * i1 * i2;
        dA[q] = 2.f * my[q] * (n2 - n1) * i1 * i2 - 2.f * mx[q] * sv * (i1 - i2);
        dB[q] = -sv * i2;
        dC[q] = 2.f * n1 * i1 * i2;
        if (mr >= kSsimR && mr < kSsimR + kSsimT && mc >= kSsimR && mc < kSsimR + kSsimT) ssum += sv;
      }
    }
  }
  __syncthreads();  // every thread is done with the moments
  if (col_item) {
#pragma unroll
    for (int q = 0; q < kColStrip; ++q) {
      const int i = (r0 + q) * kSsimM + mc;
      sB[i] = dA[q];
      sB[kSsimMom + i] = dB[q];
      sB[2 * kSsimMom + i] = dC[q];
    }
  }
  __syncthreads();

  // row pass over the derivative maps: 42 rows x 32 output columns,
  // kDRowStrip columns per work item
  for (int it = threadIdx.x; it < kSsimM * kDRowStrips; it += kBlock) {
    const int mr = it / kDRowStrips, c0 = (it - mr * kDRowStrips) * kDRowStrip;
    const float* in = sB + mr * kSsimM + c0;
    float a[kDRowStrip], b[kDRowStrip], c[kDRowStrip];
#pragma unroll
    for (int o = 0; o < kDRowStrip; ++o) a[o] = b[o] = c[o] = 0.f;
#pragma unroll
    for (int k = 0; k < kDRowStrip + 2 * kSsimR; ++k) {
      const float va = in[k], vb = in[kSsimMom + k], vc = in[2 * kSsimMom + k];
#pragma unroll
      for (int o = 0; o < kDRowStrip; ++o) {
        const int tap = k - o;
        if (tap >= 0 && tap < kSsimTaps) {
          const float w = win.w[tap];
          a[o] += w * va;
          b[o] += w * vb;
          c[o] += w * vc;
        }
      }
    }
    float* out = sA + mr * kSsimT + c0;
#pragma unroll
    for (int o = 0; o < kDRowStrip; ++o) {
      out[o] = a[o];
      out[kSsimRowD + o] = b[o];
      out[2 * kSsimRowD + o] = c[o];
    }
  }
  __syncthreads();

  // column pass onto the tile (a strip of kOutStrip rows of one column per
  // thread) and the weighted gradients
  const float inv = inv_valid[r];
  const float k_l1 = lambda_color * (1.f - lambda_ssim) * inv;
  const float k_ss = -lambda_color * lambda_ssim / (3.f * (float)hw);
  const float k_d = lambda_depth * inv;
  float l1 = 0.f, l1d = 0.f;
  {
    float fa[kOutStrip], fb[kOutStrip], fc[kOutStrip];
#pragma unroll
    for (int q = 0; q < kOutStrip; ++q) fa[q] = fb[q] = fc[q] = 0.f;
#pragma unroll
    for (int k = 0; k < kOutStrip + 2 * kSsimR; ++k) {
      const int li = (o0 + k) * kSsimT + ocol;
      const float va = sA[li], vb = sA[kSsimRowD + li], vc = sA[2 * kSsimRowD + li];
#pragma unroll
      for (int q = 0; q < kOutStrip; ++q) {
        const int tap = k - q;
        if (tap >= 0 && tap < kSsimTaps) {
          const float w = win.w[tap];
          fa[q] += w * va;
          fb[q] += w * vb;
          fc[q] += w * vc;
        }
      }
    }
    const int gx = x0 + ocol;
#pragma unroll
    for (int q = 0; q < kOutStrip; ++q) {
      const int gy = y0 + o0 + q;
      if (gx < W && gy < H) {
        const int64_t p = (int64_t)gy * W + gx;
        const float xv = xq[q], yv = yq[q];
        const float td = tq[q];
        const bool valid = td > 0.f;
        const float dc = xv - yv;
        float g = k_ss * (fa[q] + 2.f * xv * fb[q] + yv * fc[q]);
        if (valid) {
          l1 += fabsf(dc);
          g += dc > 0.f ? k_l1 : (dc < 0.f ? -k_l1 : 0.f);
        }
        if (g_rgb) g_rgb[3 * J.pix_off + ch * hw + p] = g;
        if (ch == 0) {
          const float dd = dq[q] - td;
          if (valid) l1d += fabsf(dd);
          if (g_depth) g_depth[J.pix_off + p] = valid ? (dd > 0.f ? k_d : (dd < 0.f ? -k_d : 0.f)) : 0.f;
        }
      }
    }
  }
  ssum = wave_sum(ssum);
  l1 = wave_sum(l1);
  l1d = wave_sum(l1d);
  __shared__ float ws[4][3];
  if ((threadIdx.x & 63) == 0) {
    ws[threadIdx.x >> 6][0] = ssum;
    ws[threadIdx.x >> 6][1] = l1;
    ws[threadIdx.x >> 6][2] = l1d;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int q = threadIdx.x;
    part[3 * (int64_t)blk + q] = (ws[0][q] + ws[1][q]) + (ws[2][q] + ws[3][q]);
  }
}

// One block per render: ordered sums of the block partials and the loss
//   lc ((1 - ls) L1_rgb + ls (1 - mean SSIM)) + ld L1_depth.
__global__ __launch_bounds__(256) void k_map_reduce(const JobDev* __restrict__ jobs,
                                                    const int32_t* __restrict__ sblk_off, int R,
                                                    const float* __restrict__ part,
                                                    const float* __restrict__ inv_valid, float lambda_ssim,
                                                    float lambda_color, float lambda_depth, float* __restrict__ loss,
                                                    float* __restrict__ scale) {
  __shared__ float ws[3][4];
  const int r = blockIdx.x;
  float s = 0.f, c = 0.f, d = 0.f;
  for (int b = sblk_off[r] + threadIdx.x; b < sblk_off[r + 1]; b += kBlock) {
    s += part[3 * (int64_t)b];
    c += part[3 * (int64_t)b + 1];
    d += part[3 * (int64_t)b + 2];
  }
  s = block_sum(s, ws[0]);
  c = block_sum(c, ws[1]);
  d = block_sum(d, ws[2]);
  if (threadIdx.x == 0) {
    const float inv = inv_valid[r];
    const float n = 3.f * (float)jobs[r].W * (float)jobs[r].H;
    if (loss)
      loss[r] = lambda_color * ((1.f - lambda_ssim) * c * inv + lambda_ssim * (1.f - s / n)) + lambda_depth * d * inv;
    if (scale) scale[r] = 1.f;
  }
}

// Isotropic regulariser (Eq. 5): per Gaussian sum_j |s_j - mean(s)| with
// s = exp(log_scale); its gradient coef * s_j (sign(d_j) - mean_i sign(d_i))
// is added to grad; one partial sum per block.
__global__ __launch_bounds__(256) void k_isotropic(const float* __restrict__ log_scale, int64_t n, float coef,
                                                   float* __restrict__ grad, float* __restrict__ part) {
  float acc = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const float s0 = expf(log_scale[i]), s1 = expf(log_scale[n + i]), s2 = expf(log_scale[2 * n + i]);
    const float m = (s0 + s1 + s2) * (1.f / 3.f);
    const float d0 = s0 - m, d1 = s1 - m, d2 = s2 - m;
    acc += (fabsf(d0) + fabsf(d1)) + fabsf(d2);
    if (grad) {
      const float g0 = d0 > 0.f ? 1.f : (d0 < 0.f ? -1.f : 0.f);
      const float g1 = d1 > 0.f ? 1.f : (d1 < 0.f ? -1.f : 0.f);
      const float g2 = d2 > 0.f ? 1.f : (d2 < 0.f ? -1.f : 0.f);
      const float gm = (g0 + g1 + g2) * (1.f / 3.f);
      grad[i] += coef * s0 * (g0 - gm);
      grad[n + i] += coef * s1 * (g1 - gm);
      grad[2 * n + i] += coef * s2 * (g2 - gm);
    }
  }
  acc = wave_sum(acc);
  __shared__ float ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

__global__ __launch_bounds__(256) void k_isotropic_reduce(const float* __restrict__ part, int nblk, float coef,
                                                          float* __restrict__ loss) {
  float v = 0.f;
  for (int b = threadIdx.x; b < nblk; b += kBlock) v += part[b];
  v = wave_sum(v);
  __shared__ float ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) loss[0] = coef * ((ws[0] + ws[1]) + (ws[2] + ws[3]));
}

static SsimWindow ssim_window() {
  SsimWindow w;
  double g[kSsimTaps], tot = 0.0;
  for (int k = 0; k < kSsimTaps; ++k) {
    const double d = k - kSsimR;
    g[k] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
    tot += g[k];
  }
  for (int k = 0; k < kSsimTaps; ++k) w.w[k] = (float)(g[k] / tot);
  return w;
}

void launch_valid_inv(const JobDev* jobs, const int32_t* pblk_off_d, int npblk, int R, const float* tgt_depth,
                      float* cnt_part, float* inv, hipStream_t s) {
  if (npblk > 0)
    hipLaunchKernelGGL(k_valid_count, dim3(npblk), dim3(256), 0, s, jobs, pblk_off_d, R, tgt_depth, cnt_part);
  if (R > 0) hipLaunchKernelGGL(k_valid_inv, dim3(R), dim3(kBlock), 0, s, pblk_off_d, R, (const float*)cnt_part, inv);
}

int ssim_blocks(int W, int H) { return 3 * ((W + kSsimT - 1) / kSsimT) * ((H + kSsimT - 1) / kSsimT); }

void launch_loss_mapping(const JobDev* jobs, const int32_t* pblk_off_d, int npblk, const int32_t* sblk_off_d,
                         int nsblk, int R, const float* pred_rgb, const float* pred_depth, const float* tgt_rgb,
                         const float* tgt_depth, float lambda_ssim, float lambda_color, float lambda_depth,
                         float* g_rgb, float* g_depth, float* cnt_part, float* map_part, float* loss, float* scale,
                         hipStream_t s) {
  float* inv = map_part + 3 * (int64_t)nsblk;
  if (npblk > 0)
    hipLaunchKernelGGL(k_valid_count, dim3(npblk), dim3(256), 0, s, jobs, pblk_off_d, R, tgt_depth, cnt_part);
  hipLaunchKernelGGL(k_valid_inv, dim3(R), dim3(kBlock), 0, s, pblk_off_d, R, (const float*)cnt_part, inv);
  if (nsblk > 0) {
    const int grid = 8 * ((nsblk + 7) / 8);
    hipLaunchKernelGGL(k_loss_ssim, dim3(grid), dim3(kBlock), 0, s, jobs, sblk_off_d, R, nsblk, pred_rgb, pred_depth,
                       tgt_rgb, tgt_depth, (const float*)inv, ssim_window(), lambda_ssim, lambda_color, lambda_depth,
                       g_rgb, g_depth, map_part);
  }
  hipLaunchKernelGGL(k_map_reduce, dim3(R), dim3(kBlock), 0, s, jobs, sblk_off_d, R, (const float*)map_part,
                     (const float*)inv, lambda_ssim, lambda_color, lambda_depth, loss, scale);
}

void launch_loss_isotropic(const float* log_scale, int64_t n, float lambda_reg, float* loss, float* grad, float* part,
                           hipStream_t s) {
  const float coef = n > 0 ? lambda_reg / (float)n : 0.f;
  const int nblk = (int)std::min<int64_t>(std::max<int64_t>((n + kBlock - 1) / kBlock, 1), kIsotropicBlocks);
  hipLaunchKernelGGL(k_isotropic, dim3(nblk), dim3(kBlock), 0, s, log_scale, n, coef, grad, part);
  hipLaunchKernelGGL(k_isotropic_reduce, dim3(1), dim3(kBlock), 0, s, (const float*)part, nblk, coef, loss);
}

}  // namespace ls

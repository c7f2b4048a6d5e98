// Front-to-back alpha compositing (forward) and its back-to-front
// recomputation (backward), one 16x16 tile per 256-thread block, gfx950.
//
// Splat records of a tile's list are staged through LDS in chunks of 256;
// every lane reads the same record (LDS broadcast).  The forward stops a
// block's chunk loop once every pixel of the tile has terminated.
#include "common.h"
#include "kernels.h"

namespace ls {

struct TileCtx {
  int r;         // render
  int tile;      // global tile index
  int x, y;      // pixel of this thread
  bool inside;
  int64_t pix;   // pixel index in the image arrays (if inside)
  int W, H;
};

__device__ __forceinline__ TileCtx tile_ctx(const JobDev* jobs, const int32_t* tile_off, int R, int tile) {
  TileCtx c;
  c.tile = tile;
  c.r = find_segment<int32_t>(tile_off, R, tile);
  const JobDev& J = jobs[c.r];
  const int lt = tile - J.tile_off;
  const int ty = lt / J.TX, tx = lt - ty * J.TX;
  c.x = tx * kTile + (threadIdx.x & 15);
  c.y = ty * kTile + (threadIdx.x >> 4);
  c.W = J.W;
  c.H = J.H;
  c.inside = c.x < J.W && c.y < J.H;
  c.pix = J.pix_off + (int64_t)c.y * J.W + c.x;
  return c;
}

__global__ __launch_bounds__(kBlock) void k_composite_fwd(const JobDev* __restrict__ jobs,
                                                          const int32_t* __restrict__ tile_off, int R, int T_total,
                                                          const float4* __restrict__ rec,
                                                          const int32_t* __restrict__ items,
                                                          const int32_t* __restrict__ range, float bg0, float bg1,
                                                          float bg2, float* __restrict__ out_rgb,
                                                          float* __restrict__ out_depth, float* __restrict__ out_alpha,
                                                          float* __restrict__ out_T, int32_t* __restrict__ out_n) {
  __shared__ float4 s0[kBlock], s1[kBlock], s2[kBlock];
  const int tile = xcd_remap(blockIdx.x, T_total);
  if (tile >= T_total) return;
  const TileCtx c = tile_ctx(jobs, tile_off, R, tile);
  const int start = range[2 * tile], end = range[2 * tile + 1];
  const float fx = (float)c.x + 0.5f, fy = (float)c.y + 0.5f;

  float T = 1.f, cr = 0.f, cg = 0.f, cb = 0.f, dd = 0.f;
  bool done = !c.inside;
  int nlast = end - start;
  for (int chunk = start; chunk < end; chunk += kBlock) {
    if (__syncthreads_count(done) == kBlock) break;
    const int e = chunk + threadIdx.x;
    if (e < end) {
      const int64_t it = items[e];
      s0[threadIdx.x] = rec[it * 3 + 0];
      s1[threadIdx.x] = rec[it * 3 + 1];
      s2[threadIdx.x] = rec[it * 3 + 2];
    }
    __syncthreads();
    const int cnt = min(kBlock, end - chunk);
    for (int j = 0; j < cnt; ++j) {
      if (done) continue;
      const float4 a = s0[j];
      const float4 b = s1[j];
      const float dx = fx - a.x, dy = fy - a.y;
      const float sig = falloff(a.z, a.w, b.x, dx, dy);
      if (sig < 0.f) continue;
      const float al = fminf(LS_ALPHA_MAX, b.y * __expf(-sig));
      if (al < LS_ALPHA_MIN) continue;
      const float Tn = T * (1.f - al);
      if (Tn < LS_T_STOP) {
        done = true;
        nlast = chunk + j - start;
        continue;
      }
      const float4 col = s2[j];
      const float wgt = al * T;
      cr += wgt * col.x;
      cg += wgt * col.y;
      cb += wgt * col.z;
      dd += wgt * b.z;
      T = Tn;
    }
  }
  if (!c.inside) return;
  const JobDev& J = jobs[c.r];
  const int64_t hw = (int64_t)J.W * J.H;
  float* rgb = out_rgb + 3 * J.pix_off + (int64_t)c.y * J.W + c.x;
  rgb[0] = cr + T * bg0;
  rgb[hw] = cg + T * bg1;
  rgb[2 * hw] = cb + T * bg2;
  out_depth[c.pix] = dd;
  out_alpha[c.pix] = 1.f - T;
  out_T[c.pix] = T;
  out_n[c.pix] = nlast;
}

// Backward.  Per pixel, walking the list from n_last - 1 down to 0 with the
// transmittance recovered as T_i = T_{i+1} / (1 - alpha_i) and the running
// "behind" value acc = sum_{j>i} alpha_j prod_{i<k<j}(1 - alpha_k) v_j +
// prod_{k>i}(1 - alpha_k)(bg . gC - gA), where v_j = c_j . gC + z_j gD:
//   dL/dalpha_i = T_i (v_i - acc_i).
// The ten image-space gradients of each Gaussian are summed over the wave
// (DPP), the four wave sums over the block (LDS, fixed order), and added to
// the item's accumulator with one atomic per value and tile.
__global__ __launch_bounds__(kBlock) void k_composite_bwd(const JobDev* __restrict__ jobs,
                                                          const int32_t* __restrict__ tile_off, int R, int T_total,
                                                          const float4* __restrict__ rec,
                                                          const int32_t* __restrict__ items,
                                                          const int32_t* __restrict__ range, float bg0, float bg1,
                                                          float bg2, const float* __restrict__ fwd_T,
                                                          const int32_t* __restrict__ fwd_n,
                                                          const float* __restrict__ up_rgb,
                                                          const float* __restrict__ up_depth,
                                                          const float* __restrict__ up_alpha,
                                                          const float* __restrict__ up_scale,
                                                          float* __restrict__ g2d) {
  __shared__ float4 s0[kBlock], s1[kBlock], s2[kBlock];
  __shared__ int32_t sit[kBlock];
  __shared__ float part[kBlock][4][kGrad2D];
  __shared__ int smax;
  const int tile = xcd_remap(blockIdx.x, T_total);
  if (tile >= T_total) return;
  const TileCtx c = tile_ctx(jobs, tile_off, R, tile);
  const JobDev& J = jobs[c.r];
  const int start = range[2 * tile], end = range[2 * tile + 1];
  const float fx = (float)c.x + 0.5f, fy = (float)c.y + 0.5f;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;

  float T = 1.f, gR = 0.f, gG = 0.f, gB = 0.f, gD = 0.f, acc = 0.f;
  int nl = 0;
  if (c.inside) {
    const int64_t hw = (int64_t)J.W * J.H;
    const int64_t ci = 3 * J.pix_off + (int64_t)c.y * J.W + c.x;
    const float sc = up_scale ? up_scale[c.r] : 1.f;
    if (up_rgb) { gR = sc * up_rgb[ci]; gG = sc * up_rgb[ci + hw]; gB = sc * up_rgb[ci + 2 * hw]; }
    if (up_depth) gD = sc * up_depth[c.pix];
    const float gA = up_alpha ? sc * up_alpha[c.pix] : 0.f;
    T = fwd_T[c.pix];
    nl = fwd_n[c.pix];
    acc = bg0 * gR + bg1 * gG + bg2 * gB - gA;
  }
  if (threadIdx.x == 0) smax = 0;
  __syncthreads();
  if (nl > 0) atomicMax(&smax, nl);
  __syncthreads();
  const int last = min(start + smax, end);  // exclusive end of the entries any pixel visited

  for (int chunk_end = last; chunk_end > start; chunk_end -= kBlock) {
    const int chunk = max(start, chunk_end - kBlock);
    const int cnt = chunk_end - chunk;
    if ((int)threadIdx.x < cnt) {
      const int64_t it = items[chunk + threadIdx.x];
      sit[threadIdx.x] = (int32_t)it;
      s0[threadIdx.x] = rec[it * 3 + 0];
      s1[threadIdx.x] = rec[it * 3 + 1];
      s2[threadIdx.x] = rec[it * 3 + 2];
    }
    __syncthreads();
    for (int j = cnt - 1; j >= 0; --j) {
      const int k = chunk + j - start;  // list position
      float g[kGrad2D];
#pragma unroll
      for (int q = 0; q < kGrad2D; ++q) g[q] = 0.f;
      bool act = false;
      if (k < nl) {
        const float4 a = s0[j];
        const float4 b = s1[j];
        const float dx = fx - a.x, dy = fy - a.y;
        const float sig = falloff(a.z, a.w, b.x, dx, dy);
        if (sig >= 0.f) {
          const float ex = __expf(-sig);
          const float G = b.y * ex;
          const float al = fminf(LS_ALPHA_MAX, G);
          if (al >= LS_ALPHA_MIN) {
            act = true;
            const float om = 1.f - al;
            T = T * __builtin_amdgcn_rcpf(om);
            const float4 col = s2[j];
            const float wgt = al * T;
            const float v = col.x * gR + col.y * gG + col.z * gB + b.z * gD;
            const float dal = T * (v - acc);
            acc = al * v + om * acc;
            g[7] = wgt * gR;
            g[8] = wgt * gG;
            g[9] = wgt * gB;
            g[6] = wgt * gD;
            const float dG = (G < LS_ALPHA_MAX) ? dal : 0.f;
            g[5] = dG * ex;                  // dL/d opacity
            const float ds = -dG * G;        // dL/d sigma
            g[0] = -ds * (a.z * dx + a.w * dy);  // dL/du
            g[1] = -ds * (a.w * dx + b.x * dy);  // dL/dv
            g[2] = 0.5f * ds * dx * dx;          // dL/dA
            g[3] = ds * dx * dy;                 // dL/dB
            g[4] = 0.5f * ds * dy * dy;          // dL/dC
          }
        }
      }
      if (__ballot(act) != 0ull) {
#pragma unroll
        for (int q = 0; q < kGrad2D; ++q) {
          const float s = wave_sum(g[q]);
          if (lane == 0) part[j][w][q] = s;
        }
      } else if (lane < kGrad2D) {
        part[j][w][lane] = 0.f;
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
      const int j = threadIdx.x;
      float* dst = g2d + (int64_t)sit[j] * kGrad2D;
#pragma unroll
      for (int q = 0; q < kGrad2D; ++q) {
        const float s = (part[j][0][q] + part[j][1][q]) + (part[j][2][q] + part[j][3][q]);
        if (s != 0.f) atomic_add_f32(dst + q, s);
      }
    }
    __syncthreads();
  }
}

// Work statistics of a forward pass: entries evaluated and composited.
__global__ __launch_bounds__(kBlock) void k_render_stats(const JobDev* __restrict__ jobs,
                                                         const int32_t* __restrict__ tile_off, int R, int T_total,
                                                         const float4* __restrict__ rec,
                                                         const int32_t* __restrict__ items,
                                                         const int32_t* __restrict__ range,
                                                         const int32_t* __restrict__ fwd_n,
                                                         unsigned long long* __restrict__ stats) {
  __shared__ float4 s0[kBlock], s1[kBlock];
  const int tile = xcd_remap(blockIdx.x, T_total);
  if (tile >= T_total) return;
  const TileCtx c = tile_ctx(jobs, tile_off, R, tile);
  const int start = range[2 * tile], end = range[2 * tile + 1];
  const float fx = (float)c.x + 0.5f, fy = (float)c.y + 0.5f;
  const int nl = c.inside ? fwd_n[c.pix] : 0;
  unsigned long long visited = c.inside ? (unsigned long long)min(nl + 1, end - start) : 0ull;
  unsigned long long comp = 0;
  for (int chunk = start; chunk < end; chunk += kBlock) {
    const int e = chunk + threadIdx.x;
    if (e < end) {
      const int64_t it = items[e];
      s0[threadIdx.x] = rec[it * 3 + 0];
      s1[threadIdx.x] = rec[it * 3 + 1];
    }
    __syncthreads();
    const int cnt = min(kBlock, end - chunk);
    for (int j = 0; j < cnt; ++j) {
      if (chunk + j - start >= nl) break;
      const float4 a = s0[j];
      const float4 b = s1[j];
      const float dx = fx - a.x, dy = fy - a.y;
      const float sig = falloff(a.z, a.w, b.x, dx, dy);
      if (sig < 0.f) continue;
      const float al = fminf(LS_ALPHA_MAX, b.y * __expf(-sig));
      if (al >= LS_ALPHA_MIN) ++comp;
    }
    __syncthreads();
  }
  for (int off = 32; off > 0; off >>= 1) {
    visited += __shfl_xor(visited, off, 64);
    comp += __shfl_xor(comp, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(stats, visited);
    atomicAdd(stats + 1, comp);
  }
}

}  // namespace ls

namespace ls {
void launch_render_stats(const JobDev* jobs, const int32_t* tile_off, int R, int T, const float* rec,
                         const int32_t* items, const int32_t* range, const int32_t* nl, int64_t* stats,
                         hipStream_t s) {
  launch_fill_i32(reinterpret_cast<int32_t*>(stats), 4, 0, s);
  if (T <= 0) return;
  hipLaunchKernelGGL(k_render_stats, dim3(8 * ((T + 7) / 8)), dim3(kBlock), 0, s, jobs, tile_off, R, T,
                     reinterpret_cast<const float4*>(rec), items, range, nl,
                     reinterpret_cast<unsigned long long*>(stats));
}

static inline int xcd_grid(int total) { return 8 * ((total + 7) / 8); }

void launch_composite_fwd(const JobDev* jobs, const int32_t* tile_off, int R, int T, const float* rec,
                          const int32_t* items, const int32_t* range, const float* bg, float* rgb, float* depth,
                          float* alpha, float* Tf, int32_t* nl, hipStream_t s) {
  if (T <= 0) return;
  hipLaunchKernelGGL(k_composite_fwd, dim3(xcd_grid(T)), dim3(kBlock), 0, s, jobs, tile_off, R, T,
                     reinterpret_cast<const float4*>(rec), items, range, bg[0], bg[1], bg[2], rgb, depth, alpha, Tf,
                     nl);
}

void launch_composite_bwd(const JobDev* jobs, const int32_t* tile_off, int R, int T, const float* rec,
                          const int32_t* items, const int32_t* range, const float* bg, const float* Tf,
                          const int32_t* nl, const float* up_rgb, const float* up_depth, const float* up_alpha,
                          const float* up_scale, float* g2d, hipStream_t s) {
  if (T <= 0) return;
  hipLaunchKernelGGL(k_composite_bwd, dim3(xcd_grid(T)), dim3(kBlock), 0, s, jobs, tile_off, R, T,
                     reinterpret_cast<const float4*>(rec), items, range, bg[0], bg[1], bg[2], Tf, nl, up_rgb, up_depth,
                     up_alpha, up_scale, g2d);
}
}  // namespace ls

// Tile binning on gfx950: depth keys, LSD radix sort (8-bit digits, stable),
// count scan, instance emission in depth order, tile ranges.
//
// Order of the final list: (tile, FP32 depth bits, item).  It is produced as
// a stable depth sort of the items (ties keep ascending item order), then
// emission of each item's tiles in that order, then a stable sort of the
// instances by tile key.
#include "common.h"

#include <algorithm>

namespace ls {

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = i; k < n; k += stride) p[k] = v;
}

// Depth keys: FP32 depth bits (positive depths order like their bits);
// culled items get 0xFFFFFFFF and sort last.
__global__ void k_depth_keys(const float4* __restrict__ rec, const int32_t* __restrict__ tiles, int64_t M,
                             uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const float z = rec[i * 3 + 1].z;
  keys[i] = tiles[i] > 0 ? __float_as_uint(z) : 0xFFFFFFFFu;
  vals[i] = (uint32_t)i;
}

__device__ __forceinline__ int sort_count(const int32_t* n_dev, int64_t n_static, int64_t cap) {
  int64_t n = n_static;
  if (n_dev) n = min((int64_t)n_dev[0], cap);
  return (int)n;
}

// Per-block digit histogram, stored digit-major: hist[d * nblocks + block].
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const uint32_t* __restrict__ keys, const int32_t* n_dev,
                                                            int64_t n_static, int64_t cap, int shift,
                                                            uint32_t* __restrict__ hist, int nblocks) {
  __shared__ uint32_t h[256];
  const int n = sort_count(n_dev, n_static, cap);
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  if (base < n) {
    const int lane = threadIdx.x & 63;
#pragma unroll 4
    for (int i = 0; i < kSortItems; ++i) {
      const int64_t idx = base + i * kSortThreads + threadIdx.x;
      const bool valid = idx < n;
      const uint32_t d = valid ? (keys[idx] >> shift) & 255u : 0u;
      // aggregate equal digits within the wave before touching LDS
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
      }
      if (valid && lane == (int)__builtin_ctzll(peers)) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of len words in place, one block of 1024 threads.
// If total_out is given, the total is written there.
__global__ __launch_bounds__(1024) void k_scan_excl(uint32_t* __restrict__ data, int64_t len,
                                                    uint32_t* __restrict__ total_out) {
  __shared__ uint32_t wsum[16];
  const int tid = threadIdx.x;
  const int64_t per = (len + 1023) / 1024;
  const int64_t b = tid * per;
  const int64_t e = min(b + per, len);
  uint32_t s = 0;
  for (int64_t i = b; i < e; ++i) s += data[i];
  // block exclusive scan of s
  const int lane = tid & 63, w = tid >> 6;
  uint32_t x = s;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  if (tid == 0) {
    uint32_t acc = 0;
    for (int k = 0; k < 16; ++k) { const uint32_t t = wsum[k]; wsum[k] = acc; acc += t; }
    if (total_out) *total_out = acc;
  }
  __syncthreads();
  uint32_t run = x - s + wsum[w];
  for (int64_t i = b; i < e; ++i) { const uint32_t t = data[i]; data[i] = run; run += t; }
}

// Stable scatter of one 8-bit digit pass.  Items of a block are taken in
// rounds of 256 in index order; within a round, ranks come from wave-level
// digit matching and per-wave counts combined in wave order.
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(const uint32_t* __restrict__ kin,
                                                               const uint32_t* __restrict__ vin,
                                                               uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                               const int32_t* n_dev, int64_t n_static, int64_t cap,
                                                               int shift, const uint32_t* __restrict__ hist, int nblocks) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[4][256];
  const int n = sort_count(n_dev, n_static, cap);
  const int64_t bbase = (int64_t)blockIdx.x * kSortTile;
  if (bbase >= n) return;  // uniform for the block
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  base[tid] = hist[(int64_t)tid * nblocks + blockIdx.x];
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int round = 0; round < kSortItems; ++round) {
    const int64_t rbase = bbase + (int64_t)round * kSortThreads;
    if (rbase >= n) break;  // uniform
    const int64_t idx = rbase + tid;
    const bool valid = idx < n;
    const uint32_t key = valid ? kin[idx] : 0u;
    const uint32_t val = valid ? vin[idx] : 0u;
    const uint32_t d = (key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    // clear this wave's row, then publish the per-digit count from the leader
#pragma unroll
    for (int k = 0; k < 4; ++k) wcnt[w][lane * 4 + k] = 0;
    __builtin_amdgcn_wave_barrier();
    if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    const uint32_t c0 = wcnt[0][tid], c1 = wcnt[1][tid], c2 = wcnt[2][tid], c3 = wcnt[3][tid];
    __syncthreads();
    wcnt[0][tid] = 0;
    wcnt[1][tid] = c0;
    wcnt[2][tid] = c0 + c1;
    wcnt[3][tid] = c0 + c1 + c2;
    __syncthreads();
    if (valid) {
      const uint32_t pos = base[d] + wcnt[w][d] + rank;
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    base[tid] += c0 + c1 + c2 + c3;
    __syncthreads();
  }
}

// Per-block sums of the tile counts of depth-sorted items.
__global__ __launch_bounds__(kSortThreads) void k_count_sum(const uint32_t* __restrict__ order,
                                                            const int32_t* __restrict__ tiles, int64_t M,
                                                            uint32_t* __restrict__ bsum) {
  __shared__ uint32_t ws[4];
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  uint32_t s = 0;
  for (int i = 0; i < kSortItems; ++i) {
    const int64_t k = base + i * kSortThreads + threadIdx.x;
    if (k < M) s += (uint32_t)tiles[order[k]];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) bsum[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Emission: each thread owns kSortItems consecutive depth-sorted items,
// scans their counts within the block, and writes (tile key, item) for every
// tile of each item's rectangle, row by row.  count[0] receives I (from the
// scan total), count[1] the overflow flag.
__global__ __launch_bounds__(kSortThreads) void k_emit(const JobDev* __restrict__ jobs, const int64_t* __restrict__ item_off,
                                                       int R, const uint32_t* __restrict__ order,
                                                       const float4* __restrict__ rec,
                                                       const int32_t* __restrict__ radius,
                                                       const int32_t* __restrict__ tiles, int64_t M,
                                                       const uint32_t* __restrict__ bsum_scanned,
                                                       const uint32_t* __restrict__ total, int32_t* __restrict__ count,
                                                       int64_t cap, uint32_t* __restrict__ kout,
                                                       int32_t* __restrict__ vout) {
  __shared__ uint32_t wsum[4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t first = (int64_t)blockIdx.x * kSortTile + (int64_t)tid * kSortItems;
  uint32_t s = 0;
  for (int i = 0; i < kSortItems; ++i) {
    const int64_t k = first + i;
    if (k < M) s += (uint32_t)tiles[order[k]];
  }
  uint32_t x = s;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint32_t wofs = 0;
  for (int k = 0; k < w; ++k) wofs += wsum[k];
  uint64_t pos = (uint64_t)bsum_scanned[blockIdx.x] + wofs + (x - s);
  if (blockIdx.x == 0 && tid == 0) {
    const uint32_t I = *total;
    count[0] = (int32_t)min((int64_t)I, cap);
    count[1] = (int64_t)I > cap ? 1 : 0;
  }
  for (int i = 0; i < kSortItems; ++i) {
    const int64_t k = first + i;
    if (k >= M) break;
    const uint32_t it = order[k];
    const int nt = tiles[it];
    if (nt <= 0) continue;
    const int r = find_segment<int64_t>(item_off, R, (int64_t)it);
    const JobDev& J = jobs[r];
    const float4 a = rec[(int64_t)it * 3];
    const Rect rc = tile_rect(a.x, a.y, radius[it], J.TX, J.TY);
    for (int ty = rc.y0; ty < rc.y1; ++ty) {
      for (int tx = rc.x0; tx < rc.x1; ++tx) {
        if ((int64_t)pos < cap) {
          kout[pos] = (uint32_t)(J.tile_off + ty * J.TX + tx);
          vout[pos] = (int32_t)it;
        }
        ++pos;
      }
    }
  }
}

// [start, end) of each tile's run in the sorted instance keys.
__global__ void k_tile_ranges(const uint32_t* __restrict__ keys, const int32_t* __restrict__ count,
                              int32_t* __restrict__ range) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = count[0];
  if (k >= n) return;
  const uint32_t t = keys[k];
  if (k == 0 || keys[k - 1] != t) range[2 * (int64_t)t] = (int32_t)k;
  if (k == n - 1 || keys[k + 1] != t) range[2 * (int64_t)t + 1] = (int32_t)(k + 1);
}

}  // namespace ls

namespace ls {
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
}

// One LSD pass: histogram, scan, scatter.
static void radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, const int32_t* n_dev,
                       int64_t n_static, int64_t cap, int shift, uint32_t* hist, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_sort_hist, dim3(nblocks), dim3(kSortThreads), 0, s, kin, n_dev, n_static, cap, shift, hist,
                     nblocks);
  hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, s, hist, (int64_t)256 * nblocks, (uint32_t*)nullptr);
  hipLaunchKernelGGL(k_sort_scatter, dim3(nblocks), dim3(kSortThreads), 0, s, kin, vin, kout, vout, n_dev, n_static,
                     cap, shift, (const uint32_t*)hist, nblocks);
}

void launch_bin_sort(const JobDev* jobs, const int64_t* item_off_d, int R, int64_t M, int T, int tile_passes,
                     const float* rec, const int32_t* radius, const int32_t* tiles, int64_t cap, uint32_t* tile_of,
                     int32_t* item, int32_t* range, int32_t* count, uint32_t* dk0, uint32_t* dv0, uint32_t* dk1,
                     uint32_t* dv1, uint32_t* hist, uint32_t* bsum, uint32_t* tk, uint32_t* tv, hipStream_t s) {
  const float4* rec4 = reinterpret_cast<const float4*>(rec);
  const int nbd = (int)((M + kSortTile - 1) / kSortTile);
  hipLaunchKernelGGL(k_depth_keys, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, rec4, tiles, M, dk0, dv0);
  uint32_t *ka = dk0, *va = dv0, *kb = dk1, *vb = dv1;
  for (int shift = 0; shift < 32; shift += 8) {
    radix_pass(ka, va, kb, vb, nullptr, M, M, shift, hist, nbd, s);
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  const uint32_t* order = va;
  hipLaunchKernelGGL(k_count_sum, dim3(nbd), dim3(kSortThreads), 0, s, order, tiles, M, bsum);
  hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, s, bsum, (int64_t)nbd, bsum + nbd);
  // emission lands in the buffer that, after tile_passes ping-pongs, is the output
  uint32_t* ek = (tile_passes & 1) ? tk : tile_of;
  uint32_t* ev = (tile_passes & 1) ? tv : reinterpret_cast<uint32_t*>(item);
  uint32_t* ok = (tile_passes & 1) ? tile_of : tk;
  uint32_t* ov = (tile_passes & 1) ? reinterpret_cast<uint32_t*>(item) : tv;
  hipLaunchKernelGGL(k_emit, dim3(nbd), dim3(kSortThreads), 0, s, jobs, item_off_d, R, order, rec4, radius, tiles, M,
                     (const uint32_t*)bsum, (const uint32_t*)(bsum + nbd), count, cap, ek,
                     reinterpret_cast<int32_t*>(ev));
  const int nbt = (int)((cap + kSortTile - 1) / kSortTile);
  for (int p = 0; p < tile_passes && nbt > 0; ++p) {
    radix_pass(ek, ev, ok, ov, count, 0, cap, 8 * p, hist, nbt, s);
    std::swap(ek, ok);
    std::swap(ev, ov);
  }
  launch_fill_i32(range, 2 * (int64_t)T, 0, s);
  if (cap > 0)
    hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, (const uint32_t*)tile_of,
                       (const int32_t*)count, range);
}
}  // namespace ls

// Opacity pruning of a submap after mapping (supplement, Implementation
// Details, submap update): every Gaussian whose opacity is below o_thre is
// removed and the others are compacted, in order, into new arrays.
//
// The keep test is taken on the stored FP32 logit against the FP32 rounding
// of logit(o_thre) (sigmoid is increasing), so it needs no transcendental and
// its decisions are reproducible: keep <=> logit >= tau (NaN is pruned).
//
// Three launches: per-tile keep counts, one block scanning the counts into
// tile offsets (and the total), then the scatter, which re-derives each
// item's rank within its tile from ballots and copies every component of the
// kept items.  Rows of the outputs are `count` floats apart, so they come out
// in the ls_gaussians layout for the new Gaussian count.
#include <algorithm>

#include "kernels.h"

namespace ls {

constexpr int kPruneThreads = 256;
// Items per thread: 4 for large sets; 1 below kPruneSmall items, so that a
// submap-sized set still spreads over more blocks than the GPU has CUs.
constexpr int kPruneSmall = 1 << 20;
__host__ __device__ constexpr int prune_tile(int rounds) { return kPruneThreads * rounds; }

__device__ __forceinline__ bool prune_keep(float w, float tau) { return w >= tau; }

template <int kPruneRounds>
__global__ __launch_bounds__(kPruneThreads) void k_prune_count(const float* __restrict__ logit, int n, float tau,
                                                               int32_t* __restrict__ tile_count) {
  const int64_t base = (int64_t)blockIdx.x * prune_tile(kPruneRounds);
  int c = 0;
#pragma unroll
  for (int r = 0; r < kPruneRounds; ++r) {
    const int64_t i = base + r * kPruneThreads + threadIdx.x;
    c += (i < n && prune_keep(logit[i], tau)) ? 1 : 0;
  }
  __shared__ int ws[kPruneThreads / 64];
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) tile_count[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// One block: exclusive scan of the tile counts into offsets, total to *count.
__global__ __launch_bounds__(1024) void k_prune_scan(const int32_t* __restrict__ tile_count, int ntiles,
                                                     int32_t* __restrict__ tile_off, int32_t* __restrict__ count) {
  __shared__ int32_t wsum[16];
  const int per = (ntiles + 1023) / 1024;
  const int b = threadIdx.x * per, e = min(b + per, ntiles);
  int32_t s = 0;
  for (int i = b; i < e; ++i) s += tile_count[i];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t x = s;
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int32_t run = x - s;
  for (int k = 0; k < w; ++k) run += wsum[k];
  for (int i = b; i < e; ++i) {
    tile_off[i] = run;
    run += tile_count[i];
  }
  if (threadIdx.x == 1023) *count = run;
}

template <int kPruneRounds>
__global__ __launch_bounds__(kPruneThreads) void k_prune_scatter(const float* __restrict__ logit, int n, float tau,
                                                                 const int32_t* __restrict__ tile_off,
                                                                 const int32_t* __restrict__ count, PruneArrays arr,
                                                                 int32_t* __restrict__ kept) {
  __shared__ int32_t wcnt[kPruneRounds][kPruneThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * prune_tile(kPruneRounds);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  bool keep[kPruneRounds];
  int rank[kPruneRounds];
#pragma unroll
  for (int r = 0; r < kPruneRounds; ++r) {
    const int64_t i = base + r * kPruneThreads + threadIdx.x;
    keep[r] = i < n && prune_keep(logit[i], tau);
    const uint64_t m = __ballot(keep[r]);
    rank[r] = __popcll(m & below);
    if (lane == 0) wcnt[r][w] = __popcll(m);
  }
  __syncthreads();
  const int64_t stride = count[0];
  int64_t pos[kPruneRounds];
  int run = tile_off[blockIdx.x];
#pragma unroll
  for (int r = 0; r < kPruneRounds; ++r) {
    int before = run;
    for (int k = 0; k < w; ++k) before += wcnt[r][k];
    pos[r] = before + rank[r];
    if (keep[r]) kept[pos[r]] = (int32_t)(base + r * kPruneThreads + threadIdx.x);
    run += (wcnt[r][0] + wcnt[r][1]) + (wcnt[r][2] + wcnt[r][3]);
  }
  // one row at a time: the four rounds' loads are issued before their stores
  for (int a = 0; a < kPruneArrays; ++a) {
    if (a >= arr.count) break;  // uniform
    const float* __restrict__ src = arr.src[a];
    float* __restrict__ dst = arr.dst[a];
    for (int c = 0; c < arr.comp[a]; ++c) {
      float v[kPruneRounds];
#pragma unroll
      for (int r = 0; r < kPruneRounds; ++r)
        v[r] = keep[r] ? src[(int64_t)c * n + base + r * kPruneThreads + threadIdx.x] : 0.f;
#pragma unroll
      for (int r = 0; r < kPruneRounds; ++r)
        if (keep[r]) dst[c * stride + pos[r]] = v[r];
    }
  }
}

static int prune_rounds(int n) { return n < kPruneSmall ? 1 : 4; }

size_t prune_workspace_bytes(int n) {
  const size_t tiles = (size_t)std::max((n + prune_tile(prune_rounds(n)) - 1) / prune_tile(prune_rounds(n)), 1);
  return 2 * ((4 * tiles + 255) & ~(size_t)255);
}

template <int kRounds>
static void launch_prune_rounds(const float* logit, int n, float tau, const PruneArrays& arr, int32_t* kept,
                                int32_t* count, void* work, hipStream_t s) {
  const int tiles = std::max((n + prune_tile(kRounds) - 1) / prune_tile(kRounds), 1);
  int32_t* tile_count = static_cast<int32_t*>(work);
  int32_t* tile_off = tile_count + (((4 * (size_t)tiles + 255) & ~(size_t)255) / 4);
  hipLaunchKernelGGL(k_prune_count<kRounds>, dim3(tiles), dim3(kPruneThreads), 0, s, logit, n, tau, tile_count);
  hipLaunchKernelGGL(k_prune_scan, dim3(1), dim3(1024), 0, s, (const int32_t*)tile_count, tiles, tile_off, count);
  if (n > 0)
    hipLaunchKernelGGL(k_prune_scatter<kRounds>, dim3(tiles), dim3(kPruneThreads), 0, s, logit, n, tau,
                       (const int32_t*)tile_off, (const int32_t*)count, arr, kept);
}

void launch_prune(const float* logit, int n, float tau, const PruneArrays& arr, int32_t* kept, int32_t* count,
                  void* work, hipStream_t s) {
  if (prune_rounds(n) == 1)
    launch_prune_rounds<1>(logit, n, tau, arr, kept, count, work, s);
  else
    launch_prune_rounds<4>(logit, n, tau, arr, kept, count, work, s);
}

}  // namespace ls

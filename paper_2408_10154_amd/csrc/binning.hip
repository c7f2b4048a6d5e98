// Tile binning on gfx950: depth keys, LSD radix sorts (stable; 8-bit digits),
// count scan, instance emission in depth order, tile ranges.
//
// Order of the final list: (tile, FP32 depth bits, item).  It is produced as
// a stable depth sort of the items (ties keep ascending item order), then
// emission of each item's tiles in that order, then a stable sort of the
// instances by tile key.
#include "common.h"

#include <algorithm>
#include <cstdlib>

namespace ls {

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = i; k < n; k += stride) p[k] = v;
}

__device__ __forceinline__ int sort_count(const int32_t* n_dev, int64_t n_static, int64_t cap) {
  int64_t n = n_static;
  if (n_dev) n = min((int64_t)n_dev[0], cap);
  return (int)n;
}

// Sort blocks that hold keys (n keys, rounds x 256 per block): the histogram
// columns of later blocks are neither written nor read (a capacity sized for
// the worst case leaves most blocks of a pass idle).
__device__ __forceinline__ int active_blocks(int n, int rounds) {
  return (int)(((int64_t)n + (int64_t)rounds * kSortThreads - 1) / ((int64_t)rounds * kSortThreads));
}

// Digit histogram of one sort block's keys (kSortItems registers per thread,
// rounds of them valid, nb keys in all) into LDS h, then to
// hist[d * nblocks + block] (digit-major).  Equal digits within a wave are
// merged before the LDS atomic.
template <int kBits>
__device__ __forceinline__ void block_digit_hist(const uint32_t (&key)[kSortItems], int rounds, int nb, int shift,
                                                 uint32_t* h, uint32_t* __restrict__ hist, int nblocks) {
  constexpr int kBins = 1 << kBits;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    if (r < rounds && r * kSortThreads < nb) {  // uniform; a guard, not a break, so the loop unrolls
      const bool valid = r * kSortThreads + (int)threadIdx.x < nb;
      const uint32_t d = (key[r] >> shift) & (uint32_t)(kBins - 1);
      // aggregate equal digits within the wave before touching LDS
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < kBits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
      }
      if (valid && lane == (int)__builtin_ctzll(peers)) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kBins; i += kSortThreads) hist[(int64_t)i * nblocks + blockIdx.x] = h[i];
}

// Per-block digit histogram of kBits-bit digits, stored digit-major:
// hist[d * nblocks + block], for the blocks that hold keys.  Every key of the
// block is loaded before any is counted, so the block waits for memory once,
// not once per round.
template <int kBits>
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const uint32_t* __restrict__ keys, const int32_t* n_dev,
                                                            int64_t n_static, int64_t cap, int shift,
                                                            uint32_t* __restrict__ hist, int nblocks, int rounds) {
  constexpr int kBins = 1 << kBits;
  __shared__ uint32_t h[kBins];
  const int n = sort_count(n_dev, n_static, cap);
  const int64_t base = (int64_t)blockIdx.x * rounds * kSortThreads;
  if (base >= n) return;  // uniform for the block: no keys, no column
  for (int i = threadIdx.x; i < kBins; i += kSortThreads) h[i] = 0;
  const int nb = (int)min((int64_t)rounds * kSortThreads, (int64_t)n - base);
  uint32_t key[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int i = r * kSortThreads + threadIdx.x;
    key[r] = (r < rounds && i < nb) ? keys[base + i] : 0u;
  }
  __syncthreads();
  block_digit_hist<kBits>(key, rounds, nb, shift, h, hist, nblocks);
}

// Depth keys of one sort block's items (FP32 depth bits: positive depths
// order like their bits; culled items get 0xFFFFFFFF and sort last), item ids
// as values, and the histogram of the first radix pass's digits, so that pass
// needs no histogram launch of its own.
template <int kBits>
__global__ __launch_bounds__(kSortThreads) void k_depth_keys(const float4* __restrict__ rec,
                                                             const int32_t* __restrict__ tiles, int64_t M,
                                                             uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                             uint32_t* __restrict__ hist, int nblocks, int rounds) {
  constexpr int kBins = 1 << kBits;
  __shared__ uint32_t h[kBins];
  for (int i = threadIdx.x; i < kBins; i += kSortThreads) h[i] = 0;
  const int64_t base = (int64_t)blockIdx.x * rounds * kSortThreads;
  const int nb = base < M ? (int)min((int64_t)rounds * kSortThreads, M - base) : 0;
  uint32_t key[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int i = r * kSortThreads + threadIdx.x;
    key[r] = 0u;
    if (r < rounds && i < nb) {
      const int64_t it = base + i;
      key[r] = tiles[it] > 0 ? __float_as_uint(rec[it * 3 + 1].z) : 0xFFFFFFFFu;
      keys[it] = key[r];
      vals[it] = (uint32_t)it;
    }
  }
  __syncthreads();
  block_digit_hist<kBits>(key, rounds, nb, 0, h, hist, nblocks);
}

// Block-wide exclusive scan of one value per thread (256 threads); returns
// the exclusive prefix and writes the block total to *total.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* wsum, uint32_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint32_t wofs = 0;
  for (int k = 0; k < w; ++k) wofs += wsum[k];
  const uint32_t tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  __syncthreads();
  *total = tot;
  return wofs + x - v;
}

// Exclusive scan of each row of a [rows][len] array in place, one 256-thread
// block per row; row totals go to totals[row].  Only the columns of the sort
// blocks that hold keys are scanned (n keys, rounds x 256 per block).
__global__ __launch_bounds__(256) void k_scan_rows(uint32_t* __restrict__ data, int64_t stride,
                                                   uint32_t* __restrict__ totals, const int32_t* n_dev,
                                                   int64_t n_static, int64_t cap, int rounds) {
  __shared__ uint32_t wsum[4];
  uint32_t* row = data + (int64_t)blockIdx.x * stride;
  const int64_t len = min(stride, (int64_t)active_blocks(sort_count(n_dev, n_static, cap), rounds));
  const int64_t per = (len + 255) / 256;
  const int64_t b = threadIdx.x * per;
  const int64_t e = min(b + per, len);
  uint32_t s = 0;
  for (int64_t i = b; i < e; ++i) s += row[i];
  uint32_t tot;
  uint32_t run = block_excl_scan(s, wsum, &tot);
  for (int64_t i = b; i < e; ++i) { const uint32_t t = row[i]; row[i] = run; run += t; }
  if (threadIdx.x == 0) totals[blockIdx.x] = tot;
}

// Stable scatter of one kBits-bit digit pass.  The block's keys (rounds x
// 256 consecutive positions) are split into four consecutive quarters, one
// per wave, each taken 64 at a time in order:
//  - every wave ranks its own keys alone: per 64 keys, a ballot match gives
//    each key its rank among equal digits, and the wave's running count of
//    that digit (its own LDS row) the number of earlier ones; the leader of
//    each digit present adds the group's count.  No barrier until the wave
//    has ranked all its keys;
//  - one thread per digit then turns the four wave counts into the digit's
//    place in LDS order (digits ascending, then waves in order) and its
//    global run start (the scanned histogram entry plus the digit totals'
//    block-wide scan);
//  - each key goes to LDS at its wave's base for its digit plus its rank, so
//    LDS holds the block's keys ordered by digit and, within a digit, by
//    position: the pass is stable;
//  - the block writes its keys out in LDS order: item i of digit d goes to
//    global base(d) - local base(d) + i, so neighbouring threads write
//    neighbouring addresses along each digit's run.
template <int kBits>
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(const uint32_t* __restrict__ kin,
                                                               const uint32_t* __restrict__ vin,
                                                               uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                               const int32_t* n_dev, int64_t n_static, int64_t cap,
                                                               int shift, const uint32_t* __restrict__ hist, int nblocks,
                                                               const uint32_t* __restrict__ digit_total, int rounds) {
  constexpr int kBins = 1 << kBits;
  constexpr int kPer = kBins >= kSortThreads ? kBins / kSortThreads : 1;  // digits per thread in the set-up
  static_assert(kBins % kSortThreads == 0 || kSortThreads % kBins == 0, "digits and threads must divide");
  static_assert(kSortThreads == 256, "four waves per block");
  __shared__ uint32_t wcnt[4][kBins];  // per wave: running count of each digit, then the wave's LDS base for it
  __shared__ uint32_t delta[kBins];    // global minus local start of each digit's run (mod 2^32)
  __shared__ uint32_t wsum[4];
  __shared__ uint32_t sk[kSortTile], sv[kSortTile];
  const int n = sort_count(n_dev, n_static, cap);
  const int64_t bbase = (int64_t)blockIdx.x * rounds * kSortThreads;
  if (bbase >= n) return;  // uniform for the block
  const int nb = (int)min((int64_t)rounds * kSortThreads, (int64_t)n - bbase);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wpos = w * rounds * 64;  // the wave's first position in the block
  uint32_t key[kSortItems], val[kSortItems], rk[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int i = wpos + r * 64 + lane;
    const bool ok = r < rounds && i < nb;
    key[r] = ok ? kin[bbase + i] : 0u;
    val[r] = ok ? vin[bbase + i] : 0u;
    rk[r] = 0u;
  }
  for (int d = lane; d < kBins; d += 64) wcnt[w][d] = 0u;
  __builtin_amdgcn_wave_barrier();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    if (r < rounds && wpos + r * 64 < nb) {  // uniform for the wave; a guard, not a break, so the loop unrolls
      const bool valid = wpos + r * 64 + lane < nb;
      const uint32_t d = (key[r] >> shift) & (uint32_t)(kBins - 1);
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < kBits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
      }
      const uint32_t rank = (uint32_t)__popcll(peers & lt);
      const uint32_t before = valid ? wcnt[w][d] : 0u;
      rk[r] = before + rank;
      if (valid && rank == 0) wcnt[w][d] = before + (uint32_t)__popcll(peers);
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  {
    // threads 0 .. kBins / kPer - 1 hold kPer digits each (fewer digits than
    // threads: the other threads add zeros to the scans)
    const bool has = tid * kPer < kBins;
    uint32_t tot[kPer], cnt[kPer], here[kPer], c0[kPer], c1[kPer], c2[kPer];
    uint32_t gsum = 0, lsum = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int d = tid * kPer + k;
      tot[k] = cnt[k] = here[k] = c0[k] = c1[k] = c2[k] = 0u;
      if (has) {
        c0[k] = wcnt[0][d];
        c1[k] = wcnt[1][d];
        c2[k] = wcnt[2][d];
        cnt[k] = c0[k] + c1[k] + c2[k] + wcnt[3][d];
        here[k] = hist[(int64_t)d * nblocks + blockIdx.x];
        tot[k] = digit_total[d];
      }
      gsum += tot[k];
      lsum += cnt[k];
    }
    uint32_t all;
    uint32_t grun = block_excl_scan(gsum, wsum, &all);
    uint32_t lrun = block_excl_scan(lsum, wsum, &all);
    if (has) {
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int d = tid * kPer + k;
        delta[d] = grun + here[k] - lrun;
        wcnt[0][d] = lrun;
        wcnt[1][d] = lrun + c0[k];
        wcnt[2][d] = lrun + c0[k] + c1[k];
        wcnt[3][d] = lrun + c0[k] + c1[k] + c2[k];
        grun += tot[k];
        lrun += cnt[k];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    if (r < rounds && wpos + r * 64 + lane < nb) {
      const uint32_t d = (key[r] >> shift) & (uint32_t)(kBins - 1);
      const uint32_t pos = wcnt[w][d] + rk[r];
      sk[pos] = key[r];
      sv[pos] = val[r];
    }
  }
  __syncthreads();
  for (int i = tid; i < nb; i += kSortThreads) {
    const uint32_t k = sk[i];
    const uint32_t pos = delta[(k >> shift) & (uint32_t)(kBins - 1)] + (uint32_t)i;
    kout[pos] = k;
    vout[pos] = sv[i];
  }
}

// Compaction of the items that have tiles before the depth sort (most items
// of a registration view lie outside it): kept items per sort block ...
__global__ __launch_bounds__(kSortThreads) void k_keep_count(const int32_t* __restrict__ tiles, int64_t M, int rounds,
                                                             uint32_t* __restrict__ bsum) {
  __shared__ uint32_t ws[4];
  const int64_t base = (int64_t)blockIdx.x * rounds * kSortThreads;
  uint32_t c = 0;
  for (int i = 0; i < rounds; ++i) {
    const int64_t k = base + i * kSortThreads + threadIdx.x;
    if (k < M && tiles[k] > 0) ++c;
  }
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) bsum[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// ... then their depth keys and item ids, written in item order from the
// block's offset (the sum of the preceding blocks' counts, formed here); block
// 0 writes the kept total to *nkeep.  The stable sort then orders them exactly
// as the uncompacted keys (where culled items sort last).
__global__ __launch_bounds__(kSortThreads) void k_depth_keys_compact(const float4* __restrict__ rec,
                                                                     const int32_t* __restrict__ tiles, int64_t M,
                                                                     int rounds, const uint32_t* __restrict__ bsum,
                                                                     int nbd, uint32_t* __restrict__ keys,
                                                                     uint32_t* __restrict__ vals,
                                                                     int32_t* __restrict__ nkeep) {
  __shared__ uint32_t wsum[4], wtot[4];
  const int64_t base = (int64_t)blockIdx.x * rounds * kSortThreads;
  const int upto = blockIdx.x == 0 ? nbd : (int)blockIdx.x;
  uint32_t before = 0, total = 0;
  for (int b = threadIdx.x; b < upto; b += kSortThreads) {
    const uint32_t v = bsum[b];
    total += v;
    if (b < (int)blockIdx.x) before += v;
  }
  for (int off = 32; off > 0; off >>= 1) {
    before += __shfl_xor(before, off, 64);
    total += __shfl_xor(total, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    wsum[threadIdx.x >> 6] = before;
    wtot[threadIdx.x >> 6] = total;
  }
  __syncthreads();
  uint32_t run = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  if (blockIdx.x == 0 && threadIdx.x == 0) *nkeep = (int32_t)(wtot[0] + wtot[1] + wtot[2] + wtot[3]);
  // every round's keep flags first; per wave a ballot gives each lane its rank
  // and the wave's count; one barrier, then each lane's place follows from
  // the counts of the earlier rounds and waves (item order kept)
  __shared__ uint32_t wcnt[kSortItems][4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint64_t bal[kSortItems];
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const int64_t k = base + i * kSortThreads + threadIdx.x;
    const bool keep = i < rounds && k < M && tiles[k] > 0;
    bal[i] = __ballot(keep);
    if (i < rounds && lane == 0) wcnt[i][w] = (uint32_t)__popcll(bal[i]);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    if (i >= rounds) break;
    uint32_t pre = 0;
    for (int u = 0; u < w; ++u) pre += wcnt[i][u];
    if ((bal[i] >> lane) & 1ull) {
      const uint32_t pos = run + pre + (uint32_t)__popcll(bal[i] & lt);
      const int64_t k = base + i * kSortThreads + threadIdx.x;
      keys[pos] = __float_as_uint(rec[k * 3 + 1].z);
      vals[pos] = (uint32_t)k;
    }
    run += (wcnt[i][0] + wcnt[i][1]) + (wcnt[i][2] + wcnt[i][3]);
  }
}

// Inclusive prefix sum over the 64 lanes (DPP: shifts within 16-lane rows,
// then the row ends broadcast to the later rows); 0 is the identity.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v) {
  int x = (int)v;
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15 -> rows 1, 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31 -> rows 2, 3
  return (uint32_t)x;
}

// Items in the depth order: M, or the kept count when the items were
// compacted before the sort.
__device__ __forceinline__ int64_t order_len(int64_t M, const int32_t* n_dev) {
  return n_dev ? min((int64_t)n_dev[0], M) : M;
}

// Per-block (rounds x 256 items) sums of the tile counts of depth-sorted items.
__global__ __launch_bounds__(kSortThreads) void k_count_sum(const uint32_t* __restrict__ order,
                                                            const int32_t* __restrict__ tiles, int64_t M,
                                                            const int32_t* n_dev, int rounds,
                                                            uint32_t* __restrict__ bsum) {
  __shared__ uint32_t ws[4];
  const int64_t base = (int64_t)blockIdx.x * rounds * kSortThreads;
  const int64_t n = order_len(M, n_dev);
  if (base >= n) {  // no item here
    if (threadIdx.x == 0) bsum[blockIdx.x] = 0;
    return;
  }
  uint32_t s = 0;
  for (int i = 0; i < rounds; ++i) {
    const int64_t k = base + i * kSortThreads + threadIdx.x;
    if (k < n) s += (uint32_t)tiles[order[k]];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) bsum[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Exclusive offsets of every depth-sorted item: block offset (the sum of the
// preceding block sums, formed here rather than by a scan launch) plus the
// in-block prefix, 16 rounds of 256 items in order.  The item whose instance
// range holds instance m * span (m < nspan) is recorded in first[m].
// Block 0 also writes count = {min(I, cap), I > cap, min(I, INT32_MAX), 0}.
__global__ __launch_bounds__(kSortThreads) void k_offsets(const uint32_t* __restrict__ order,
                                                          const int32_t* __restrict__ tiles, int64_t M,
                                                          const int32_t* n_dev, const uint32_t* __restrict__ bsum,
                                                          int nbd,
                                                          uint32_t* __restrict__ offs, int32_t* __restrict__ count,
                                                          int64_t cap, int rounds, uint32_t* __restrict__ first,
                                                          int64_t span, int64_t nspan) {
  __shared__ uint32_t wsum[4];
  __shared__ uint64_t wtot[4];
  const int64_t base = (int64_t)blockIdx.x * rounds * kSortThreads;
  const int64_t n = order_len(M, n_dev);
  if (blockIdx.x != 0 && base >= n) return;  // no item here (block 0 writes the counts)
  // the offset of this block (and, for block 0, the total over all blocks)
  const int upto = blockIdx.x == 0 ? nbd : (int)blockIdx.x;
  uint64_t before = 0, total = 0;
  for (int b = threadIdx.x; b < upto; b += kSortThreads) {
    const uint64_t v = bsum[b];
    total += v;
    if (b < (int)blockIdx.x) before += v;
  }
  for (int off = 32; off > 0; off >>= 1) {
    before += __shfl_xor(before, off, 64);
    total += __shfl_xor(total, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    wsum[threadIdx.x >> 6] = (uint32_t)before;
    wtot[threadIdx.x >> 6] = total;
  }
  __syncthreads();
  uint32_t run = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  const uint64_t I64 = wtot[0] + wtot[1] + wtot[2] + wtot[3];
  // every round's counts first, an inclusive scan per wave and round (DPP),
  // the wave totals to LDS, one barrier; then each lane's offset follows from
  // the totals of the earlier rounds and waves
  __shared__ uint32_t wt[kSortItems][4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t c[kSortItems], x[kSortItems];
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const int64_t k = base + i * kSortThreads + threadIdx.x;
    c[i] = (i < rounds && k < n) ? (uint32_t)tiles[order[k]] : 0u;
  }
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    if (i >= rounds) break;
    const uint32_t incl = wave_incl_sum(c[i]);
    x[i] = incl - c[i];
    if (lane == 63) wt[i][w] = incl;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    if (i >= rounds) break;
    uint32_t pre = 0;
    for (int u = 0; u < w; ++u) pre += wt[i][u];
    const int64_t k = base + i * kSortThreads + threadIdx.x;
    if (k < n) {
      const int64_t o = (int64_t)run + pre + x[i];
      offs[k] = (uint32_t)o;
      for (int64_t m = (o + span - 1) / span; m < nspan && m * span < o + c[i]; ++m)
        first[m] = (uint32_t)k;
    }
    run += (wt[i][0] + wt[i][1]) + (wt[i][2] + wt[i][3]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int64_t I = (int64_t)I64;
    count[0] = (int32_t)min(I, cap);
    count[1] = I > cap ? 1 : 0;
    count[2] = (int32_t)min(I, (int64_t)INT32_MAX);
    count[3] = 0;
  }
}

// Inclusive prefix maximum over the 64 lanes (DPP: shifts within 16-lane
// rows, then the row ends broadcast to the later rows); -1 is the identity.
__device__ __forceinline__ int wave_incl_max(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x111, 0xF, 0xF, false));  // row_shr:1
  v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x112, 0xF, 0xF, false));  // row_shr:2
  v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x114, 0xF, 0xF, false));  // row_shr:4
  v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x118, 0xF, 0xF, false));  // row_shr:8
  v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x142, 0xA, 0xF, false));  // row_bcast:15 -> rows 1, 3
  v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x143, 0xC, 0xF, false));  // row_bcast:31 -> rows 2, 3
  return v;
}

// Emission of the tile instances in depth order, one wave per span of
// consecutive instances (so every wave has the same work, however many tiles
// its items cover).  The wave takes the items from the span's first
// one on, 64 at a time, lane l item kb + l: its instance offset, its tile
// rectangle and the key of the rectangle's first tile.  It fills the span 64
// instances at a time, lane l writing instance W0 + l, so every store is one
// contiguous run; windows stop at the end of the loaded items, and the next
// 64 items start there.  The owner of an instance is the last item that starts
// at or before it: items starting inside the window mark their start position
// (LDS), a prefix maximum over the lanes carries each mark forward, and
// positions before the first start keep the previous owner (at first, lane 0:
// the item that holds the span's first instance).  Within its owner's
// rectangle, instance q lies in row q / width (row by row, as the tiles are
// counted).  Instances at or beyond the capacity are not written.  The
// kEmitWaves spans of a block are the positions of one block of the first
// tile radix pass, whose histogram of the keys' low `dbits` bits the block
// counts as it writes (LDS) and stores digit-major in
// hist[d * gridDim.x + block], as the histogram kernel would.
__global__ __launch_bounds__(64 * kEmitWaves) void k_emit(const JobDev* __restrict__ jobs, const int64_t* __restrict__ item_off,
                                              int R, const uint32_t* __restrict__ order,
                                              const float4* __restrict__ rec, const int32_t* __restrict__ radius,
                                              const int32_t* __restrict__ tiles, int64_t M_all, const int32_t* n_dev,
                                              const uint32_t* __restrict__ offs, const int32_t* __restrict__ count,
                                              const uint32_t* __restrict__ first, int64_t span_len, int64_t nspan,
                                              uint32_t* __restrict__ kout, int32_t* __restrict__ vout,
                                              uint32_t* __restrict__ hist, int dbits) {
  static_assert(kTileDigitBits <= 8 && 64 * kEmitWaves >= 256, "a histogram bin per thread of the first 256");
  const uint32_t dmask = (1u << dbits) - 1u;
  __shared__ int marks[kEmitWaves][64];
  __shared__ uint32_t h[256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t I = count[0];  // already clamped to the capacity
  if ((int64_t)blockIdx.x * kEmitWaves * span_len >= I) return;  // uniform: no instance, no histogram column
  if (threadIdx.x < 256) h[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t span = (int64_t)blockIdx.x * kEmitWaves + w;
  const int64_t M = order_len(M_all, n_dev);
  const bool work = span < nspan && span * span_len < I;  // uniform for the wave
  const int64_t iend = work ? min((span + 1) * span_len, I) : 0;
  int64_t kb = work ? (int64_t)first[span] : M;
  int64_t W0 = span * span_len;
  while (W0 < iend && kb < M) {
    const int64_t k = kb + lane;
    const int last = (int)min((int64_t)63, M - 1 - kb);  // last lane with an item
    uint32_t off = 0xFFFFFFFFu, it = 0;
    int nt = 0, base_key = 0, stride = 0, wdt = 1;
    if (k < M) {
      off = offs[k];
      it = order[k];
      nt = tiles[it];
      if (nt > 0) {
        const int r = find_segment<int64_t>(item_off, R, (int64_t)it);
        const JobDev& J = jobs[r];
        const float4 a = rec[(int64_t)it * 3];
        const Rect rc = tile_rect(a.x, a.y, radius[it], J.TX, J.TY);
        wdt = rc.x1 - rc.x0;
        base_key = J.tile_off + rc.y0 * J.TX + rc.x0;
        stride = J.TX - wdt;
      }
    }
    const float inv = 1.0f / (float)wdt;
    const int64_t cend = min((int64_t)(uint32_t)__builtin_amdgcn_readlane((int)(off + (uint32_t)nt), last), iend);
    int carry = 0;
    while (W0 < cend) {
      marks[w][lane] = -1;
      const int64_t rel = (int64_t)off - W0;
      if (nt > 0 && rel >= 0 && rel < 64) marks[w][(int)rel] = lane;
      __builtin_amdgcn_wave_barrier();
      int o = wave_incl_max(marks[w][lane]);
      o = o < 0 ? carry : o;
      carry = __builtin_amdgcn_readlane(o, 63);
      const int64_t i = W0 + lane;
      const int o_key = __shfl(base_key, o, 64), o_stride = __shfl(stride, o, 64), o_wdt = __shfl(wdt, o, 64);
      const float o_inv = __shfl(inv, o, 64);
      const uint32_t o_off = (uint32_t)__shfl((int)off, o, 64), o_it = (uint32_t)__shfl((int)it, o, 64);
      if (i < cend) {
        const int q = (int)(i - (int64_t)o_off);
        int dy = (int)((float)q * o_inv);
        if ((dy + 1) * o_wdt <= q) ++dy;
        else if (dy * o_wdt > q) --dy;
        const uint32_t key = (uint32_t)(o_key + dy * o_stride + q);
        kout[i] = key;
        vout[i] = (int32_t)o_it;
        atomicAdd(&h[key & dmask], 1u);
      }
      __builtin_amdgcn_wave_barrier();
      W0 = min(W0 + 64, cend);
    }
    kb += 64;
  }
  __syncthreads();
  if (threadIdx.x <= dmask) hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// [start, end) of each tile's run in the sorted instance keys, for every one
// of the T tiles, empty tiles [0, 0).  A thread takes 4 consecutive keys
// (one 16-byte load, and its neighbours' edge keys); at the start of a run it
// also clears the tiles between the previous run's tile and its own (the
// first key those before the first run, the last key those after the last
// run).  With no instances, thread t clears tiles 4t..4t+3.  The grid covers
// ceil(max(capacity, T) / 4) threads (keys not 16-byte aligned are read one
// by one).
__global__ void k_tile_ranges(const uint32_t* __restrict__ keys, const int32_t* __restrict__ count,
                              int32_t* __restrict__ range, int T) {
  const int64_t k0 = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
  const int64_t n = count[0];
  if (n == 0) {
    for (int64_t u = k0; u < k0 + 4 && u < T; ++u) {
      range[2 * u] = 0;
      range[2 * u + 1] = 0;
    }
    return;
  }
  if (k0 >= n) return;
  uint32_t kk[6];  // keys k0 - 1 .. k0 + 4 (valid where 0 <= index < n)
  kk[0] = k0 > 0 ? keys[k0 - 1] : 0u;
  if (k0 + 4 <= n && (reinterpret_cast<uintptr_t>(keys) & 15) == 0) {
    const uint4 q = *reinterpret_cast<const uint4*>(keys + k0);
    kk[1] = q.x;
    kk[2] = q.y;
    kk[3] = q.z;
    kk[4] = q.w;
  } else {
    for (int j = 0; j < 4; ++j) kk[1 + j] = k0 + j < n ? keys[k0 + j] : 0u;
  }
  kk[5] = k0 + 4 < n ? keys[k0 + 4] : 0u;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t k = k0 + j;
    if (k >= n) break;
    const int64_t t = kk[1 + j];
    if (k == 0 || kk[j] != (uint32_t)t) {
      for (int64_t u = k == 0 ? 0 : (int64_t)kk[j] + 1; u < t; ++u) {
        range[2 * u] = 0;
        range[2 * u + 1] = 0;
      }
      range[2 * t] = (int32_t)k;
    }
    if (k == n - 1 || kk[2 + j] != (uint32_t)t) {
      range[2 * t + 1] = (int32_t)(k + 1);
      if (k == n - 1)
        for (int64_t u = t + 1; u < T; ++u) {
          range[2 * u] = 0;
          range[2 * u + 1] = 0;
        }
    }
  }
}

}  // namespace ls

namespace ls {
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
}

// One LSD pass of kBits-bit digits: histogram, per-digit row scan (row totals
// to digit_total), scatter (which scans the digit totals itself).
template <int kBits>
static void radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, const int32_t* n_dev,
                       int64_t n_static, int64_t cap, int shift, uint32_t* hist, uint32_t* digit_total, int nblocks,
                       int rounds, hipStream_t s, bool hist_done = false) {
  if (!hist_done)
    hipLaunchKernelGGL(k_sort_hist<kBits>, dim3(nblocks), dim3(kSortThreads), 0, s, kin, n_dev, n_static, cap, shift,
                       hist, nblocks, rounds);
  hipLaunchKernelGGL(k_scan_rows, dim3(1 << kBits), dim3(256), 0, s, hist, (int64_t)nblocks, digit_total, n_dev,
                     n_static, cap, rounds);
  hipLaunchKernelGGL(k_sort_scatter<kBits>, dim3(nblocks), dim3(kSortThreads), 0, s, kin, vin, kout, vout, n_dev,
                     n_static, cap, shift, (const uint32_t*)hist, nblocks, (const uint32_t*)digit_total, rounds);
}

int launch_radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n, int bits,
                            uint32_t* hist, uint32_t* digit_total, hipStream_t s) {
  if (n <= 0) return 0;
  const int rd = sort_rounds(n), nb = (int)sort_blocks(n);
  uint32_t *ka = k0, *va = v0, *kb = k1, *vb = v1;
  int passes = 0;
  for (int shift = 0; shift < bits; shift += 8, ++passes) {
    radix_pass<8>(ka, va, kb, vb, nullptr, n, n, shift, hist, digit_total, nb, rd, s);
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  return passes & 1;
}

// Compaction before the depth sort for batches of at least 1 M items (the
// registration views, where most items are culled); the environment variable
// LS_COMPACT=0 / 1 forces it off / on (read at every launch; for tests and
// measurements).
static bool compact_items(int64_t M) {
  const char* e = std::getenv("LS_COMPACT");
  if (e && (e[0] == '0' || e[0] == '1') && e[1] == '\0') return e[0] == '1';
  return M >= (int64_t)1 << 20;
}

void launch_bin_sort(const JobDev* jobs, const int64_t* item_off_d, int R, int64_t M, int T, int tile_bits,
                     const float* rec, const int32_t* radius, const int32_t* tiles, int64_t cap, uint32_t* tile_of,
                     int32_t* item, int32_t* range, int32_t* count, uint32_t* dk0, uint32_t* dv0, uint32_t* dk1,
                     uint32_t* dv1, uint32_t* hist, uint32_t* bsum, uint32_t* tk, uint32_t* tv, hipStream_t s) {
  const float4* rec4 = reinterpret_cast<const float4*>(rec);
  const int rd = sort_rounds(M), nbd = (int)sort_blocks(M);
  const int npass = tile_passes(tile_bits), tbits = tile_digit_bits(tile_bits);
  uint32_t* digit_base = bsum + nbd + 8;  // digit totals (up to kMaxSortBins) after the block sums
  // large batches sort only the items with tiles; the kept count sits in a
  // spare word after the block sums
  const bool compact = compact_items(M);
  int32_t* nkeep = compact ? reinterpret_cast<int32_t*>(bsum + nbd) : nullptr;
  if (compact) {
    hipLaunchKernelGGL(k_keep_count, dim3(nbd), dim3(kSortThreads), 0, s, tiles, M, rd, bsum);
    hipLaunchKernelGGL(k_depth_keys_compact, dim3(nbd), dim3(kSortThreads), 0, s, rec4, tiles, M, rd,
                       (const uint32_t*)bsum, nbd, dk0, dv0, nkeep);
  } else {
    hipLaunchKernelGGL(k_depth_keys<kDepthDigitBits>, dim3(nbd), dim3(kSortThreads), 0, s, rec4, tiles, M, dk0, dv0,
                       hist, nbd, rd);
  }
  uint32_t *ka = dk0, *va = dv0, *kb = dk1, *vb = dv1;
  for (int shift = 0; shift < 32; shift += kDepthDigitBits) {
    radix_pass<kDepthDigitBits>(ka, va, kb, vb, nkeep, M, M, shift, hist, digit_base, nbd, rd, s,
                                shift == 0 && !compact);
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  const uint32_t* order = va;
  uint32_t* offs = ka;  // the free key buffer holds the per-item offsets
  hipLaunchKernelGGL(k_count_sum, dim3(nbd), dim3(kSortThreads), 0, s, order, tiles, M, (const int32_t*)nkeep, rd,
                     bsum);
  const int rt = sort_rounds(cap), nbt = (int)sort_blocks(cap);
  const int64_t span = emit_span(cap), nspan = emit_spans(cap);
  // the emission spans of block b are the positions of tile-sort block b
  // (kEmitWaves spans per block: nbt blocks cover the spans)
  uint32_t* first = hist + (int64_t)(1 << kTileDigitBits) * nbt;  // after the first tile pass's histogram
  hipLaunchKernelGGL(k_offsets, dim3(nbd), dim3(kSortThreads), 0, s, order, tiles, M, (const int32_t*)nkeep,
                     (const uint32_t*)bsum, nbd,
                     offs, count, cap, rd, first, span, nspan);
  // emission lands in the buffer that, after npass ping-pongs, is the output
  uint32_t* ek = (npass & 1) ? tk : tile_of;
  uint32_t* ev = (npass & 1) ? tv : reinterpret_cast<uint32_t*>(item);
  uint32_t* ok = (npass & 1) ? tile_of : tk;
  uint32_t* ov = (npass & 1) ? reinterpret_cast<uint32_t*>(item) : tv;
  const bool emitted = nbt > 0 && M > 0;
  if (emitted)
    hipLaunchKernelGGL(k_emit, dim3((unsigned)nbt), dim3(64 * kEmitWaves), 0, s, jobs, item_off_d, R, order, rec4, radius, tiles,
                       M, (const int32_t*)nkeep, (const uint32_t*)offs, (const int32_t*)count,
                       (const uint32_t*)first, span, nspan, ek, reinterpret_cast<int32_t*>(ev), hist, tbits);
  for (int p = 0; p < npass && nbt > 0; ++p) {
    const bool hd = p == 0 && emitted;
    if (tbits == 6)
      radix_pass<6>(ek, ev, ok, ov, count, 0, cap, 6 * p, hist, digit_base, nbt, rt, s, hd);
    else if (tbits == 7)
      radix_pass<7>(ek, ev, ok, ov, count, 0, cap, 7 * p, hist, digit_base, nbt, rt, s, hd);
    else
      radix_pass<8>(ek, ev, ok, ov, count, 0, cap, 8 * p, hist, digit_base, nbt, rt, s, hd);
    std::swap(ek, ok);
    std::swap(ev, ov);
  }
  const int64_t nr = (std::max<int64_t>(cap, T) + 3) / 4;  // threads of 4 keys (or tiles)
  if (nr > 0)
    hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s, (const uint32_t*)tile_of,
                       (const int32_t*)count, range, T);
}
}  // namespace ls

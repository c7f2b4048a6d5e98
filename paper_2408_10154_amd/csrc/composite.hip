// Front-to-back alpha compositing (forward) and its back-to-front
// recomputation (backward) on gfx950.  A 16x16 tile is four 8x8-pixel bands
// (quadrants), one wave each: the forward runs one band per 64-thread block,
// the backward one tile per 256-thread block.
//
// Splat records of a tile's list are staged through LDS in chunks; every lane
// reads the same record (LDS broadcast), and each band walks only the entries
// that can reach it.  The forward stops a band once every pixel of it has
// terminated.  The backward kernels also exist in a persistent form: a grid
// that fills the GPU once pulls tiles from device-side queues.
#include "common.h"
#include "kernels.h"

#include <cstdlib>
#include <mutex>

namespace ls {

struct TileCtx {
  int r;         // render
  int tile;      // global tile index
  int x, y;      // pixel of this thread
  int x0, y0;    // the tile's first pixel
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
  // wave w of the block covers the 8x8 quadrant (w & 1, w >> 1); lane l its
  // pixel (l & 7, l >> 3)
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  c.x0 = tx * kTile;
  c.y0 = ty * kTile;
  c.x = c.x0 + 8 * (w & 1) + (l & 7);
  c.y = c.y0 + 8 * (w >> 1) + (l >> 3);
  c.W = J.W;
  c.H = J.H;
  c.inside = c.x < J.W && c.y < J.H;
  c.pix = J.pix_off + (int64_t)c.y * J.W + c.x;
  return c;
}

// The y-extent of the support ellipse over the column strip x0 <= x <= x1:
// from its lowest to its highest point when those lie inside the strip, else
// to the ends of the chord on the nearer strip edge (the ellipse's y-range
// over a vertical line x = xb is the root interval of a quadratic in y).
// False when the ellipse does not reach the strip.
__device__ __forceinline__ bool strip_extent(float u, float v, float A, float B, float C, float dq, float smax,
                                             float hx, float hy, float x0, float x1, float& ylo, float& yhi) {
  if (u + hx < x0 || u - hx > x1) return false;
  const float sx = B / A * hy;  // the highest point sits at x = u - sx, the lowest at u + sx
  const float top_x = u - sx, bot_x = u + sx;
  yhi = v + hy;
  ylo = v - hy;
  if (top_x < x0 || top_x > x1) {
    const float dx = (top_x < x0 ? x0 : x1) - u;
    const float D = 2.f * C * smax - dq * dx * dx;
    if (!(D >= 0.f)) return false;
    yhi = v + (-B * dx + sqrtf(D)) / C;
  }
  if (bot_x < x0 || bot_x > x1) {
    const float dx = (bot_x < x0 ? x0 : x1) - u;
    const float D = 2.f * C * smax - dq * dx * dx;
    if (!(D >= 0.f)) return false;
    ylo = v + (-B * dx - sqrtf(D)) / C;
  }
  yhi += fabsf(yhi - v) * 1e-3f + 0.02f;
  ylo -= fabsf(v - ylo) * 1e-3f + 0.02f;
  return true;
}

// Which of the tile's four 8x8-pixel wave quadrants (bit 2 qy + qx for the
// quadrant at column qx, row qy) the Gaussian can reach with alpha >= 1/255.
// The support {o exp(-sigma) >= 1/255} is the ellipse sigma <= s = ln(255 o);
// its x half-extent is sqrt(2 s Sigma_xx) (Sigma = conic^-1).  Over each of
// the two 8-pixel column strips the ellipse's y-extent (strip_extent) is
// tested against the two 8-pixel row ranges.  s is widened by 0.1% + 1e-4
// and every extent by 0.1% + 0.02 px, so FP32 rounding never drops a
// contributor.  (Against 16x4 row bands, 8x8 quadrants are reached by 7 %
// fewer (Gaussian, band) pairs on the 200k-Gaussian render loop.)
__device__ __forceinline__ uint32_t wave_mask(float4 a, float4 b, int tile_x0, int tile_y0) {
  const float o = b.y;
  if (!(o >= LS_ALPHA_MIN)) return 0u;
  const float A = a.z, B = a.w, C = b.x;
  const float dq = A * C - B * B;
  if (!(dq > 0.f)) return 0xFu;
  const float smax = __logf(o * (1.0f / LS_ALPHA_MIN)) * 1.001f + 1e-4f;
  const float hx = sqrtf(fmaxf(2.f * smax * C / dq, 0.f)) * 1.001f + 0.02f;
  const float hy = sqrtf(fmaxf(2.f * smax * A / dq, 0.f)) * 1.001f + 0.02f;
  const float xa = (float)tile_x0 + 0.5f, ya = (float)tile_y0 + 0.5f;
  uint32_t m = 0;
#pragma unroll
  for (int qx = 0; qx < 2; ++qx) {
    float ylo, yhi;
    if (!strip_extent(a.x, a.y, A, B, C, dq, smax, hx, hy, xa + 8.f * qx, xa + 8.f * qx + 7.f, ylo, yhi)) continue;
#pragma unroll
    for (int qy = 0; qy < 2; ++qy) {
      const float y0 = ya + 8.f * qy, y1 = y0 + 7.f;
      if (!(yhi < y0 || ylo > y1)) m |= 1u << (2 * qy + qx);
    }
  }
  return m;
}

// The rows of one 8x8 band (pixel centres from (bx0, by0), 1 px apart) that
// the Gaussian's alpha >= 1/255 support can reach, as a mask of whole rows
// (bit 8 r + c for every column c of a reached row r): the support's y-extent
// over the band's column strip (strip_extent, widened as in wave_mask) holds
// every pixel centre the support contains, so a row whose centre lies outside
// it holds no pixel that composites the entry.
__device__ __forceinline__ uint64_t band_rows(float4 a, float4 b, float bx0, float by0) {
  const float o = b.y;
  if (!(o >= LS_ALPHA_MIN)) return 0ull;
  const float A = a.z, B = a.w, C = b.x;
  const float dq = A * C - B * B;
  if (!(dq > 0.f)) return ~0ull;
  const float smax = __logf(o * (1.0f / LS_ALPHA_MIN)) * 1.001f + 1e-4f;
  const float hx = sqrtf(fmaxf(2.f * smax * C / dq, 0.f)) * 1.001f + 0.02f;
  const float hy = sqrtf(fmaxf(2.f * smax * A / dq, 0.f)) * 1.001f + 0.02f;
  float ylo, yhi;
  if (!strip_extent(a.x, a.y, A, B, C, dq, smax, hx, hy, bx0, bx0 + 7.f, ylo, yhi)) return 0ull;
  const int r0 = (int)fmaxf(ceilf(ylo - by0), 0.f), r1 = (int)fminf(floorf(yhi - by0), 7.f);
  if (r0 > r1) return 0ull;
  return (~0ull >> (8 * (7 - r1))) & (~0ull << (8 * r0));
}

// Tile queues of the persistent compositing kernels (in the bins workspace:
// zero on first use, re-zeroed by every launch).  The tiles are cut into 8
// contiguous ranges; block b runs on XCD b % 8 under round-robin dispatch and
// starts on range b % 8, so each XCD's L2 sees neighbouring tiles.  A block's
// first tile is fixed (the (b / 8)-th of its range, as a plain one-block-per-
// tile launch would map it); later tiles come from a counter per range,
// first of its own range and then of the others.  Each counter has a cache
// line to itself.  No block ever waits for another: a block exits once every
// range is drained, and the last block to exit re-zeroes the counters.
struct TileQueue {
  struct alignas(128) Line {
    uint32_t v;
    uint32_t pad[31];
  };
  Line next[8];  // dynamic claims from each range (may overshoot)
  Line done;     // blocks that have exited
};
static_assert(sizeof(TileQueue) == 9 * 128, "queue record size");

__device__ __forceinline__ void range_of(int T, int x, int& lo, int& n) {
  lo = (int)(((int64_t)T * x) >> 3);
  n = (int)(((int64_t)T * (x + 1)) >> 3) - lo;
}

// Statically mapped tiles of range x: one per block b < nstatic with
// b % 8 == x (blocks past nstatic only ever claim from the counters).
__device__ __forceinline__ int static_claims(int nstatic, int x, int n) {
  const int blocks = nstatic > x ? (nstatic - x + 7) >> 3 : 0;
  return blocks < n ? blocks : n;
}

// The block's next tile, or -1 when all ranges are drained.  `first` and
// `dead` (ranges found empty) are kept by the caller in wave 0.  The home
// range is tried with one atomic; after that, lanes 0..7 of wave 0 read all
// eight counters at once (one memory latency instead of eight in a row) and
// the first range in probe order that still has tiles is claimed from; a
// lost race marks that range and probes again.  Called by every thread.
__device__ __forceinline__ int claim_tile(TileQueue* q, int T, int nstatic, bool& first, uint32_t& dead,
                                          int* s_tile) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const int home = blockIdx.x & 7;
    int t = -1;
    if (first) {
      first = false;
      int lo, n;
      range_of(T, home, lo, n);
      const int k = (int)(blockIdx.x >> 3);
      if ((int)blockIdx.x < nstatic && k < n) t = lo + k;
    }
    if (t < 0 && !(dead & 1u << home)) {
      int lo, n;
      range_of(T, home, lo, n);
      const int s0 = static_claims(nstatic, home, n);
      const uint32_t i = (lane == 0 && s0 < n) ? atomicAdd(&q->next[home].v, 1u) : 0u;
      const int ti = __shfl(s0 + (int)i < n ? lo + s0 + (int)i : -1, 0, 64);
      if (ti >= 0) t = ti;
      else dead |= 1u << home;
    }
    while (t < 0 && dead != 0xFFu) {
      // parallel probe of the ranges still alive, in order home+1, home+2, ...
      const int x = (home + 1 + (lane & 7)) & 7;
      int lo, n;
      range_of(T, x, lo, n);
      const int s0 = static_claims(nstatic, x, n);
      bool avail = false;
      if (lane < 8 && !((dead >> x) & 1u) && s0 < n)
        avail = s0 + (int)__hip_atomic_load(&q->next[x].v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < n;
      const uint64_t m = __ballot(avail);
      uint32_t gone = 0;
      for (int l = 0; l < 8; ++l)
        if (!((m >> l) & 1ull)) gone |= 1u << ((home + 1 + l) & 7);
      dead |= gone;  // counters only grow: a drained range stays drained
      if (m == 0ull) {
        dead = 0xFFu;
        break;
      }
      const int pick = (int)__builtin_ctzll(m);
      const int y = (home + 1 + pick) & 7;
      int ly, ny;
      range_of(T, y, ly, ny);
      const int sy = static_claims(nstatic, y, ny);
      const uint32_t i = lane == 0 ? atomicAdd(&q->next[y].v, 1u) : 0u;
      const int ti = __shfl(sy + (int)i < ny ? ly + sy + (int)i : -1, 0, 64);
      if (ti >= 0) t = ti;
      else dead |= 1u << y;
    }
    if (lane == 0) *s_tile = t;
  }
  __syncthreads();
  const int t = *s_tile;
  __syncthreads();
  return t;
}

// After a block's last claim: the last block to exit re-zeroes the queue, so
// the next launch (or graph replay) on the stream starts from zero.  No fence:
// every claim of a block returned (its value decided the block's exit) before
// the block counts itself done, and the atomics are ordered at the device
// scope; a release fence here would write back the L2 once per block.
__device__ __forceinline__ void release_queue(TileQueue* q) {
  if (threadIdx.x == 0) {
    if (atomicAdd(&q->done.v, 1u) == gridDim.x - 1) {
      for (int x = 0; x < 8; ++x) atomicExch(&q->next[x].v, 0u);
      atomicExch(&q->done.v, 0u);
    }
  }
}

// Forward, one wave per 8x8-pixel band of a tile (a 64-thread block): no
// block barriers, and a band stops reading its tile's list as soon as all of
// its pixels have terminated.  The wave walks the list 64 entries at a time:
// each lane loads one record and tests it against the band (wave_mask, the
// test the backward uses), and the entries that can reach the band are
// compacted, in list order, into the wave's LDS.  (Measured against a
// 256-thread block per tile that staged each record once for all four bands:
// 1 % faster on the render loop and on a registration pair.)
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(8))) void k_composite_fwd_band(
    const JobDev* __restrict__ jobs, const int32_t* __restrict__ tile_off, int R, int T_total,
    const float4* __restrict__ rec, const int32_t* __restrict__ items, const int32_t* __restrict__ range, float bg0,
    float bg1, float bg2, float* __restrict__ out_rgb, float* __restrict__ out_depth, float* __restrict__ out_alpha,
    float* __restrict__ out_T, int32_t* __restrict__ out_n, uint64_t* __restrict__ used, int64_t ustride,
    int cover) {
  // one entry of padding: the walk reads entry j + 1 ahead without a clamp
  __shared__ float4 s0[65], s1[65], s2[65];
  __shared__ int32_t spos[64];
  const int unit = xcd_remap(blockIdx.x, 4 * T_total);
  if (unit >= 4 * T_total) return;
  const int tile = unit >> 2, band = unit & 3;
  const int lane = threadIdx.x;
  const int r = find_segment<int32_t>(tile_off, R, tile);
  const JobDev& J = jobs[r];
  const int local = tile - J.tile_off;  // tile index within its render
  const int tile_y = local / J.TX, tile_x = local - tile_y * J.TX;
  const int tx0 = tile_x * kTile, ty0 = tile_y * kTile;
  const int x = tx0 + 8 * (band & 1) + (lane & 7), y = ty0 + 8 * (band >> 1) + (lane >> 3);
  const bool inside = x < J.W && y < J.H;
  const int start = range[2 * tile], end = range[2 * tile + 1];
  const float fx = (float)x + 0.5f, fy = (float)y + 0.5f;
  const float bx0 = (float)(tx0 + 8 * (band & 1)) + 0.5f, by0 = (float)(ty0 + 8 * (band >> 1)) + 0.5f;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  float T = 1.f, cr = 0.f, cg = 0.f, cb = 0.f, dd = 0.f;
  int nlast = end - start;
  uint64_t alive = __ballot(inside);  // lane l is pixel (l & 7, l >> 3) of the band: bit l of band_rows
  // chunk k of the tile's list keeps its "used" bits in slot (start / 64) +
  // tile + k of the band's row: the slots of successive tiles never overlap
  int64_t slot = (int64_t)(start >> 6) + tile;
  for (int chunk = start; chunk < end && alive != 0ull; chunk += 64, ++slot) {
    const int e = chunk + lane;
    uint64_t usedm = 0ull;  // bit j: some pixel of the band composited its j-th staged entry
    bool in = false;
    float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;  // this lane's record
    if (e < end) {
      const int64_t it = items[e];
      r0 = rec[it * 3 + 0];
      r1 = rec[it * 3 + 1];
      if (cover)  // some row the entry can reach holds a pixel still compositing
        in = (band_rows(r0, r1, bx0, by0) & alive) != 0ull;
      else
        in = (wave_mask(r0, r1, tx0, ty0) >> band) & 1u;
      if (in) {
        stage_conic(r0, r1);
        r2 = rec[it * 3 + 2];
      }
    }
    const uint64_t bal = __ballot(in);
    const int pos = __popcll(bal & lt);
    if (in) {
      s0[pos] = r0;
      s1[pos] = r1;
      s2[pos] = r2;
      spos[pos] = e - start;
    }
    __builtin_amdgcn_wave_barrier();
    const int cw = __popcll(bal);
    // one step at staged entry j; returns whether every pixel has now stopped
    // (decided only where pixels stop, so a step that stops none tests nothing)
    auto step = [&](int j, const float4& a, const float4& b, const float4& col) -> bool {
      bool ended = false;
      const float dx = fx - a.x, dy = fy - a.y;
      const float sl = falloff_log2(a.z, a.w, b.x, dx, dy);
      const float al = fminf(LS_ALPHA_MAX, b.y * __builtin_amdgcn_exp2f(-sl));
      // the weight alpha T, and T (1 - alpha) as T - alpha T in one FMA
      const float w = al * T, Tn = __builtin_fmaf(-al, T, T);
      const uint64_t hit = alive & __ballot(composited(sl, b));
      const uint64_t stop = hit & __ballot(Tn < LS_T_STOP);
      const uint64_t use = hit & ~stop;
      if (stop != 0ull) {
        if (__builtin_amdgcn_inverse_ballot_w64(stop)) nlast = spos[j];
        alive &= ~stop;
        ended = alive == 0ull;
      }
      if (use != 0ull) {
        const bool u = __builtin_amdgcn_inverse_ballot_w64(use);
        const float wgt = u ? w : 0.f;  // 0 adds an exact zero below
        cr += wgt * col.x;
        cg += wgt * col.y;
        cb += wgt * col.z;
        dd += wgt * b.z;
        T = u ? Tn : T;
        // usedm |= 1 << j in one scalar instruction (a register-only bit set)
        asm volatile("s_bitset1_b64 %0, %1" : "+s"(usedm) : "s"(j));
      }
      return ended;
    };
    // Records are read one entry ahead into two alternating register sets
    // (the loop unrolled by hand, so no copies), so the LDS latency of the
    // next entry overlaps the arithmetic of this one; the read past the last
    // staged entry (at most entry 64, the padding) is never used.  The walk
    // ends after the staged entries or once every pixel has stopped.
    float4 aA = s0[0], bA = s1[0], cA = s2[0], aB, bB, cB;
    for (int jj = 0; jj < cw;) {
      aB = s0[jj + 1];
      bB = s1[jj + 1];
      cB = s2[jj + 1];
      if (step(jj, aA, bA, cA) || ++jj >= cw) break;
      aA = s0[jj + 1];
      bA = s1[jj + 1];
      cA = s2[jj + 1];
      if (step(jj, aB, bB, cB)) break;
      ++jj;
    }
    // the entries of this chunk that some pixel of the band composited
    // (bit l: entry chunk + l): exactly the (entry, band) pairs in which the
    // backward has an active lane
    const uint64_t um = __ballot(in && ((usedm >> pos) & 1ull));
    if (lane == 0) used[band * ustride + slot] = um;
    __builtin_amdgcn_wave_barrier();
  }
  if (!inside) return;
  const int64_t hw = (int64_t)J.W * J.H;
  const int64_t pix = J.pix_off + (int64_t)y * J.W + x;
  float* rgb = out_rgb + 3 * J.pix_off + (int64_t)y * J.W + x;
  rgb[0] = cr + T * bg0;
  rgb[hw] = cg + T * bg1;
  rgb[2 * hw] = cb + T * bg2;
  out_depth[pix] = dd;
  out_alpha[pix] = 1.f - T;
  out_T[pix] = T;
  out_n[pix] = nlast;
}

// Lane exchanges of gfx950 that trade halves of two registers:
// permlane32_swap gives x the lower 32 lanes of y in place of its upper 32,
// permlane16_swap gives x the even 16-lane rows of y in place of its odd rows
// (and y what x gave up).  Adding the two results sums each value over lane
// pairs 32 (or 16) apart while packing two values into one register.
__device__ __forceinline__ float swap32_sum(float x, float y) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap16_sum(float x, float y) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Swap-add of two registers between the two halves of each group of 2m
// lanes (m = 8: row_ror:8 pairs lane i with i +- 8 of its row; m = 4:
// row_half_mirror pairs lane i with 7 - i of its 8-lane half): lanes of the
// lower m keep a's value summed with a's partner, lanes of the upper m keep
// b's.  With a == b this is a plain add of the partner (one instruction).
template <int kCtrl, int kM>
__device__ __forceinline__ float pair_sum(float a, float b, int lane) {
  const bool lo = (lane & kM) == 0;
  const float s = lo ? a : b, t = lo ? b : a;
  return s + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(t), kCtrl, 0xF, 0xF, true));
}

// Sums of N values (N even, N <= 16) over the 64 lanes of the wave, by a
// transposing reduction that halves the lanes holding each value at every
// level while packing more values per register:
//  - 32-lane swaps and adds: value 2k in the lower half of register h[k],
//    2k + 1 in the upper half;
//  - 16-lane swaps and adds: four values per register q[i], one per row
//    (value 4 i + slot(r) in row r, slot = 0, 2, 1, 3);
//  - within rows, swap-adds 8 lanes apart (q[0] with q[1], q[2] with q[3]),
//    then 4 apart, leave one value per 4-lane group of one register, and two
//    DPP adds sum each group.
// The result: the lane that wave_value() names holds the total of that
// value.  N = 10 costs 5 + 3 swaps and 17 VALU adds or selects; a plain row
// sum after the 16-lane level would take 20 adds.  When N/2 is odd the last
// 16-lane pair is the register with itself (its rows 1 and 3 repeat rows 0
// and 2), and with fewer than three row registers the 8-apart level pairs a
// register with itself: those duplicates are not named by wave_value().  The
// whole wave must be active.
template <int N>
__device__ __forceinline__ float wave_sums(const float* g, int lane) {
  static_assert(N % 2 == 0 && N <= 16, "an even number of values, at most 16");
  constexpr int H = N / 2, O = (H + 1) / 2;
  float h[H], q[O];
#pragma unroll
  for (int k = 0; k < H; ++k) h[k] = swap32_sum(g[2 * k], g[2 * k + 1]);
#pragma unroll
  for (int i = 0; i < O; ++i) q[i] = swap16_sum(h[2 * i], h[2 * i + 1 < H ? 2 * i + 1 : 2 * i]);
  constexpr int kRor8 = 0x128, kHalfMirror = 0x141, kQuad1032 = 0xB1, kQuad2301 = 0x4E;
  const float z0 = pair_sum<kRor8, 8>(q[0], O > 1 ? q[O > 1 ? 1 : 0] : q[0], lane);
  const float z1 = O > 2 ? pair_sum<kRor8, 8>(q[O > 2 ? 2 : 0], q[O > 3 ? 3 : (O > 2 ? 2 : 0)], lane) : z0;
  float y = pair_sum<kHalfMirror, 4>(z0, z1, lane);
  y += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(y), kQuad1032, 0xF, 0xF, true));
  y += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(y), kQuad2301, 0xF, 0xF, true));
  // Keep the last add in every lane: callers store the sum from a few lanes,
  // and sinking the add into that branch splits the fused DPP add into a DPP
  // move plus an add (an empty asm that reads and writes y, no code).
  asm volatile("" : "+v"(y));
  return y;
}

// The value whose total lane `lane` holds after wave_sums<N>, or -1 for the
// lanes that hold none, a duplicate, or one of the same group (exactly one
// lane per value is named).
template <int N>
__device__ __forceinline__ int wave_value(int lane) {
  constexpr int O = (N / 2 + 1) / 2;
  if (lane & 3) return -1;
  const int r = lane >> 4, grp = (lane >> 2) & 3;
  // 8 apart: lanes 0-7 of a row keep q[0] (q[2]), 8-15 q[1] (q[3]); 4 apart:
  // groups 0 and 2 keep the first register's, 1 and 3 the second's
  int qi;
  if (O > 2)
    qi = (grp & 1) ? ((grp >> 1) ? 3 : 2) : (grp >> 1);
  else if (O == 2)
    qi = (grp & 1) ? -1 : (grp >> 1);
  else
    qi = grp == 0 ? 0 : -1;
  if (qi < 0 || qi >= O) return -1;
  const int v = 4 * qi + (((r & 1) << 1) | (r >> 1));
  return v < N ? v : -1;
}

constexpr int kBwdChunk = 64;   // list entries staged per round (full mode)
constexpr int kWaveSlots = 4 * ((kGrad2D / 2 + 1) / 2);  // floats per wave partial (a slot per value index)
constexpr int kPartStride = 4 * kWaveSlots + 1;         // floats per entry: 4 wave partials, odd against bank conflicts

// Backward.  Per pixel, walking the list from n_last - 1 down to 0 with the
// transmittance recovered as T_i = T_{i+1} / (1 - alpha_i) and the running
// "behind" value acc = sum_{j>i} alpha_j prod_{i<k<j}(1 - alpha_k) v_j +
// prod_{k>i}(1 - alpha_k)(bg . gC - gA), where v_j = c_j . gC + z_j gD:
//   dL/dalpha_i = T_i (v_i - acc_i).
// One such step at a pixel, in two parts.  bwd_eval (every entry of the
// band's list) says whether the entry was composited there: act = visited,
// sigma >= 0 and alpha >= 1/255.  bwd_apply (entries some lane of the wave
// composited), branch-free: where act, T is recovered, acc updated, and
// wgt = alpha T, ds = dL/dsigma and dop = dL/d(opacity) are set (both zero
// while the 0.99 clamp is active).  Elsewhere the step runs with alpha = 0,
// which leaves T (times 1 / 1) and acc (plus 0) unchanged and gives wgt = 0,
// and with G and exp(-sigma) selected to 0, which gives ds = dop = 0: three
// selects instead of one per output.
struct BwdEval {
  float ex, G, al;  // exp(-sigma), o exp(-sigma), alpha
  bool act;
};

__device__ __forceinline__ BwdEval bwd_eval(bool visited, float4 a, float4 b, float dx, float dy) {
  BwdEval e;
  const float sl = falloff_log2(a.z, a.w, b.x, dx, dy);
  e.ex = __builtin_amdgcn_exp2f(-sl);
  e.G = b.y * e.ex;
  e.al = fminf(LS_ALPHA_MAX, e.G);
  e.act = visited && composited(sl, b);
  return e;
}

__device__ __forceinline__ void bwd_apply(const BwdEval& e, float4 col, float z, float gR, float gG, float gB,
                                          float gD, float& T, float& acc, float& wgt, float& ds, float& dop) {
  const float al = e.act ? e.al : 0.f;
  T = T * __builtin_amdgcn_rcpf(1.f - al);
  wgt = al * T;
  const float v = col.x * gR + col.y * gG + col.z * gB + z * gD;
  const float d = v - acc;
  const float dal = T * d;
  acc = fmaf(al, d, acc);  // alpha v + (1 - alpha) acc
  const bool grad = e.act && e.G < LS_ALPHA_MAX;  // dL/dG = dal; no gradient through an active clamp
  ds = -dal * (grad ? e.G : 0.f);
  dop = dal * (grad ? e.ex : 0.f);
}

// Per-pixel state shared by both backward kernels: upstream gradients (scaled),
// final transmittance, entries visited, and the initial "behind" value.
struct BwdPixel {
  float T, gR, gG, gB, gD, acc;
  int nl;
  float lsum, lcnt;  // the pixel's L1 terms and 1 when it lies in Omega (L1 targets only), else 0
};

__device__ __forceinline__ float l1_sign(float d) { return d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f); }

__device__ __forceinline__ BwdPixel bwd_pixel(const TileCtx& c, const JobDev& J, float bg0, float bg1, float bg2,
                                              const float* fwd_T, const int32_t* fwd_n, const float* up_rgb,
                                              const float* up_depth, const float* up_alpha, const float* up_scale,
                                              const L1Targets& l1) {
  BwdPixel p{1.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0, 0.f, 0.f};
  if (c.inside) {
    const int64_t hw = (int64_t)J.W * J.H;
    const int64_t ci = 3 * J.pix_off + (int64_t)c.y * J.W + c.x;
    const float sc = up_scale ? up_scale[c.r] : 1.f;
    if (l1.pred_rgb) {
      // the loss gradient of this pixel, as the L1 loss kernel forms it
      const int64_t q = (int64_t)c.y * J.W + c.x;
      const float* trgb = l1.tgt_rgb ? l1.tgt_rgb + ci : J.tgt_rgb + q;
      const float td = l1.tgt_depth ? l1.tgt_depth[c.pix] : J.tgt_depth[q];
      const bool valid = td > 0.f;
      const float d0 = l1.pred_rgb[ci] - trgb[0], d1 = l1.pred_rgb[ci + hw] - trgb[hw];
      const float d2 = l1.pred_rgb[ci + 2 * hw] - trgb[2 * hw], dd = l1.pred_depth[c.pix] - td;
      p.gR = sc * (valid ? l1_sign(d0) : 0.f);
      p.gG = sc * (valid ? l1_sign(d1) : 0.f);
      p.gB = sc * (valid ? l1_sign(d2) : 0.f);
      p.gD = sc * (valid ? l1_sign(dd) : 0.f);
      if (valid) {  // summed as the loss kernel sums a pixel: depth, then the channels in order
        p.lsum = ((fabsf(dd) + fabsf(d0)) + fabsf(d1)) + fabsf(d2);
        p.lcnt = 1.f;
      }
    }
    if (up_rgb) { p.gR = sc * up_rgb[ci]; p.gG = sc * up_rgb[ci + hw]; p.gB = sc * up_rgb[ci + 2 * hw]; }
    if (up_depth) p.gD = sc * up_depth[c.pix];
    const float gA = up_alpha ? sc * up_alpha[c.pix] : 0.f;
    p.T = fwd_T[c.pix];
    p.nl = fwd_n[c.pix];
    p.acc = bg0 * p.gR + bg1 * p.gG + bg2 * p.gB - gA;
  }
  return p;
}

// Wave 0 stages a chunk of the tile's list (records and item ids) and builds,
// for each of the four wave bands, the list-ordered positions of the entries
// that some pixel of the band composited in the forward (its "used" bits:
// per band row, 64 entries per slot, slot (start / 64) + tile + k for the
// entries from start + 64 k on; list positions at or beyond the band's
// largest entry count bmax were never walked there and are dropped).
template <int kChunk>
__device__ __forceinline__ void stage_chunk(int lane, int cnt, int chunk, int start, int tile, const int* bmax,
                                            const int32_t* items, const float4* rec, const uint64_t* used,
                                            int64_t ustride, float4* s0, float4* s1, float4* s2, int32_t* sit,
                                            uint32_t* smask, uint8_t (*slist)[kChunk], uint32_t* swc) {
  // the chunk's bits of each band (bit l: entry chunk + l), from one or two slots
  const int rel = chunk - start, sh = rel & 63;
  const int64_t slot = (int64_t)(start >> 6) + tile + (rel >> 6);
  uint64_t ub[4];
#pragma unroll
  for (int b2 = 0; b2 < 4; ++b2) {
    const uint64_t w0 = used[b2 * ustride + slot];
    const uint64_t w1 = sh ? used[b2 * ustride + slot + 1] : 0ull;
    ub[b2] = sh ? (w0 >> sh) | (w1 << (64 - sh)) : w0;
  }
  uint32_t m = 0;
  const bool valid = lane < cnt;
  if (valid) {
    const int64_t it = items[chunk + lane];
    float4 a = rec[it * 3 + 0], b = rec[it * 3 + 1];
    const int k = chunk + lane - start;
#pragma unroll
    for (int b2 = 0; b2 < 4; ++b2) m |= (uint32_t)((ub[b2] >> lane) & 1ull) << b2;
#pragma unroll
    for (int b2 = 0; b2 < 4; ++b2)
      if (k >= bmax[b2]) m &= ~(1u << b2);
    stage_conic(a, b);
    sit[lane] = (int32_t)it;
    s0[lane] = a;
    s1[lane] = b;
    s2[lane] = rec[it * 3 + 2];
    smask[lane] = m;
  }
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int b2 = 0; b2 < 4; ++b2) {
    const bool in = valid && ((m >> b2) & 1u);
    const uint64_t bal = __ballot(in);
    if (in) slist[b2][__popcll(bal & lt)] = (uint8_t)lane;
    if (lane == 0) swc[b2] = (uint32_t)__popcll(bal);
  }
}

// The tile's L1 loss partial (L1 targets with loss_part): each wave's sums to
// LDS before the caller's next barrier (tile_loss_put), and after it threads 0
// and 1 write {sum, count} over the four waves in order (tile_loss_get).
__device__ __forceinline__ void tile_loss_put(const L1Targets& l1, const BwdPixel& px, float (*sl)[4]) {
  if (!l1.loss_part) return;
  const float s = wave_sum(px.lsum), n = wave_sum(px.lcnt);
  if ((threadIdx.x & 63) == 0) {
    sl[0][threadIdx.x >> 6] = s;
    sl[1][threadIdx.x >> 6] = n;
  }
}
__device__ __forceinline__ void tile_loss_get(const L1Targets& l1, float (*sl)[4], int tile) {
  if (l1.loss_part && threadIdx.x < 2) {
    const float* v = sl[threadIdx.x];
    l1.loss_part[2 * (int64_t)tile + threadIdx.x] = (v[0] + v[1]) + (v[2] + v[3]);
  }
}

// Full mode: the ten per-pixel terms of each entry are summed over each
// wave's 64 lanes (wave_sums), the four wave sums of the block over LDS in a
// fixed order, and the ten gradients formed from them are added to the item's
// accumulator (one atomic per nonzero value and tile).
__device__ __forceinline__ void composite_bwd_tile(const JobDev* __restrict__ jobs,
                                                          const int32_t* __restrict__ tile_off, int R, int T_total,
                                                          const float4* __restrict__ rec,
                                                          const int32_t* __restrict__ items,
                                                          const int32_t* __restrict__ range,
                                                          const uint64_t* __restrict__ used, int64_t ustride,
                                                          float bg0, float bg1, float bg2,
                                                          const float* __restrict__ fwd_T,
                                                          const int32_t* __restrict__ fwd_n,
                                                          const float* __restrict__ up_rgb,
                                                          const float* __restrict__ up_depth,
                                                          const float* __restrict__ up_alpha,
                                                          const float* __restrict__ up_scale,
                                                          float* __restrict__ g2d, const L1Targets& l1, int tile) {
  __shared__ float4 s0[kBwdChunk], s1[kBwdChunk], s2[kBwdChunk];
  __shared__ float sloss[2][4];
  __shared__ int32_t sit[kBwdChunk];
  __shared__ uint32_t smask[kBwdChunk];
  __shared__ uint8_t slist[4][kBwdChunk];
  __shared__ uint32_t swc[4];
  __shared__ __attribute__((aligned(16))) float part[kBwdChunk * kPartStride];
  static_assert(kBwdChunk <= 64 && kBlock % kBwdChunk == 0, "chunk must fit one staging wave");
  __shared__ int bmax[4];
  const TileCtx c = tile_ctx(jobs, tile_off, R, tile);
  const JobDev& J = jobs[c.r];
  const int start = range[2 * tile], end = range[2 * tile + 1];
  const float fx = (float)c.x + 0.5f, fy = (float)c.y + 0.5f;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wval = wave_value<kGrad2D>(lane);  // the value whose wave sum this lane stores, or -1
  BwdPixel px = bwd_pixel(c, J, bg0, bg1, bg2, fwd_T, fwd_n, up_rgb, up_depth, up_alpha, up_scale, l1);
  tile_loss_put(l1, px, sloss);
  if (threadIdx.x < 4) bmax[threadIdx.x] = 0;
  __syncthreads();
  if (px.nl > 0) atomicMax(&bmax[w], px.nl);
  __syncthreads();
  tile_loss_get(l1, sloss, tile);
  const int smax = max(max(bmax[0], bmax[1]), max(bmax[2], bmax[3]));
  const int last = min(start + smax, end);  // exclusive end of the entries any pixel visited

  for (int chunk_end = last; chunk_end > start; chunk_end -= kBwdChunk) {
    const int chunk = max(start, chunk_end - kBwdChunk);
    const int cnt = chunk_end - chunk;
    if (w == 0)
      stage_chunk<kBwdChunk>(lane, cnt, chunk, start, tile, bmax, items, rec, used, ustride, s0, s1, s2, sit, smask,
                             slist, swc);
    __syncthreads();
    const int cw = __builtin_amdgcn_readfirstlane((int)swc[w]);
    // the band's list in a register; lanes past its end hold 0, so the
    // read-ahead index (jj - 1) & 63 below names a staged entry even at jj = 0
    const uint32_t myj = lane < cw ? slist[w][lane] : 0u;
    auto bstep = [&](int j, const float4& a, const float4& b, const float4& col) {
      float* pj = part + j * kPartStride + w * kWaveSlots + max(wval, 0);  // written only where wval >= 0
      const int k = chunk + j - start;  // list position
      const float dx = fx - a.x, dy = fy - a.y;
      // every staged entry has an active lane (the forward's bits), so the
      // step runs unconditionally; inactive lanes contribute exact zeros
      const BwdEval e = bwd_eval(k < px.nl, a, b, dx, dy);
      float wgt, ds, dop;
      bwd_apply(e, col, b.z, px.gR, px.gG, px.gB, px.gD, px.T, px.acc, wgt, ds, dop);
      // per-pixel terms whose sums give the ten gradients; the conic factors
      // of dL/du, dL/dv and the halves of dL/dA, dL/dC are applied once per
      // entry after the sums
      float g[kGrad2D];
      g[0] = ds * dx;
      g[1] = ds * dy;
      g[2] = g[0] * dx;
      g[3] = g[0] * dy;
      g[4] = g[1] * dy;
      g[5] = dop;
      g[6] = wgt * px.gD;
      g[7] = wgt * px.gR;
      g[8] = wgt * px.gG;
      g[9] = wgt * px.gB;
      const float out = wave_sums<kGrad2D>(g, lane);
      if (wval >= 0) *pj = out;
    };
    // records read one entry ahead into alternating register sets (as in the forward)
    int jA = (int)__builtin_amdgcn_readlane(myj, cw > 0 ? cw - 1 : 0), jB = 0;
    float4 aA = s0[jA], bA = s1[jA], cA = s2[jA], aB, bB, cB;
    for (int jj = cw - 1; jj >= 0;) {
      jB = (int)__builtin_amdgcn_readlane(myj, (jj - 1) & 63);
      aB = s0[jB];
      bB = s1[jB];
      cB = s2[jB];
      bstep(jA, aA, bA, cA);
      if (--jj < 0) break;
      jA = (int)__builtin_amdgcn_readlane(myj, (jj - 1) & 63);
      aA = s0[jA];
      bA = s1[jA];
      cA = s2[jA];
      bstep(jB, aB, bB, cB);
      --jj;
    }
    __syncthreads();
    {
      // kBlock / kBwdChunk threads per entry, each summing its values over
      // the waves (bands) that reached the entry, in wave order; the partials
      // of other waves are stale and skipped.  Thread 0 forms dL/du, dL/dv
      // from the sums of ds dx and ds dy with the conic (A, B, C); the other
      // threads split values 2..9 between them.
      constexpr int kPer = kBlock / kBwdChunk;
      static_assert(kPer >= 2 && kGrad2D == 10, "value split assumes at least two threads per entry and 10 values");
      const int j = threadIdx.x / kPer, t = threadIdx.x % kPer;
      const uint32_t mj = j < cnt ? smask[j] : 0u;
      if (mj != 0u) {
        float* dst = g2d + (int64_t)sit[j] * kGrad2D;
        const float* pj = part + j * kPartStride;
        auto band_sum = [&](int q) {
          float v = 0.f;
#pragma unroll
          for (int b2 = 0; b2 < 4; ++b2)
            if ((mj >> b2) & 1u) v += pj[b2 * kWaveSlots + q];
          return v;
        };
        auto put = [&](int q, float v) {
          if (v != 0.f) atomic_add_f32(dst + q, v);
        };
        if (t == 0) {
          const float sx = band_sum(0), sy = band_sum(1);
          const float cA = kTwoLn2 * s0[j].z, cB = kLn2 * s0[j].w, cC = kTwoLn2 * s1[j].x;  // staged -> (A, B, C)
          put(0, -(cA * sx + cB * sy));
          put(1, -(cB * sx + cC * sy));
        } else {
          const int lo = 2 + ((t - 1) * (kGrad2D - 2)) / (kPer - 1), hi = 2 + (t * (kGrad2D - 2)) / (kPer - 1);
          for (int q = lo; q < hi; ++q) {
            const float v = band_sum(q);
            put(q, (q == 2 || q == 4) ? 0.5f * v : v);
          }
        }
      }
    }
    __syncthreads();
  }
}

// One block per tile (XCD-aware mapping), for launches with few tiles per
// resident block.
__global__ __launch_bounds__(kBlock) void k_composite_bwd(const JobDev* __restrict__ jobs,
                                                          const int32_t* __restrict__ tile_off, int R, int T_total,
                                                          const float4* __restrict__ rec,
                                                          const int32_t* __restrict__ items,
                                                          const int32_t* __restrict__ range,
                                                          const uint64_t* __restrict__ used, int64_t ustride,
                                                          float bg0, float bg1, float bg2,
                                                          const float* __restrict__ fwd_T,
                                                          const int32_t* __restrict__ fwd_n,
                                                          const float* __restrict__ up_rgb,
                                                          const float* __restrict__ up_depth,
                                                          const float* __restrict__ up_alpha,
                                                          const float* __restrict__ up_scale,
                                                          float* __restrict__ g2d, L1Targets l1) {
  const int tile = xcd_remap(blockIdx.x, T_total);
  if (tile >= T_total) return;
  composite_bwd_tile(jobs, tile_off, R, T_total, rec, items, range, used, ustride, bg0, bg1, bg2, fwd_T, fwd_n,
                     up_rgb, up_depth, up_alpha, up_scale, g2d, l1, tile);
}

__global__ __launch_bounds__(kBlock) void k_composite_bwd_persistent(const JobDev* __restrict__ jobs,
    const int32_t* __restrict__ tile_off, int R, int T_total, const float4* __restrict__ rec,
    const int32_t* __restrict__ items, const int32_t* __restrict__ range, const uint64_t* __restrict__ used,
    int64_t ustride, float bg0, float bg1, float bg2, const float* __restrict__ fwd_T,
    const int32_t* __restrict__ fwd_n, const float* __restrict__ up_rgb, const float* __restrict__ up_depth,
    const float* __restrict__ up_alpha, const float* __restrict__ up_scale, float* __restrict__ g2d,
    TileQueue* __restrict__ queue, int nstatic, L1Targets l1) {
  __shared__ int s_tile;
  bool first = true;
  uint32_t dead = 0;
  for (;;) {
    const int tile = claim_tile(queue, T_total, nstatic, first, dead, &s_tile);
    if (tile < 0) break;
    composite_bwd_tile(jobs, tile_off, R, T_total, rec, items, range, used, ustride, bg0, bg1, bg2, fwd_T, fwd_n,
                       up_rgb, up_depth, up_alpha, up_scale, g2d, l1, tile);
  }
  release_queue(queue);
}


// Pose-only mode (registration): only the gradients a pose correction acts
// through (u, v, conic, depth) are formed.  Each entry's sums over the tile
// are parked in an LDS queue; whenever it is full (and at the end) every
// thread of the block applies the pose Jacobian of one queued Gaussian, so
// the Jacobian work is spread over all four waves.  Each
// round's results are reduced over the block in a fixed order and added to the
// tile's running sum, written once as the tile's 12-value partial: no atomics,
// so the pose gradient is deterministic and independent of the other renders.
constexpr int kPoseChunk = 64;                    // entries staged per round
constexpr int kPoseRow = 6;                       // sums giving du, dv, dA, dB, dC, d(depth weight)
constexpr int kPoseSlots = 4 * ((kPoseRow / 2 + 1) / 2);  // floats per wave partial (a slot per value index)
constexpr int kPoseStride = 4 * kPoseSlots + 1;   // floats per entry: 4 wave partials, odd against bank conflicts
constexpr int kPoseQueue = kBlock;                // queued entries per Jacobian round

__device__ __forceinline__ void composite_bwd_pose_tile(const JobDev* __restrict__ jobs,
                                                               const int32_t* __restrict__ tile_off, int R,
                                                               int T_total, const float4* __restrict__ rec,
                                                               const float4* __restrict__ aux,
                                                               const float* __restrict__ pose,
                                                               const int32_t* __restrict__ items,
                                                               const int32_t* __restrict__ range,
                                                               const uint64_t* __restrict__ used, int64_t ustride,
                                                               float bg0, float bg1, float bg2,
                                                               const float* __restrict__ fwd_T,
                                                               const int32_t* __restrict__ fwd_n,
                                                               const float* __restrict__ up_rgb,
                                                               const float* __restrict__ up_depth,
                                                               const float* __restrict__ up_alpha,
                                                               const float* __restrict__ up_scale,
                                                               float* __restrict__ tile_part, const L1Targets& l1,
                                                               int tile) {
  __shared__ float4 s0[kPoseChunk], s1[kPoseChunk], s2[kPoseChunk];
  __shared__ int32_t sit[kPoseChunk];
  __shared__ uint32_t smask[kPoseChunk];
  __shared__ uint8_t slist[4][kPoseChunk];
  __shared__ uint32_t swc[4];
  __shared__ __attribute__((aligned(16))) float part[kPoseChunk * kPoseStride];
  __shared__ float qsum[kPoseRow * kPoseQueue];  // [value][slot]
  __shared__ int32_t qit[kPoseQueue];
  __shared__ float wred[4][kPoseAcc];
  __shared__ int bmax[4];
  static_assert(kPoseChunk <= 64 && kPoseQueue % kPoseChunk == 0, "chunk must fit one staging wave");
  const TileCtx c = tile_ctx(jobs, tile_off, R, tile);
  const JobDev& J = jobs[c.r];
  const int start = range[2 * tile], end = range[2 * tile + 1];
  const float fx = (float)c.x + 0.5f, fy = (float)c.y + 0.5f;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wval = wave_value<kPoseRow>(lane);
  __shared__ float sloss[2][4];
  BwdPixel px = bwd_pixel(c, J, bg0, bg1, bg2, fwd_T, fwd_n, up_rgb, up_depth, up_alpha, up_scale, l1);
  tile_loss_put(l1, px, sloss);
  if (threadIdx.x < 4) bmax[threadIdx.x] = 0;
  __syncthreads();
  if (px.nl > 0) atomicMax(&bmax[w], px.nl);
  __syncthreads();
  tile_loss_get(l1, sloss, tile);
  const int smax = max(max(bmax[0], bmax[1]), max(bmax[2], bmax[3]));
  const int last = min(start + smax, end);

  float total = 0.f;  // threads 0..11: the tile's running pose-gradient sum
  int nq = 0;  // queued entries (uniform)
  for (int chunk_end = last; chunk_end > start; chunk_end -= kPoseChunk) {
    const int chunk = max(start, chunk_end - kPoseChunk);
    const int cnt = chunk_end - chunk;
    if (w == 0)
      stage_chunk<kPoseChunk>(lane, cnt, chunk, start, tile, bmax, items, rec, used, ustride, s0, s1, s2, sit, smask,
                              slist, swc);
    __syncthreads();
    const int cw = __builtin_amdgcn_readfirstlane((int)swc[w]);
    // the band's list in a register; lanes past its end hold 0, so the
    // read-ahead index (jj - 1) & 63 below names a staged entry even at jj = 0
    const uint32_t myj = lane < cw ? slist[w][lane] : 0u;
    auto pstep = [&](int j, const float4& a, const float4& b, const float4& col) {
      float* pj = part + j * kPoseStride + w * kPoseSlots + max(wval, 0);  // written only where wval >= 0
      const int k = chunk + j - start;
      const float dx = fx - a.x, dy = fy - a.y;
      // unconditional, as in the full-mode kernel
      const BwdEval e = bwd_eval(k < px.nl, a, b, dx, dy);
      float wgt, ds, dop;
      bwd_apply(e, col, b.z, px.gR, px.gG, px.gB, px.gD, px.T, px.acc, wgt, ds, dop);
      // as in the full-mode kernel: conic factors and halves after the sums
      float g[kPoseRow];
      g[0] = ds * dx;
      g[1] = ds * dy;
      g[2] = g[0] * dx;
      g[3] = g[0] * dy;
      g[4] = g[1] * dy;
      g[5] = wgt * px.gD;
      const float out = wave_sums<kPoseRow>(g, lane);
      if (wval >= 0) *pj = out;
    };
    // records read one entry ahead into alternating register sets (as in the forward)
    int jA = (int)__builtin_amdgcn_readlane(myj, cw > 0 ? cw - 1 : 0), jB = 0;
    float4 aA = s0[jA], bA = s1[jA], cA = s2[jA], aB, bB, cB;
    for (int jj = cw - 1; jj >= 0;) {
      jB = (int)__builtin_amdgcn_readlane(myj, (jj - 1) & 63);
      aB = s0[jB];
      bB = s1[jB];
      cB = s2[jB];
      pstep(jA, aA, bA, cA);
      if (--jj < 0) break;
      jA = (int)__builtin_amdgcn_readlane(myj, (jj - 1) & 63);
      aA = s0[jA];
      bA = s1[jA];
      cA = s2[jA];
      pstep(jB, aB, bB, cB);
      --jj;
    }
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
      // entry j: its sums over the waves (bands) it reaches, in wave order,
      // turned into the six image-space gradients, into queue slot nq + j
      const int j = threadIdx.x;
      const uint32_t mj = smask[j];
      const float* pj = part + j * kPoseStride;
      float g6[kPoseRow] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (mj != 0u) {
        float sum[kPoseRow] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b2 = 0; b2 < 4; ++b2) {
          if (!((mj >> b2) & 1u)) continue;
#pragma unroll
          for (int q = 0; q < kPoseRow; ++q) sum[q] += pj[b2 * kPoseSlots + q];
        }
        const float cA = kTwoLn2 * s0[j].z, cB = kLn2 * s0[j].w, cC = kTwoLn2 * s1[j].x;  // staged -> (A, B, C)
        g6[0] = -(cA * sum[0] + cB * sum[1]);
        g6[1] = -(cB * sum[0] + cC * sum[1]);
        g6[2] = 0.5f * sum[2];
        g6[3] = sum[3];
        g6[4] = 0.5f * sum[4];
        g6[5] = sum[5];
      }
      const int slot = nq + j;
      qit[slot] = mj != 0u ? sit[j] : -1;
#pragma unroll
      for (int q = 0; q < kPoseRow; ++q) qsum[q * kPoseQueue + slot] = g6[q];
    }
    nq += cnt;
    if (nq + kPoseChunk > kPoseQueue || chunk == start) {
      __syncthreads();
      const int t = threadIdx.x;
      float pc[kPoseAcc];
#pragma unroll
      for (int k = 0; k < kPoseAcc; ++k) pc[k] = 0.f;
      if (t < nq && qit[t] >= 0) {
        const int64_t it = qit[t];
        float g6[kPoseRow];
#pragma unroll
        for (int q = 0; q < kPoseRow; ++q) g6[q] = qsum[q * kPoseQueue + t];
        float Rd[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f}, td[3] = {0.f, 0.f, 0.f};
        if (pose) {
          const float* pr = pose + 7 * c.r;
          quat_to_rot(pr[0], pr[1], pr[2], pr[3], Rd);
          td[0] = pr[4];
          td[1] = pr[5];
          td[2] = pr[6];
        }
        const float4 a0 = aux[it * 3 + 0], a1 = aux[it * 3 + 1], a2 = aux[it * 3 + 2];
        const float p[3] = {a0.x, a0.y, a0.z};
        const float s6[6] = {a0.w, a1.x, a1.y, a1.z, a1.w, a2.x};
        float Sc[9], dp[3], Gm[9];
        sym3(s6, Sc);
        camera_space_grads(p, Sc, J.fx, J.fy, g6, dp, Gm);
        pose_contrib(p, Sc, Rd, td, dp, Gm, pc);
      }
      // fixed-order reduction of this round over the block
      {
        const float out = wave_sums<kPoseAcc>(pc, lane);
        const int v = wave_value<kPoseAcc>(lane);
        if (v >= 0) wred[w][v] = out;
      }
      __syncthreads();
      if (t < kPoseAcc) total += (wred[0][t] + wred[1][t]) + (wred[2][t] + wred[3][t]);
      nq = 0;
    }
    __syncthreads();
  }
  if ((int)threadIdx.x < kPoseAcc) tile_part[(int64_t)tile * kPoseAcc + threadIdx.x] = total;
}

// One block per tile (XCD-aware mapping), for launches with few tiles per
// resident block.
__global__ __launch_bounds__(kBlock) void k_composite_bwd_pose(const JobDev* __restrict__ jobs,
                                                               const int32_t* __restrict__ tile_off, int R,
                                                               int T_total, const float4* __restrict__ rec,
                                                               const float4* __restrict__ aux,
                                                               const float* __restrict__ pose,
                                                               const int32_t* __restrict__ items,
                                                               const int32_t* __restrict__ range,
                                                               const uint64_t* __restrict__ used, int64_t ustride,
                                                               float bg0, float bg1, float bg2,
                                                               const float* __restrict__ fwd_T,
                                                               const int32_t* __restrict__ fwd_n,
                                                               const float* __restrict__ up_rgb,
                                                               const float* __restrict__ up_depth,
                                                               const float* __restrict__ up_alpha,
                                                               const float* __restrict__ up_scale,
                                                               float* __restrict__ tile_part, L1Targets l1) {
  const int tile = xcd_remap(blockIdx.x, T_total);
  if (tile >= T_total) return;
  composite_bwd_pose_tile(jobs, tile_off, R, T_total, rec, aux, pose, items, range, used, ustride, bg0, bg1, bg2,
                          fwd_T, fwd_n, up_rgb, up_depth, up_alpha, up_scale, tile_part, l1, tile);
}

// Six waves per SIMD (at most 80 VGPRs, a few spilled): the walk now takes
// only entries with an active lane, and latency hiding pays (one 16-view
// registration pair: 104 VGPRs / 4 waves 0.228 s, 5 waves 0.216 s, 6 waves
// 0.214 s).
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_composite_bwd_pose_persistent(
    const JobDev* __restrict__ jobs,
    const int32_t* __restrict__ tile_off, int R, int T_total, const float4* __restrict__ rec,
    const float4* __restrict__ aux, const float* __restrict__ pose, const int32_t* __restrict__ items,
    const int32_t* __restrict__ range, const uint64_t* __restrict__ used, int64_t ustride, float bg0, float bg1,
    float bg2, const float* __restrict__ fwd_T,
    const int32_t* __restrict__ fwd_n, const float* __restrict__ up_rgb, const float* __restrict__ up_depth,
    const float* __restrict__ up_alpha, const float* __restrict__ up_scale, float* __restrict__ tile_part,
    TileQueue* __restrict__ queue, int nstatic, L1Targets l1) {
  __shared__ int s_tile;
  bool first = true;
  uint32_t dead = 0;
  for (;;) {
    const int tile = claim_tile(queue, T_total, nstatic, first, dead, &s_tile);
    if (tile < 0) break;
    composite_bwd_pose_tile(jobs, tile_off, R, T_total, rec, aux, pose, items, range, used, ustride, bg0, bg1, bg2,
                            fwd_T, fwd_n, up_rgb, up_depth, up_alpha, up_scale, tile_part, l1, tile);
  }
  release_queue(queue);
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
      float4 a = rec[it * 3 + 0], b = rec[it * 3 + 1];
      stage_conic(a, b);
      s0[threadIdx.x] = a;
      s1[threadIdx.x] = b;
    }
    __syncthreads();
    const int cnt = min(kBlock, end - chunk);
    for (int j = 0; j < cnt; ++j) {
      if (chunk + j - start >= nl) break;
      const float4 a = s0[j];
      const float4 b = s1[j];
      const float dx = fx - a.x, dy = fy - a.y;
      const float sl = falloff_log2(a.z, a.w, b.x, dx, dy);
      if (composited(sl, b)) ++comp;
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

// Grid of a backward compositing kernel.  With more than 4 tiles per
// resident block (residency = occupancy x compute units, as the runtime
// reports it) the persistent kernel runs: nstatic = the resident blocks get
// the statically mapped first tiles and then claim from the counters, and
// one more block per compute unit fills slots the runtime's estimate leaves
// empty (such blocks only claim, so if they cannot be resident they start
// late, find the queues drained and exit).  With fewer tiles the plain
// one-block-per-tile kernel is faster (the loop-and-claim wrapper cost 4-5 %
// on the 1200x680 render loop), with many the queues are (one 16-view
// registration iteration: 8.5 % faster).  The residency is queried once per
// (kernel, device) and cached.  The environment variable LS_PERSISTENT=0 / 1
// forces the plain / persistent form (read at every launch; for tests and
// measurements).
static inline int xcd_grid(int total) { return 8 * ((total + 7) / 8); }

static int forced_persistent() {
  const char* e = std::getenv("LS_PERSISTENT");
  if (!e || (e[0] != '0' && e[0] != '1') || e[1] != '\0') return -1;
  return e[0] - '0';
}

struct PersistentGrid {
  bool on;
  int blocks, nstatic;
};
static PersistentGrid persistent_grid(int which, const void* kernel, int T) {
  static std::mutex mu;
  static int cache[2][64][2] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  int resident, cus;
  {
    std::lock_guard<std::mutex> g(mu);
    resident = cache[which][dev][0];
    cus = cache[which][dev][1];
    if (resident == 0) {
      int per = 0;
      cus = 0;
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock, 0) != hipSuccess || per <= 0) per = 1;
      resident = cache[which][dev][0] = cus * per;
      cache[which][dev][1] = cus;
    }
  }
  PersistentGrid g;
  const int forced = forced_persistent();
  g.on = forced >= 0 ? forced == 1 : T > 4 * resident;
  g.blocks = g.on ? resident + cus : xcd_grid(T);
  g.nstatic = g.on ? resident : 0;
  return g;
}

void launch_composite_fwd(const JobDev* jobs, const int32_t* tile_off, int R, int T, const float* rec,
                          const int32_t* items, const int32_t* range, const float* bg, float* rgb, float* depth,
                          float* alpha, float* Tf, int32_t* nl, uint64_t* used, int64_t ustride,
                          hipStream_t s) {
  if (T <= 0) return;
  // always one block per band: a band is short, and claiming tiles from the
  // queues cost more than it balanced (registration iteration A/B: 1.3 %
  // slower persistent)
  // LS_COVER=0 (read at every launch; for tests and measurements): stage by
  // the band rectangle test alone, whatever pixels have stopped
  const char* cv = std::getenv("LS_COVER");
  const int cover = (cv && cv[0] == '0' && cv[1] == '\0') ? 0 : 1;
  hipLaunchKernelGGL(k_composite_fwd_band, dim3(xcd_grid(4 * T)), dim3(64), 0, s, jobs, tile_off, R, T,
                     reinterpret_cast<const float4*>(rec), items, range, bg[0], bg[1], bg[2], rgb, depth, alpha, Tf,
                     nl, used, ustride, cover);
}

void launch_composite_bwd(const JobDev* jobs, const int32_t* tile_off, int R, int T, const float* rec,
                          const float* aux, const float* pose, const int32_t* items, const int32_t* range,
                          const uint64_t* used, int64_t ustride, const float* bg, const float* Tf,
                          const int32_t* nl,
                          const float* up_rgb, const float* up_depth, const float* up_alpha, const float* up_scale,
                          float* g2d, float* tile_part, int pose_only, void* queues, hipStream_t s,
                          const L1Targets* l1) {
  if (T <= 0) return;
  const L1Targets l1v = l1 ? *l1 : L1Targets{nullptr, nullptr, nullptr, nullptr, nullptr};
  const float4* rec4 = reinterpret_cast<const float4*>(rec);
  const float4* aux4 = reinterpret_cast<const float4*>(aux);
  if (pose_only) {
    const PersistentGrid g = persistent_grid(1, reinterpret_cast<const void*>(k_composite_bwd_pose_persistent), T);
    if (g.on)
      hipLaunchKernelGGL(k_composite_bwd_pose_persistent, dim3(g.blocks), dim3(kBlock), 0, s, jobs, tile_off, R, T,
                         rec4, aux4, pose, items, range, used, ustride, bg[0], bg[1], bg[2], Tf, nl, up_rgb, up_depth,
                         up_alpha, up_scale, tile_part, reinterpret_cast<TileQueue*>(queues) + 1, g.nstatic, l1v);
    else
      hipLaunchKernelGGL(k_composite_bwd_pose, dim3(g.blocks), dim3(kBlock), 0, s, jobs, tile_off, R, T, rec4, aux4,
                         pose, items, range, used, ustride, bg[0], bg[1], bg[2], Tf, nl, up_rgb, up_depth, up_alpha,
                         up_scale, tile_part, l1v);
  } else {
    const PersistentGrid g = persistent_grid(0, reinterpret_cast<const void*>(k_composite_bwd_persistent), T);
    if (g.on)
      hipLaunchKernelGGL(k_composite_bwd_persistent, dim3(g.blocks), dim3(kBlock), 0, s, jobs, tile_off, R, T, rec4,
                         items, range, used, ustride, bg[0], bg[1], bg[2], Tf, nl, up_rgb, up_depth, up_alpha, up_scale,
                         g2d, reinterpret_cast<TileQueue*>(queues) + 0, g.nstatic, l1v);
    else
      hipLaunchKernelGGL(k_composite_bwd, dim3(g.blocks), dim3(kBlock), 0, s, jobs, tile_off, R, T, rec4, items, range,
                         used, ustride, bg[0], bg[1], bg[2], Tf, nl, up_rgb, up_depth, up_alpha, up_scale, g2d,
                         l1v);
  }
}
}  // namespace ls

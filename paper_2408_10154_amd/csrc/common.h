// Internal definitions shared by the gfx950 kernels and the host API.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "loopsplat.h"

namespace ls {

constexpr int kTile = LS_TILE;
constexpr int kBlock = 256;         // one 16x16 tile per block, 4 wave64
constexpr int kSortThreads = 256;   // radix sort block
// Radix digit widths (the sort kernels take any width whose bin count is a
// multiple of the block size).  11-bit depth digits (3 passes instead of 4)
// measured 3 % slower on the render loop: the 2048-bin histograms, row scans
// and scatter set-up cost more than the pass they save.
constexpr int kDepthDigitBits = 8;  // depth keys: 4 passes over 32 bits
constexpr int kTileDigitBits = 8;   // tile keys: ceil(bits / 8) passes of at most 8 bits
constexpr int kMaxSortBins = 1 << (kDepthDigitBits > kTileDigitBits ? kDepthDigitBits : kTileDigitBits);
constexpr int kSortItems = 16;      // most items per thread per sort block
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int64_t kSortBlocksTarget = 1024;  // blocks a sort pass aims for (fills the chip)

// Rounds of kSortThreads items per sort block for n keys: as few as keep
// about kSortBlocksTarget blocks busy, between 2 and kSortItems (one round
// per block measured slower: the per-block set-up then dominates).  Host and
// device use it for the launch grids and for the workspace layout.
__host__ __device__ inline int sort_rounds(int64_t n) {
  const int64_t r = (n + kSortBlocksTarget * kSortThreads - 1) / (kSortBlocksTarget * kSortThreads);
  return (int)(r < 2 ? 2 : (r > kSortItems ? kSortItems : r));
}
__host__ __device__ inline int64_t sort_blocks(int64_t n) {
  const int64_t per = (int64_t)sort_rounds(n) * kSortThreads;
  return (n + per - 1) / per;
}
// Digit width of the tile-key passes for keys of `bits` bits: as many passes
// as 8-bit digits need, the bits split evenly between them, rounded up to 6,
// 7 or 8 (12-bit keys: two 6-bit passes).  Fewer bins per pass give each sort
// block longer runs of equal digits to count and to write.
__host__ __device__ inline int tile_digit_bits(int bits) {
  const int passes = bits <= 0 ? 1 : (bits + kTileDigitBits - 1) / kTileDigitBits;
  const int w = (bits + passes - 1) / passes;
  return w < 6 ? 6 : (w > kTileDigitBits ? kTileDigitBits : w);
}
__host__ __device__ inline int tile_passes(int bits) {
  return bits <= 0 ? 0 : (bits + tile_digit_bits(bits) - 1) / tile_digit_bits(bits);
}

// Tile instances emitted per wave: an eighth of a tile-sort block, so the
// kEmitWaves waves of an emission block fill exactly the positions of one
// block of the first tile pass and can count its digits.  The first item of
// every span is recorded while the item offsets are formed.
constexpr int kEmitWaves = 8;
__host__ __device__ inline int64_t emit_span(int64_t cap) {
  return (int64_t)sort_rounds(cap) * (kSortThreads / kEmitWaves);
}
__host__ __device__ inline int64_t emit_spans(int64_t cap) { return (cap + emit_span(cap) - 1) / emit_span(cap); }
constexpr int kGrad2D = 10;         // du dv dA dB dC dop dz dr dg db
constexpr int kPoseAcc = 12;        // dL/dR (9, row-major) and dL/dt (3)
constexpr int kAuxFloats = 12;      // per item: camera-space mean (3), covariance (6), 0 x3

// Device view of one render job.
struct JobDev {
  const float* mean;
  const float* log_scale;
  const float* quat;
  const float* opac;
  const float* rgb;
  float fx, fy, cx, cy;
  int32_t n, W, H, TX, TY;
  int32_t tile_off;
  int32_t blk_off;  // first 256-item block of this render
  int32_t pad0;
  int64_t item_off;
  int64_t pix_off;
  float w2c[12];
  const float* tgt_rgb;    // optional per-render measurements [3][H][W] (internal batches)
  const float* tgt_depth;  // [H][W]
};

// Gradient pointers of one render, device copy.
struct GradDev {
  float* mean;
  float* log_scale;
  float* quat;
  float* opac;
  float* rgb;
  int32_t shared;  // another render writes the same arrays: use atomics
  int32_t pad;
};

// Binary search: largest r in [0, R) with off[r] <= x (off is [R+1], ascending).
template <typename T>
__device__ __forceinline__ int find_segment(const T* off, int R, T x) {
  int lo = 0, hi = R - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Rotation matrix (row-major) of q / |q|, q = (w, x, y, z).
__device__ __forceinline__ void quat_to_rot(float w, float x, float y, float z, float* R) {
  float inv = rsqrtf(w * w + x * x + y * y + z * z);
  w *= inv; x *= inv; y *= inv; z *= inv;
  R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z);       R[2] = 2.f * (x * z + w * y);
  R[3] = 2.f * (x * y + w * z);       R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
  R[6] = 2.f * (x * z - w * y);       R[7] = 2.f * (y * z + w * x);       R[8] = 1.f - 2.f * (x * x + y * y);
}

// Effective world-to-camera W (row-major 3x3) and t of a job and its pose.
__device__ __forceinline__ void camera_of(const JobDev& j, const float* pose, float* W, float* t) {
  const float* A = j.w2c;
  if (pose == nullptr) {
    W[0] = A[0]; W[1] = A[1]; W[2] = A[2];
    W[3] = A[4]; W[4] = A[5]; W[5] = A[6];
    W[6] = A[8]; W[7] = A[9]; W[8] = A[10];
    t[0] = A[3]; t[1] = A[7]; t[2] = A[11];
    return;
  }
  float Rd[9];
  quat_to_rot(pose[0], pose[1], pose[2], pose[3], Rd);
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c)
      W[r * 3 + c] = Rd[r * 3 + 0] * A[0 * 4 + c] + Rd[r * 3 + 1] * A[1 * 4 + c] + Rd[r * 3 + 2] * A[2 * 4 + c];
    t[r] = Rd[r * 3 + 0] * A[3] + Rd[r * 3 + 1] * A[7] + Rd[r * 3 + 2] * A[11] + pose[4 + r];
  }
}

// Tile rectangle in FP32 from the projected centre and integer radius; the
// same instruction sequence is used for counting and for emission.
struct Rect { int x0, x1, y0, y1; };
__device__ __forceinline__ Rect tile_rect(float u, float v, int r, int TX, int TY) {
  const float rf = (float)r;
  const float inv = 1.0f / (float)kTile;
  Rect o;
  o.x0 = min(max((int)floorf((u - rf) * inv), 0), TX);
  o.x1 = min(max((int)floorf((u + rf) * inv) + 1, 0), TX);
  o.y0 = min(max((int)floorf((v - rf) * inv), 0), TY);
  o.y1 = min(max((int)floorf((v + rf) * inv) + 1, 0), TY);
  return o;
}

// The compositing kernels stage each splat's conic (A, B, C) pre-scaled to
// (A / 2, B, C / 2) log2(e), so that the falloff sigma = (A dx^2 + 2 B dx dy +
// C dy^2) / 2 comes out as sigma log2(e) and exp(-sigma) = 2^(-that): no
// per-pixel multiply before the exponential.  Factors back to (A, B, C).
constexpr float kHalfLog2e = 0.72134752044448170368f;  // log2(e) / 2
constexpr float kLog2e = 1.44269504088896340736f;
constexpr float kLn2 = 0.69314718055994530942f;
constexpr float kTwoLn2 = 1.38629436111989061883f;

// The staged record also carries, in its free slot b.w, the bits of the
// bound on sigma log2(e) within which the splat is composited: alpha =
// opacity 2^(-sigma log2 e) >= 1/255 with sigma >= 0 holds (in exact
// arithmetic; in FP32 up to a few ulps of the threshold) when
// 0 <= sigma log2(e) <= log2(255 opacity), i.e. when the bits of sigma log2(e)
// (a float >= +0, so ordered like its bits; a negative sigma has the sign bit
// and fails) are below those of log2(255 opacity) plus one.  One unsigned
// compare per pixel and entry replaces the two tests, and forward and
// backward take the same decisions from the same staged bound; below
// opacity 1/255 the bound is 0 and nothing passes.
__device__ __forceinline__ void stage_conic(float4& a, float4& b) {
  a.z *= kHalfLog2e;
  a.w *= kLog2e;
  b.x *= kHalfLog2e;
  const float t = __builtin_amdgcn_logf(b.y * (1.0f / LS_ALPHA_MIN));
  b.w = __uint_as_float(t >= 0.f ? __float_as_uint(t) + 1u : 0u);
}

// Whether a staged splat (b from stage_conic) is composited at a pixel whose
// sigma log2(e) is sl: alpha >= 1/255 and sigma >= 0, the test of both the
// forward and the backward.
__device__ __forceinline__ bool composited(float sl, const float4& b) {
  return __float_as_uint(sl) < __float_as_uint(b.w);
}

// sigma log2(e) at pixel offset (dx, dy) from a staged conic, as
// dx (hA dx + B dy) + hC dy^2 (three multiplies and two FMAs), with explicit
// FMAs so that forward and backward take identical decisions.
__device__ __forceinline__ float falloff_log2(float hA, float B, float hC, float dx, float dy) {
  return __builtin_fmaf(dx, __builtin_fmaf(hA, dx, B * dy), hC * dy * dy);
}

// The DPP reductions below use moves without an "old" operand (bound_ctrl
// set): every lane's source is in range for these patterns, and the
// compiler can fold each move into its add (v_add_f32 with a DPP operand).
// Full-wave (64-lane) sum; the total is returned in every lane.
__device__ __forceinline__ float wave_sum(float v) {
  // within rows of 16 lanes: swap pairs, quads, half-rows, rows
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));  // quad_perm 1,0,3,2
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));  // quad_perm 2,3,0,1
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, true)); // row_half_mirror
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x140, 0xF, 0xF, true)); // row_mirror
  // every lane of a row now holds the row sum; combine the four rows
  float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
  float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
  float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
  return (r0 + r1) + (r2 + r3);
}

// XCD-aware block -> work-unit map: consecutive work units (neighbouring
// tiles) go to the same XCD so its L2 holds the splats they share.  The grid
// must have 8 * ceil(total / 8) blocks; units >= total are idle.
__device__ __forceinline__ int xcd_remap(int b, int total) {
  const int per = (total + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ void atomic_add_f32(float* p, float v) {
  unsafeAtomicAdd(p, v);
}

// Image-space gradients of one Gaussian -> gradients w.r.t. its camera-space
// mean p (dp) and camera-space covariance Sc (G, symmetric 3x3), through
// u = fx x/z + cx, v = fy y/z + cy, Sigma_2D = J Sc J^T + eps I and the conic
// (A, B, C) = (c, -b, a) / det.  g = (du, dv, dA, dB, dC, dz).
__device__ __forceinline__ void camera_space_grads(const float* p, const float* Sc, float fx, float fy,
                                                   const float* g, float* dp, float* G) {
  const float px = p[0], py = p[1], pz = p[2];
  const float du = g[0], dv = g[1], dA = g[2], dB = g[3], dC = g[4], dz = g[5];
  const float iz = 1.0f / pz;
  const float J0[3] = {fx * iz, 0.f, -fx * px * iz * iz};
  const float J1[3] = {0.f, fy * iz, -fy * py * iz * iz};
  float SJ0[3], SJ1[3];  // Sc J0^T, Sc J1^T
  for (int i = 0; i < 3; ++i) {
    SJ0[i] = Sc[i * 3 + 0] * J0[0] + Sc[i * 3 + 1] * J0[1] + Sc[i * 3 + 2] * J0[2];
    SJ1[i] = Sc[i * 3 + 0] * J1[0] + Sc[i * 3 + 1] * J1[1] + Sc[i * 3 + 2] * J1[2];
  }
  const float a = J0[0] * SJ0[0] + J0[1] * SJ0[1] + J0[2] * SJ0[2] + LS_EPS_2D;
  const float b = J0[0] * SJ1[0] + J0[1] * SJ1[1] + J0[2] * SJ1[2];
  const float c = J1[0] * SJ1[0] + J1[1] * SJ1[1] + J1[2] * SJ1[2] + LS_EPS_2D;
  const float det = a * c - b * b;
  const float id2 = 1.0f / (det * det);
  const float ga = (-c * c * dA + b * c * dB - b * b * dC) * id2;
  const float gb = (2.f * b * c * dA - (det + 2.f * b * b) * dB + 2.f * a * b * dC) * id2;
  const float gc = (-b * b * dA + a * b * dB - a * a * dC) * id2;
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k)
      G[i * 3 + k] = ga * J0[i] * J0[k] + 0.5f * gb * (J0[i] * J1[k] + J1[i] * J0[k]) + gc * J1[i] * J1[k];
  const float gJ00 = 2.f * ga * SJ0[0] + gb * SJ1[0];
  const float gJ02 = 2.f * ga * SJ0[2] + gb * SJ1[2];
  const float gJ11 = gb * SJ0[1] + 2.f * gc * SJ1[1];
  const float gJ12 = gb * SJ0[2] + 2.f * gc * SJ1[2];
  const float iz2 = iz * iz, iz3 = iz2 * iz;
  dp[0] = du * fx * iz - gJ02 * fx * iz2;
  dp[1] = dv * fy * iz - gJ12 * fy * iz2;
  dp[2] = -du * fx * px * iz2 - dv * fy * py * iz2 + dz - gJ00 * fx * iz2 + gJ02 * 2.f * fx * px * iz3 -
          gJ11 * fy * iz2 + gJ12 * 2.f * fy * py * iz3;
}

// Contribution of a Gaussian to dL/dR_d (9, row-major) and dL/dt_d (3) of its
// render's camera-frame correction (R_d, t_d): p = R_d p0 + t_d and
// Sc = R_d Sc0 R_d^T give dL/dR_d = dp p0^T + 2 G Sc R_d, dL/dt_d = dp, with
// p0 = R_d^T (p - t_d).  Accumulated into acc[12].
__device__ __forceinline__ void pose_contrib(const float* p, const float* Sc, const float* Rd, const float* td,
                                             const float* dp, const float* G, float* acc) {
  const float d[3] = {p[0] - td[0], p[1] - td[1], p[2] - td[2]};
  float q0[3];
  for (int k = 0; k < 3; ++k) q0[k] = Rd[0 * 3 + k] * d[0] + Rd[1 * 3 + k] * d[1] + Rd[2 * 3 + k] * d[2];
  float GS[9];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) GS[i * 3 + k] = G[i * 3 + 0] * Sc[0 * 3 + k] + G[i * 3 + 1] * Sc[1 * 3 + k] + G[i * 3 + 2] * Sc[2 * 3 + k];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k)
      acc[i * 3 + k] += dp[i] * q0[k] + 2.f * (GS[i * 3 + 0] * Rd[0 * 3 + k] + GS[i * 3 + 1] * Rd[1 * 3 + k] + GS[i * 3 + 2] * Rd[2 * 3 + k]);
  acc[9] += dp[0];
  acc[10] += dp[1];
  acc[11] += dp[2];
}

// Row-major 3x3 covariance from the 6 stored entries (xx xy xz yy yz zz).
__device__ __forceinline__ void sym3(const float* s6, float* S) {
  S[0] = s6[0]; S[1] = s6[1]; S[2] = s6[2];
  S[3] = s6[1]; S[4] = s6[3]; S[5] = s6[4];
  S[6] = s6[2]; S[7] = s6[4]; S[8] = s6[5];
}

}  // namespace ls

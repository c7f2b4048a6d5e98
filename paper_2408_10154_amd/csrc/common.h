// Internal definitions shared by the gfx950 kernels and the host API.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "loopsplat.h"

namespace ls {

constexpr int kTile = LS_TILE;
constexpr int kBlock = 256;         // one 16x16 tile per block, 4 wave64
constexpr int kSortThreads = 256;   // radix sort block
constexpr int kSortItems = 16;      // items per thread per sort block
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kGrad2D = 10;         // du dv dA dB dC dop dz dr dg db
constexpr int kPoseAcc = 12;        // dL/dR (9, row-major) and dL/dt (3)

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

// Gaussian falloff exponent at pixel offset (dx, dy) with explicit FMAs so
// that forward and backward take identical decisions.
__device__ __forceinline__ float falloff(float A, float B, float C, float dx, float dy) {
  return __builtin_fmaf(0.5f * A * dx, dx, __builtin_fmaf(B * dx, dy, 0.5f * C * dy * dy));
}

// Full-wave (64-lane) sum; the total is returned in every lane.
__device__ __forceinline__ float wave_sum(float v) {
  // within rows of 16 lanes: swap pairs, quads, half-rows, rows
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));  // quad_perm 1,0,3,2
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));  // quad_perm 2,3,0,1
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false)); // row_half_mirror
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false)); // row_mirror
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

}  // namespace ls

// Geometric overlap ratio of two submaps (supplement, loop detection,
// Eq. 9): the fraction of reciprocal nearest-neighbour pairs between the
// Gaussian means of P, moved by an estimate of T_{P->Q}, and those of Q whose
// distance is below tau_1.
//
// Every nearest neighbour is exact: both point sets are sorted along a
// 30-bit Morton curve and cut into leaf blocks of 64 points (one wave) and
// superblocks of 32 leaves, each with its bounding box.  A wave of 64 query
// points visits the candidate superblocks and leaves outward from the
// query's place on the curve and skips any box that is farther from every
// one of its points than that point's current best (with a margin over FP32
// rounding), so no skipped point can win or tie.  Distances and the
// transform follow one fixed FP32 rounding sequence (no fused multiply-add)
// so that matches and ties are reproducible: d^2 = (dx^2 + dy^2) + dz^2,
// ties to the lower index.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "kernels.h"

namespace ls {

constexpr int kOvLeaf = 64;       // points per leaf block (one wave)
constexpr int kOvSuper = 32;      // leaves per superblock
constexpr int kOvBoxBlocks = 256; // blocks of the bounding-box reduction
constexpr float kOvPrune = 1.f - 1e-5f;  // a box is skipped only if lb^2 * kOvPrune > bound

__device__ __forceinline__ float sq_dist_rn(float ax, float ay, float az, float bx, float by, float bz) {
#pragma clang fp contract(off)
  const float dx = ax - bx, dy = ay - by, dz = az - bz;
  return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ float wave_min_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  return v;
}

// P moved by T (row-major 3x4): ((R_r0 x + R_r1 y) + R_r2 z) + t_r, each
// operation rounded to FP32 (contraction into fused multiply-adds is off in
// this and the distance function).
struct Rigid {
  float m[12];
};
__global__ __launch_bounds__(256) void k_ov_transform(const float* __restrict__ p, int n, Rigid T,
                                                      float* __restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float x = p[i], y = p[(int64_t)n + i], z = p[2 * (int64_t)n + i];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma clang fp contract(off)
    const float* M = T.m + 4 * r;
    out[(int64_t)r * n + i] = ((M[0] * x + M[1] * y) + M[2] * z) + M[3];
  }
}

// Bounding box of both sets: per-block partials, then one block.
__global__ __launch_bounds__(256) void k_ov_box_part(const float* __restrict__ a, int na, const float* __restrict__ b,
                                                     int nb, float* __restrict__ part) {
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < (int64_t)na + nb; i += (int64_t)gridDim.x * kBlock) {
    const float* s = i < na ? a : b;
    const int64_t n = i < na ? na : nb, k = i < na ? i : i - na;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float v = s[d * n + k];
      lo[d] = fminf(lo[d], v);
      hi[d] = fmaxf(hi[d], v);
    }
  }
  __shared__ float ws[4][6];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = wave_min_f(lo[d]);
    hi[d] = wave_max_f(hi[d]);
  }
  if ((threadIdx.x & 63) == 0)
    for (int d = 0; d < 3; ++d) {
      ws[threadIdx.x >> 6][d] = lo[d];
      ws[threadIdx.x >> 6][3 + d] = hi[d];
    }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int d = threadIdx.x;
    float v = ws[0][d];
    for (int w = 1; w < 4; ++w) v = d < 3 ? fminf(v, ws[w][d]) : fmaxf(v, ws[w][d]);
    part[6 * blockIdx.x + d] = v;
  }
}

__global__ __launch_bounds__(256) void k_ov_box_final(const float* __restrict__ part, int nblk,
                                                      float* __restrict__ box) {
  __shared__ float ws[4][6];
  float v[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) v[d] = d < 3 ? INFINITY : -INFINITY;
  for (int k = threadIdx.x; k < nblk; k += kBlock)
#pragma unroll
    for (int d = 0; d < 6; ++d) v[d] = d < 3 ? fminf(v[d], part[6 * k + d]) : fmaxf(v[d], part[6 * k + d]);
#pragma unroll
  for (int d = 0; d < 6; ++d) v[d] = d < 3 ? wave_min_f(v[d]) : wave_max_f(v[d]);
  if ((threadIdx.x & 63) == 0)
    for (int d = 0; d < 6; ++d) ws[threadIdx.x >> 6][d] = v[d];
  __syncthreads();
  if (threadIdx.x < 6) {
    const int d = threadIdx.x;
    float r = ws[0][d];
    for (int w = 1; w < 4; ++w) r = d < 3 ? fminf(r, ws[w][d]) : fmaxf(r, ws[w][d]);
    box[d] = r;
  }
}

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// 30-bit Morton code of every point on a cubic grid of 1024 cells per axis
// over the common box; value = the point's index.
__global__ __launch_bounds__(256) void k_ov_codes(const float* __restrict__ p, int n, const float* __restrict__ box,
                                                  uint32_t* __restrict__ code, uint32_t* __restrict__ idx) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float ext = fmaxf(fmaxf(box[3] - box[0], box[4] - box[1]), box[5] - box[2]);
  const float inv = ext > 0.f ? 1023.f / ext : 0.f;
  uint32_t c = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float q = (p[(int64_t)d * n + i] - box[d]) * inv;
    const uint32_t u = (uint32_t)fminf(fmaxf(q, 0.f), 1023.f);
    c |= spread10(u) << d;
  }
  code[i] = c;
  idx[i] = (uint32_t)i;
}

// Points in curve order (SoA x, y, z, original index, code) and one box per leaf
// (one wave per leaf).
__global__ __launch_bounds__(256) void k_ov_gather(const float* __restrict__ p, int n,
                                                   const uint32_t* __restrict__ order,
                                                   const uint32_t* __restrict__ code, float* __restrict__ sp,
                                                   int32_t* __restrict__ sidx, uint32_t* __restrict__ scode,
                                                   float* __restrict__ leaf_box) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool v = i < n;
  float c[3] = {0.f, 0.f, 0.f};
  if (v) {
    const uint32_t k = order[i];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      c[d] = p[(int64_t)d * n + k];
      sp[(int64_t)d * n + i] = c[d];
    }
    sidx[i] = (int32_t)k;
    scode[i] = code[i];
  }
  float lo[3], hi[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = wave_min_f(v ? c[d] : INFINITY);
    hi[d] = wave_max_f(v ? c[d] : -INFINITY);
  }
  const int leaf = i / kOvLeaf;
  if ((threadIdx.x & 63) == 0 && leaf * kOvLeaf < n)
    for (int d = 0; d < 3; ++d) {
      leaf_box[6 * leaf + d] = lo[d];
      leaf_box[6 * leaf + 3 + d] = hi[d];
    }
}

__global__ __launch_bounds__(256) void k_ov_super(const float* __restrict__ leaf_box, int nleaf,
                                                  float* __restrict__ super_box, int nsuper) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= nsuper) return;
  float b[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  const int l1 = (s + 1) * kOvSuper < nleaf ? (s + 1) * kOvSuper : nleaf;
  for (int l = s * kOvSuper; l < l1; ++l)
    for (int d = 0; d < 3; ++d) {
      b[d] = fminf(b[d], leaf_box[6 * l + d]);
      b[3 + d] = fmaxf(b[3 + d], leaf_box[6 * l + 3 + d]);
    }
  for (int d = 0; d < 6; ++d) super_box[6 * s + d] = b[d];
}

struct OvSet {
  const float* p;        // [3][n] in curve order
  const int32_t* idx;    // original indices
  const uint32_t* code;  // sorted Morton codes
  const float* leaf;     // [nleaf][6]
  const float* super;    // [nsuper][6]
  int n, nleaf, nsuper;
};

// Squared distance from a point to a box (min xyz, max xyz); 0 inside.
__device__ __forceinline__ float point_box_dist2(float x, float y, float z, const float* b) {
  const float g0 = fmaxf(fmaxf(b[0] - x, x - b[3]), 0.f);
  const float g1 = fmaxf(fmaxf(b[1] - y, y - b[4]), 0.f);
  const float g2 = fmaxf(fmaxf(b[2] - z, z - b[5]), 0.f);
  return g0 * g0 + g1 * g1 + g2 * g2;
}

// One wave per query leaf: the exact nearest candidate of each of its points.
// The wave first scans the candidate leaf at the query leaf's place on the
// curve (a close first bound), then every superblock outward from there; a
// superblock or leaf is skipped when, for every lane, its box is farther than
// that lane's current best (scaled by kOvPrune against FP32 rounding), so a
// skipped point can neither win nor tie.
__device__ __forceinline__ void ov_scan_leaf(const OvSet& c, int l, int lane, float px, float py, float pz,
                                             float& best, int& bi, float4* stage) {
  // the leaf's candidates go through the wave's LDS slot and are read back
  // with one uniform (broadcast) load each
  const int ci = l * kOvLeaf + lane;
  const bool cv = ci < c.n;
  const float ax = cv ? c.p[ci] : 0.f, ay = cv ? c.p[(int64_t)c.n + ci] : 0.f;
  const float az = cv ? c.p[2 * (int64_t)c.n + ci] : 0.f;
  const int aid = cv ? c.idx[ci] : 0;
  stage[lane] = make_float4(ax, ay, az, __int_as_float(aid));
  __builtin_amdgcn_wave_barrier();
  const int cnt = c.n - l * kOvLeaf < kOvLeaf ? c.n - l * kOvLeaf : kOvLeaf;
#pragma unroll 4
  for (int j = 0; j < cnt; ++j) {
    const float4 b = stage[j];
    const float d = sq_dist_rn(px, py, pz, b.x, b.y, b.z);
    const int bid = __float_as_int(b.w);
    const bool take = d < best || (d == best && bid < bi);
    best = take ? d : best;
    bi = take ? bid : bi;
  }
  __builtin_amdgcn_wave_barrier();  // every lane has read the slot before it is refilled
}

__global__ __launch_bounds__(256) void k_ov_nn(OvSet q, OvSet c, int32_t* __restrict__ nn_out) {
  __shared__ float4 stage_all[kBlock];
  const int leaf = (int)((blockIdx.x * (int64_t)kBlock + threadIdx.x) / kOvLeaf);
  const int lane = threadIdx.x & 63;
  float4* stage = stage_all + (threadIdx.x & ~63);  // this wave's slot
  if (leaf >= q.nleaf) return;  // whole waves; no block-wide barrier follows
  const int qi = leaf * kOvLeaf + lane;
  const bool qv = qi < q.n;
  const float px = qv ? q.p[qi] : 0.f, py = qv ? q.p[(int64_t)q.n + qi] : 0.f;
  const float pz = qv ? q.p[2 * (int64_t)q.n + qi] : 0.f;
  // the candidate leaf holding the query leaf's first code on the curve
  const uint32_t code0 = q.code[leaf * kOvLeaf];
  int lo = 0, hi = c.n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (c.code[mid] < code0) lo = mid + 1; else hi = mid;
  }
  const int l0 = lo / kOvLeaf < c.nleaf - 1 ? lo / kOvLeaf : c.nleaf - 1;
  const int s0 = l0 / kOvSuper;
  float best = INFINITY;
  int bi = 0x7fffffff;
  ov_scan_leaf(c, l0, lane, px, py, pz, best, bi, stage);
  for (int k = 0; k < 2 * c.nsuper; ++k) {
    const int s = (k & 1) ? s0 + (k + 1) / 2 : s0 - k / 2;
    if (s < 0 || s >= c.nsuper) continue;
    if (!__ballot(qv && point_box_dist2(px, py, pz, c.super + 6 * s) * kOvPrune <= best)) continue;
    const int l1 = (s + 1) * kOvSuper < c.nleaf ? (s + 1) * kOvSuper : c.nleaf;
    for (int l = s * kOvSuper; l < l1; ++l) {
      if (l == l0) continue;
      if (!__ballot(qv && point_box_dist2(px, py, pz, c.leaf + 6 * l) * kOvPrune <= best)) continue;
      ov_scan_leaf(c, l, lane, px, py, pz, best, bi, stage);
    }
  }
  if (qv) nn_out[q.idx[qi]] = bi;
}

// Reciprocity and the threshold test per point of P; one integer atomic per
// block and count.
__global__ __launch_bounds__(256) void k_ov_count(const float* __restrict__ pt, int np, const float* __restrict__ q,
                                                  int nq, const int32_t* __restrict__ nn_pq,
                                                  const int32_t* __restrict__ nn_qp, float tau2,
                                                  int32_t* __restrict__ counts) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  bool pair = false, in = false;
  if (i < np) {
    const int j = nn_pq[i];
    if (j >= 0 && j < nq && nn_qp[j] == i) {
      pair = true;
      const float d = sq_dist_rn(pt[i], pt[(int64_t)np + i], pt[2 * (int64_t)np + i], q[j], q[(int64_t)nq + j],
                                 q[2 * (int64_t)nq + j]);
      in = d < tau2;
    }
  }
  __shared__ int32_t ws[4][2];
  const uint64_t bp = __ballot(pair), bn = __ballot(in);
  if ((threadIdx.x & 63) == 0) {
    ws[threadIdx.x >> 6][0] = (int32_t)__popcll(bp);
    ws[threadIdx.x >> 6][1] = (int32_t)__popcll(bn);
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int32_t v = (ws[0][threadIdx.x] + ws[1][threadIdx.x]) + (ws[2][threadIdx.x] + ws[3][threadIdx.x]);
    if (v) atomicAdd(&counts[threadIdx.x], v);
  }
}

// Workspace layout (all pieces 256-byte aligned).
struct OvLayout {
  size_t pt, box_part, box, code_a, idx_a, code_b, idx_b, hist, digits, set_p[5], set_q[5], total;
};
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
static OvLayout ov_layout(int np, int nq) {
  OvLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  const int64_t nmax = std::max(np, nq);
  L.pt = take(12 * (size_t)np);
  L.box_part = take(4 * 6 * kOvBoxBlocks);
  L.box = take(4 * 6);
  L.code_a = take(4 * (size_t)nmax);
  L.idx_a = take(4 * (size_t)nmax);
  L.code_b = take(4 * (size_t)nmax);
  L.idx_b = take(4 * (size_t)nmax);
  L.hist = take(4 * 256 * (size_t)std::max<int64_t>(sort_blocks(nmax), 1));
  L.digits = take(4 * 256);
  for (int s = 0; s < 2; ++s) {
    const int n = s ? nq : np;
    const int nleaf = (n + kOvLeaf - 1) / kOvLeaf, nsuper = (nleaf + kOvSuper - 1) / kOvSuper;
    size_t* S = s ? L.set_q : L.set_p;
    S[0] = take(12 * (size_t)n);         // points in curve order
    S[1] = take(4 * (size_t)n);          // original indices
    S[2] = take(4 * (size_t)n);          // sorted codes
    S[3] = take(24 * (size_t)nleaf);     // leaf boxes
    S[4] = take(24 * (size_t)nsuper);    // superblock boxes
  }
  L.total = o;
  return L;
}

size_t overlap_workspace_bytes(int np, int nq) { return ov_layout(np, nq).total; }

void launch_overlap(const float* p_mean, int np, const float* q_mean, int nq, const float* T, float tau,
                    int32_t* nn_pq, int32_t* nn_qp, int32_t* counts, void* work, hipStream_t s) {
  const OvLayout L = ov_layout(np, nq);
  char* w = static_cast<char*>(work);
  launch_fill_i32(counts, 2, 0, s);
  if (np == 0 || nq == 0) {
    launch_fill_i32(nn_pq, np, -1, s);
    launch_fill_i32(nn_qp, nq, -1, s);
    return;
  }
  float* pt = reinterpret_cast<float*>(w + L.pt);
  Rigid R;
  for (int k = 0; k < 12; ++k) R.m[k] = T[k];
  hipLaunchKernelGGL(k_ov_transform, dim3((np + kBlock - 1) / kBlock), dim3(kBlock), 0, s, p_mean, np, R, pt);
  float* box_part = reinterpret_cast<float*>(w + L.box_part);
  float* box = reinterpret_cast<float*>(w + L.box);
  hipLaunchKernelGGL(k_ov_box_part, dim3(kOvBoxBlocks), dim3(kBlock), 0, s, (const float*)pt, np, q_mean, nq,
                     box_part);
  hipLaunchKernelGGL(k_ov_box_final, dim3(1), dim3(kBlock), 0, s, (const float*)box_part, kOvBoxBlocks, box);
  OvSet set[2];
  for (int k = 0; k < 2; ++k) {
    const int n = k ? nq : np;
    const float* src = k ? q_mean : pt;
    const size_t* S = k ? L.set_q : L.set_p;
    uint32_t* ca = reinterpret_cast<uint32_t*>(w + L.code_a);
    uint32_t* ia = reinterpret_cast<uint32_t*>(w + L.idx_a);
    uint32_t* cb = reinterpret_cast<uint32_t*>(w + L.code_b);
    uint32_t* ib = reinterpret_cast<uint32_t*>(w + L.idx_b);
    hipLaunchKernelGGL(k_ov_codes, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, src, n, (const float*)box, ca,
                       ia);
    const int which = launch_radix_sort_pairs(ca, ia, cb, ib, n, 30, reinterpret_cast<uint32_t*>(w + L.hist),
                                              reinterpret_cast<uint32_t*>(w + L.digits), s);
    const uint32_t* code = which ? cb : ca;
    const uint32_t* order = which ? ib : ia;
    const int nleaf = (n + kOvLeaf - 1) / kOvLeaf, nsuper = (nleaf + kOvSuper - 1) / kOvSuper;
    float* sp = reinterpret_cast<float*>(w + S[0]);
    int32_t* sidx = reinterpret_cast<int32_t*>(w + S[1]);
    uint32_t* scode = reinterpret_cast<uint32_t*>(w + S[2]);
    float* leaf = reinterpret_cast<float*>(w + S[3]);
    float* sup = reinterpret_cast<float*>(w + S[4]);
    hipLaunchKernelGGL(k_ov_gather, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, src, n, order, code, sp,
                       sidx, scode, leaf);
    hipLaunchKernelGGL(k_ov_super, dim3((nsuper + kBlock - 1) / kBlock), dim3(kBlock), 0, s, (const float*)leaf,
                       nleaf, sup, nsuper);
    set[k] = OvSet{sp, sidx, scode, leaf, sup, n, nleaf, nsuper};
  }
  const int waves_per_block = kBlock / kOvLeaf;
  hipLaunchKernelGGL(k_ov_nn, dim3((set[0].nleaf + waves_per_block - 1) / waves_per_block), dim3(kBlock), 0, s,
                     set[0], set[1], nn_pq);
  hipLaunchKernelGGL(k_ov_nn, dim3((set[1].nleaf + waves_per_block - 1) / waves_per_block), dim3(kBlock), 0, s,
                     set[1], set[0], nn_qp);
  const float tau2 = tau * tau;
  hipLaunchKernelGGL(k_ov_count, dim3((np + kBlock - 1) / kBlock), dim3(kBlock), 0, s, (const float*)pt, np, q_mean,
                     nq, (const int32_t*)nn_pq, (const int32_t*)nn_qp, tau2, counts);
}

}  // namespace ls

// ---------------------------------------------------------------------------
// Overlap ratio without allocation: the workspace is a file-scope device
// array, one copy per GPU, held until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in
// symbol): its device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and kept in a per-device
// table.  Every call on a device shares its copy; the kernels write every
// byte they read from it within the call, so nothing needs clearing, and
// calls that overlap on one device race.
namespace {

constexpr size_t kNoAllocBytes = (size_t)LS_OVERLAP_NOALLOC_BYTES;
static_assert(kNoAllocBytes % 256 == 0, "scratch size must keep 256-byte alignment");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_dev;  // device address of `scratch`, by device ordinal

ls_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return ls::api_fail(LS_ERR_HIP, "hipGetDevice failed");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((size_t)dev >= g_scratch_dev.size()) g_scratch_dev.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_dev[(size_t)dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return ls::api_fail(LS_ERR_HIP, "hipGetSymbolAddress of the overlap scratch array failed");
    }
    g_scratch_dev[(size_t)dev] = ptr;
  }
  *out = g_scratch_dev[(size_t)dev];
  return LS_OK;
}

}  // namespace

extern "C" ls_status ls_overlap_ratio_noalloc(const float* p_mean, int32_t np, const float* q_mean, int32_t nq,
                                              const float* T_pq, float tau, int32_t* nn_pq, int32_t* nn_qp,
                                              int32_t* counts, hipStream_t s) {
  const ls_status st = ls::overlap_check_args(p_mean, np, q_mean, nq, T_pq, tau, nn_pq, nn_qp, counts);
  if (st != LS_OK) return st;
  if (np > LS_OVERLAP_NOALLOC_MAX_POINTS || nq > LS_OVERLAP_NOALLOC_MAX_POINTS)
    return ls::api_fail(LS_ERR_CAPACITY, "ls_overlap_ratio_noalloc takes at most LS_OVERLAP_NOALLOC_MAX_POINTS "
                                         "points per set; use ls_overlap_ratio with a workspace");
  if (ls::overlap_workspace_bytes(np, nq) > kNoAllocBytes)
    return ls::api_fail(LS_ERR_CAPACITY, "overlap workspace exceeds the static scratch array");
  void* work = nullptr;
  const ls_status sa = scratch_address(&work);
  if (sa != LS_OK) return sa;
  ls::launch_overlap(p_mean, np, q_mean, nq, T_pq, tau, nn_pq, nn_qp, counts, work, s);
  return ls::api_hip_check("ls_overlap_ratio_noalloc");
}

// Candidate selection of the intra-agent consensus (Sec. 3.4, "1) Selection"):
// the Gaussians of the local map within the camera's field of view and within
// a distance of its pose, as an index list in map order.
//
// A Gaussian is selected when its mean p = R mu + t in camera coordinates
// lies beyond the near plane, within max_dist of the camera centre (|p|),
// and projects onto the image widened by a pixel margin. The decisions are
// integers taken in binary64 from the binary32 inputs, in one fixed order
// with no fused operations:
//   p_k = ((R_k0 mu_0 + R_k1 mu_1) + R_k2 mu_2) + t_k,
//   d2 = (p_0 p_0 + p_1 p_1) + p_2 p_2 <= max_dist^2,
//   rz = 1 / p_z,  u = fx (p_x rz) + cx,  v = fy (p_y rz) + cy,
//   -m <= u <= W - 1 + m,  -m <= v <= H - 1 + m,  p_z > near.
//
// Three launches, an order-preserving stream compaction that reads the 12
// bytes of each mean twice and writes 4 bytes per candidate:
//   1. k_select_count: candidates per block of kSelSlots Gaussians;
//   2. the block scan shared with pruning: exclusive block offsets, total;
//   3. k_select_scatter: each block re-evaluates, ranks its candidates in
//      index order (ballots and per-wave counts) and writes their indices.
#include "ms_internal.h"

#pragma clang fp contract(off)

namespace ms {
namespace {

constexpr int kSelThreads = 256;
constexpr int kSelSub = 4;                             // slots per thread
constexpr int kSelSlots = kSelThreads * kSelSub;       // Gaussians per block

struct Pose {
  double r[12];
};

__device__ inline Pose load_pose(const float* __restrict__ vm) {
  Pose P;
#pragma unroll
  for (int k = 0; k < 12; k++) P.r[k] = (double)vm[k];
  return P;
}

__device__ inline bool is_candidate(const SelectArgs& A, const Pose& P, int64_t i) {
  const int64_t n = A.n;
  const double m0 = (double)A.means[i], m1 = (double)A.means[n + i], m2 = (double)A.means[2 * n + i];
  const double p0 = ((P.r[0] * m0 + P.r[1] * m1) + P.r[2] * m2) + P.r[3];
  const double p1 = ((P.r[4] * m0 + P.r[5] * m1) + P.r[6] * m2) + P.r[7];
  const double p2 = ((P.r[8] * m0 + P.r[9] * m1) + P.r[10] * m2) + P.r[11];
  if (!(__builtin_isfinite(p0) && __builtin_isfinite(p1) && __builtin_isfinite(p2))) return false;
  if (!(p2 > A.near)) return false;
  const double d2 = (p0 * p0 + p1 * p1) + p2 * p2;
  if (!(d2 <= A.dmax2)) return false;
  const double rz = 1.0 / p2;
  const double u = A.fx * (p0 * rz) + A.cx;
  const double v = A.fy * (p1 * rz) + A.cy;
  return u >= A.xmin && u <= A.xmax && v >= A.ymin && v <= A.ymax;
}

__global__ void __launch_bounds__(kSelThreads) k_select_count(SelectArgs A, uint32_t* __restrict__ bcount) {
  __shared__ uint32_t red[kSelThreads / 64];
  const Pose P = load_pose(A.viewmat);
  const int t = threadIdx.x;
  uint32_t c = 0;
#pragma unroll
  for (int u = 0; u < kSelSub; u++) {
    const int64_t i = (int64_t)blockIdx.x * kSelSlots + u * kSelThreads + t;
    if (i < A.n && is_candidate(A, P, i)) c++;
  }
  for (int off = 32; off > 0; off >>= 1) c += (uint32_t)__shfl_xor((int)c, off, 64);
  if ((t & 63) == 0) red[t >> 6] = c;
  __syncthreads();
  if (t == 0) {
    uint32_t s = 0;
    for (int w = 0; w < kSelThreads / 64; w++) s += red[w];
    bcount[blockIdx.x] = s;
  }
}

__global__ void __launch_bounds__(kSelThreads) k_select_scatter(SelectArgs A, const uint32_t* __restrict__ boff,
                                                                int32_t* __restrict__ idx) {
  __shared__ uint32_t wcnt[kSelSub][kSelThreads / 64];
  const Pose P = load_pose(A.viewmat);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  bool sel[kSelSub];
  uint64_t bal[kSelSub];
#pragma unroll
  for (int u = 0; u < kSelSub; u++) {
    const int64_t i = (int64_t)blockIdx.x * kSelSlots + u * kSelThreads + t;
    sel[u] = i < A.n && is_candidate(A, P, i);
    bal[u] = __ballot(sel[u]);
    if (lane == 0) wcnt[u][wave] = (uint32_t)__popcll(bal[u]);
  }
  __syncthreads();
  uint32_t run = 0;
#pragma unroll
  for (int u = 0; u < kSelSub; u++) {
    uint32_t before = run;
    for (int w = 0; w < kSelThreads / 64; w++) {
      if (w < wave) before += wcnt[u][w];
      run += wcnt[u][w];
    }
    if (!sel[u]) continue;
    const int64_t i = (int64_t)blockIdx.x * kSelSlots + u * kSelThreads + t;
    const int64_t d = (int64_t)boff[blockIdx.x] + before +
                      __builtin_amdgcn_mbcnt_hi((uint32_t)(bal[u] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal[u], 0u));
    idx[d] = (int32_t)i;
  }
}

}  // namespace

size_t select_workspace_bytes(int64_t n) {
  const int64_t blocks = n > 0 ? (n + kSelSlots - 1) / kSelSlots : 1;
  return (size_t)blocks * sizeof(uint32_t);
}

hipError_t launch_select(const SelectArgs& a, int32_t* idx, int64_t* count, void* ws, hipStream_t st) {
  const int64_t blocks = a.n > 0 ? (a.n + kSelSlots - 1) / kSelSlots : 0;
  uint32_t* bcount = static_cast<uint32_t*>(ws);
  if (blocks > 0) hipLaunchKernelGGL(k_select_count, dim3((unsigned)blocks), dim3(kSelThreads), 0, st, a, bcount);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_block_offsets(bcount, blocks, count, st);
  if (e != hipSuccess) return e;
  if (blocks > 0) hipLaunchKernelGGL(k_select_scatter, dim3((unsigned)blocks), dim3(kSelThreads), 0, st, a, bcount, idx);
  return hipGetLastError();
}

}  // namespace ms

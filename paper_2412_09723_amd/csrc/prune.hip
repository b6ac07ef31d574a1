// Map pruning (App. C.1, Algorithm 1): a Gaussian is removed when its
// opacity is below tau_o, or, with a scale threshold (tau_s > 0), when its
// largest scale exceeds tau_s or tau_e times the sum of its other two
// scales. The survivors are compacted in their original order into planar
// output arrays of row stride `kept`.
//
// Three launches, each streaming the map once or less:
//   1. k_prune_count: survivors per block of kPruneSlots Gaussians;
//   2. k_prune_scan (one workgroup): exclusive offsets of the blocks and the
//      total, which is also the row stride of the output;
//   3. k_prune_scatter: each block re-evaluates its flags, ranks its
//      survivors in index order (ballots and per-wave counts) and writes
//      their 14 floats.
#include "ms_internal.h"

#include <mutex>

namespace ms {
namespace {

constexpr int kPruneThreads = 256;
constexpr int kPruneSub = 4;                                  // slots per thread
constexpr int kPruneSlots = kPruneThreads * kPruneSub;        // Gaussians per block
constexpr int kPruneScanThreads = 1024;

// The removal decision in binary32: the largest scale is the first of s0,
// s1, s2 that no later one exceeds; the other two are added in index order.
__device__ inline bool prune_removed(float o, float s0, float s1, float s2, float to, float ts, float te) {
  bool r = o < to;
  if (ts > 0.f) {
    float big = s0, other = s1 + s2;
    if (s1 > big) {
      big = s1;
      other = s0 + s2;
    }
    if (s2 > big) {
      big = s2;
      other = s0 + s1;
    }
    r = r || big > ts || big > te * other;
  }
  return r;
}

struct PruneArgs {
  const float *means, *scales, *quats, *opacity, *colors;
  float *o_means, *o_scales, *o_quats, *o_opacity, *o_colors;
  int64_t n;
  float to, ts, te;
};

__device__ inline bool keep_at(const PruneArgs& A, int64_t i) {
  const int64_t n = A.n;
  return !prune_removed(A.opacity[i], A.scales[i], A.scales[n + i], A.scales[2 * n + i], A.to, A.ts, A.te);
}

__global__ void __launch_bounds__(kPruneThreads) k_prune_count(PruneArgs A, uint32_t* __restrict__ bcount) {
  __shared__ uint32_t red[kPruneThreads / 64];
  const int t = threadIdx.x;
  uint32_t c = 0;
#pragma unroll
  for (int u = 0; u < kPruneSub; u++) {
    const int64_t i = (int64_t)blockIdx.x * kPruneSlots + u * kPruneThreads + t;
    if (i < A.n && keep_at(A, i)) c++;
  }
  for (int off = 32; off > 0; off >>= 1) c += (uint32_t)__shfl_xor((int)c, off, 64);
  if ((t & 63) == 0) red[t >> 6] = c;
  __syncthreads();
  if (t == 0) {
    uint32_t s = 0;
    for (int w = 0; w < kPruneThreads / 64; w++) s += red[w];
    bcount[blockIdx.x] = s;
  }
}

// In place: bcount[b] becomes the exclusive offset of block b; *kept the total.
// (Also the middle pass of the candidate selection's compaction.)
__global__ void __launch_bounds__(kPruneScanThreads) k_prune_scan(uint32_t* __restrict__ bcount, int64_t nblocks,
                                                                  int64_t* __restrict__ kept) {
  __shared__ int64_t wsum[kPruneScanThreads / 64];
  __shared__ int64_t carry_s;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  if (t == 0) carry_s = 0;
  __syncthreads();
  for (int64_t base = 0; base < nblocks; base += kPruneScanThreads) {
    const int64_t j = base + t;
    const int64_t v = j < nblocks ? (int64_t)bcount[j] : 0;
    int64_t inc = v;
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t y = __shfl_up(inc, off, 64);
      if (lane >= off) inc += y;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    int64_t before = carry_s;
    int64_t chunk = 0;
    for (int w = 0; w < kPruneScanThreads / 64; w++) {
      if (w < wave) before += wsum[w];
      chunk += wsum[w];
    }
    if (j < nblocks) bcount[j] = (uint32_t)(before + inc - v);
    __syncthreads();
    if (t == 0) carry_s += chunk;
    __syncthreads();
  }
  if (t == 0) *kept = carry_s;
}

__global__ void __launch_bounds__(kPruneThreads) k_prune_scatter(PruneArgs A, const uint32_t* __restrict__ boff,
                                                                 const int64_t* __restrict__ kept) {
  __shared__ uint32_t wcnt[kPruneSub][kPruneThreads / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t n = A.n;
  bool keep[kPruneSub];
  uint64_t bal[kPruneSub];
#pragma unroll
  for (int u = 0; u < kPruneSub; u++) {
    const int64_t i = (int64_t)blockIdx.x * kPruneSlots + u * kPruneThreads + t;
    keep[u] = i < n && keep_at(A, i);
    bal[u] = __ballot(keep[u]);
    if (lane == 0) wcnt[u][wave] = (uint32_t)__popcll(bal[u]);
  }
  __syncthreads();
  const int64_t m = *kept;   // row stride of the output
  uint32_t run = 0;
#pragma unroll
  for (int u = 0; u < kPruneSub; u++) {
    uint32_t before = run;
    for (int w = 0; w < kPruneThreads / 64; w++) {
      if (w < wave) before += wcnt[u][w];
      run += wcnt[u][w];
    }
    if (!keep[u]) continue;
    const int64_t i = (int64_t)blockIdx.x * kPruneSlots + u * kPruneThreads + t;
    const int64_t d = (int64_t)boff[blockIdx.x] + before +
                      __builtin_amdgcn_mbcnt_hi((uint32_t)(bal[u] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal[u], 0u));
#pragma unroll
    for (int k = 0; k < 3; k++) {
      A.o_means[k * m + d] = A.means[k * n + i];
      A.o_scales[k * m + d] = A.scales[k * n + i];
      A.o_colors[k * m + d] = A.colors[k * n + i];
    }
#pragma unroll
    for (int k = 0; k < 4; k++) A.o_quats[k * m + d] = A.quats[k * n + i];
    A.o_opacity[d] = A.opacity[i];
  }
}

}  // namespace

// Scratch of the allocation-free entry point (ms_prune_noalloc): one survivor
// count per block of kPruneSlots Gaussians, for maps of up to
// kPruneNoAllocMaxN Gaussians (256 KB). Every GPU the library runs on holds
// its own copy until the process ends. In host code `scratch` names a host
// stand-in, not the device copy: its device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
constexpr int64_t kPruneNoAllocBlocks = kPruneNoAllocMaxN / kPruneSlots;
static_assert(kPruneNoAllocMaxN % kPruneSlots == 0, "whole blocks");
static __device__ __align__(256) uint32_t scratch[kPruneNoAllocBlocks];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[kMaxDevices];   // device address of `scratch` per device, once looked up
}  // namespace

// The device address of `scratch` on the current device (looked up on the
// first call on that device, with it current).
hipError_t prune_scratch(uint32_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<uint32_t*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_block_offsets(uint32_t* bcount, int64_t nblocks, int64_t* total, hipStream_t st) {
  hipLaunchKernelGGL(k_prune_scan, dim3(1), dim3(kPruneScanThreads), 0, st, bcount, nblocks, total);
  return hipGetLastError();
}

size_t prune_workspace_bytes(int64_t n) {
  const int64_t blocks = n > 0 ? (n + kPruneSlots - 1) / kPruneSlots : 1;
  return (size_t)blocks * sizeof(uint32_t);
}

hipError_t launch_prune(const ms_map& in, const ms_map& out, float tau_o, float tau_s, float tau_e, int64_t* kept,
                        void* ws, hipStream_t st) {
  PruneArgs A;
  A.means = in.means;
  A.scales = in.scales;
  A.quats = in.quats;
  A.opacity = in.opacity;
  A.colors = in.colors;
  A.o_means = const_cast<float*>(out.means);
  A.o_scales = const_cast<float*>(out.scales);
  A.o_quats = const_cast<float*>(out.quats);
  A.o_opacity = const_cast<float*>(out.opacity);
  A.o_colors = const_cast<float*>(out.colors);
  A.n = in.n;
  A.to = tau_o;
  A.ts = tau_s;
  A.te = tau_e;
  const int64_t blocks = in.n > 0 ? (in.n + kPruneSlots - 1) / kPruneSlots : 0;
  uint32_t* bcount = static_cast<uint32_t*>(ws);
  if (blocks > 0) hipLaunchKernelGGL(k_prune_count, dim3((unsigned)blocks), dim3(kPruneThreads), 0, st, A, bcount);
  hipLaunchKernelGGL(k_prune_scan, dim3(1), dim3(kPruneScanThreads), 0, st, bcount, blocks, kept);
  if (blocks > 0) hipLaunchKernelGGL(k_prune_scatter, dim3((unsigned)blocks), dim3(kPruneThreads), 0, st, A, bcount, kept);
  return hipGetLastError();
}

}  // namespace ms

// Tile binning: from per-Gaussian projection outputs to per-tile lists of
// depth ranks, ordered by (depth key, Gaussian index) within every tile.
//
//   1. compaction of the visible Gaussians (exclusive scan of the 0/1 flags);
//   2. stable LSD radix sort of the N_v binary32 depth keys (values = index),
//      which yields each Gaussian's depth rank with index tie-break;
//   3. gather of the records into rank order, scan of the per-rank tile
//      counts (the (Gaussian, tile) pair offsets) and the capacity check;
//   4. emission of (tile, rank) pairs in rank-major order;
//   5. stable LSD radix sort of the pairs by tile id only: since the pairs
//      were emitted in rank order, each tile's run comes out in rank order,
//      so the K pairs need ceil(log2(tiles)/8) passes instead of sorting
//      64-bit (tile, depth) keys;
//   6. tile ranges from the run boundaries.
// All counts stay on the device; grids are sized by capacities and every
// block reads the live count, so the sequence needs no host round trip.
#include <utility>

#include "ms_internal.h"

namespace ms {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;   // 2048 items per block
constexpr int kSortThreads = 256;

// Inclusive block-wide sum scan of one value per thread (256 threads).
template <typename T>
__device__ inline T block_inclusive_scan(T v, T* sh, T& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 1; off < 64; off <<= 1) {
    T y = __shfl_up(v, off, 64);
    if (lane >= off) v += y;
  }
  if (lane == 63) sh[wave] = v;
  __syncthreads();
  T carry = 0;
  total = 0;
  for (int w = 0; w < kScanThreads / 64; w++) {
    T s = sh[w];
    if (w < wave) carry += s;
    total += s;
  }
  __syncthreads();
  return v + carry;
}

__device__ inline int64_t live_count(const uint64_t* counters, int which, int64_t fallback) {
  return which < 0 ? fallback : (int64_t)counters[which];
}

// Per-block sums of in[0..count).
template <typename TOut>
__global__ void __launch_bounds__(kScanThreads) k_scan_partials(const uint32_t* __restrict__ in, int64_t n_static,
                                                                const uint64_t* __restrict__ counters,
                                                                int which, TOut* __restrict__ partials) {
  __shared__ TOut sh[kScanThreads / 64];
  const int64_t count = live_count(counters, which, n_static);
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  TOut s = 0;
  for (int k = 0; k < kScanItems; k++) {
    const int64_t j = base + (int64_t)k * kScanThreads + threadIdx.x;
    if (j < count) s += (TOut)in[j];
  }
  TOut total;
  block_inclusive_scan<TOut>(s, sh, total);
  if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

// Exclusive scan of the block partials (one block); the grand total goes to
// counters[total_slot]. For the pair offsets, also checks the capacity.
template <typename TOut>
__global__ void __launch_bounds__(kScanThreads) k_scan_top(TOut* __restrict__ partials, int nblocks,
                                                           uint64_t* __restrict__ counters, int total_slot,
                                                           int64_t capacity) {
  __shared__ TOut sh[kScanThreads / 64];
  TOut carry = 0;
  for (int base = 0; base < nblocks; base += kScanThreads) {
    const int j = base + threadIdx.x;
    TOut v = j < nblocks ? partials[j] : 0;
    TOut total;
    TOut inc = block_inclusive_scan<TOut>(v, sh, total);
    if (j < nblocks) partials[j] = carry + inc - v;
    carry += total;
  }
  if (threadIdx.x == 0) {
    counters[total_slot] = (uint64_t)carry;
    if (capacity >= 0) counters[C_OVERFLOW] = ((int64_t)carry > capacity) ? 1ull : 0ull;
  }
}

// Block-local exclusive scan plus the block offset. Mode 0: write the scan to
// out. Mode 1 (compaction): for in[j] != 0 write ckey[pos] = key[j],
// cval[pos] = j.
template <typename TOut, int MODE>
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const uint32_t* __restrict__ in, int64_t n_static,
                                                             const uint64_t* __restrict__ counters, int which,
                                                             const TOut* __restrict__ partials,
                                                             TOut* __restrict__ out,
                                                             const uint32_t* __restrict__ key,
                                                             uint32_t* __restrict__ ckey,
                                                             uint32_t* __restrict__ cval) {
  __shared__ TOut sh[kScanThreads / 64];
  const int64_t count = live_count(counters, which, n_static);
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  if (base >= count) return;
  // each thread owns kScanItems consecutive items
  const int64_t j0 = base + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  TOut s = 0;
  for (int k = 0; k < kScanItems; k++) {
    const int64_t j = j0 + k;
    v[k] = j < count ? in[j] : 0u;
    s += (TOut)v[k];
  }
  TOut total;
  TOut inc = block_inclusive_scan<TOut>(s, sh, total);
  TOut run = partials[blockIdx.x] + inc - s;
  for (int k = 0; k < kScanItems; k++) {
    const int64_t j = j0 + k;
    if (j < count) {
      if (MODE == 0) {
        out[j] = run;
      } else if (v[k]) {
        ckey[run] = key[j];
        cval[run] = (uint32_t)j;
      }
    }
    run += (TOut)v[k];
  }
}

// ------------------------------------------------------------- radix sort
// Live element count of a sort; a count above the buffer capacity (pair
// overflow) sorts nothing, so no kernel ever indexes past the buffers.
__device__ inline int64_t sort_count(const uint64_t* counters, int which, int64_t limit) {
  const int64_t c = (int64_t)counters[which];
  return c > limit ? 0 : c;
}

// Per-block digit histogram of keys[0..count), digit = (key >> shift) & mask.
__global__ void __launch_bounds__(kSortThreads) k_radix_hist(const uint32_t* __restrict__ keys,
                                                             const uint64_t* __restrict__ counters, int which,
                                                             int64_t limit, int shift, int bits, int nblocks,
                                                             uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  const int64_t count = sort_count(counters, which, limit);
  const int bins = 1 << bits;
  const uint32_t mask = (uint32_t)bins - 1u;
  for (int d = threadIdx.x; d < bins; d += blockDim.x) h[d] = 0u;
  __syncthreads();
  const int64_t per = (count + nblocks - 1) / nblocks;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < count ? lo + per : count;
  for (int64_t j = lo + threadIdx.x; j < hi; j += blockDim.x) atomicAdd(&h[(keys[j] >> shift) & mask], 1u);
  __syncthreads();
  for (int d = threadIdx.x; d < bins; d += blockDim.x) hist[(int64_t)d * nblocks + blockIdx.x] = h[d];
}

// Exclusive scan over hist laid out [digit][block] (one block, 1024 threads).
__global__ void __launch_bounds__(1024) k_radix_scan(uint32_t* __restrict__ hist, int total_entries) {
  __shared__ uint32_t sh[1024 / 64];
  __shared__ uint32_t carry_sh;
  if (threadIdx.x == 0) carry_sh = 0u;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int base = 0; base < total_entries; base += 1024) {
    const int j = base + threadIdx.x;
    uint32_t v = j < total_entries ? hist[j] : 0u;
    uint32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
      uint32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    uint32_t pre = 0u, tot = 0u;
    for (int w = 0; w < 1024 / 64; w++) {
      if (w < wave) pre += sh[w];
      tot += sh[w];
    }
    const uint32_t carry = carry_sh;
    if (j < total_entries) hist[j] = carry + pre + x - v;
    __syncthreads();
    if (threadIdx.x == 0) carry_sh = carry + tot;
    __syncthreads();
  }
}

// Stable scatter. Each block walks its contiguous range in tiles of 256 keys;
// a key's destination is the block's running offset for its digit plus the
// number of equal digits before it in the tile (earlier waves, then earlier
// lanes of the same wave, found by matching the digit bits with ballots).
__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(const uint32_t* __restrict__ keys_in,
                                                                const uint32_t* __restrict__ vals_in,
                                                                uint32_t* __restrict__ keys_out,
                                                                uint32_t* __restrict__ vals_out,
                                                                const uint64_t* __restrict__ counters, int which,
                                                                int64_t limit, int shift, int bits, int nblocks,
                                                                const uint32_t* __restrict__ hist) {
  constexpr int W = kSortThreads / 64;
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[W][256];
  const int64_t count = sort_count(counters, which, limit);
  const int bins = 1 << bits;
  const uint32_t mask = (uint32_t)bins - 1u;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int d = threadIdx.x; d < bins; d += blockDim.x) base[d] = hist[(int64_t)d * nblocks + blockIdx.x];
  const int64_t per = (count + nblocks - 1) / nblocks;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < count ? lo + per : count;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int64_t t0 = lo; t0 < hi; t0 += kSortThreads) {
    for (int d = threadIdx.x; d < W * 256; d += blockDim.x) (&wcnt[0][0])[d] = 0u;
    __syncthreads();
    const int64_t j = t0 + threadIdx.x;
    const bool ok = j < hi;
    uint32_t k = 0u, v = 0u, dg = 0u;
    if (ok) {
      k = keys_in[j];
      v = vals_in[j];
      dg = (k >> shift) & mask;
    }
    uint64_t peers = __ballot(ok);
    for (int b = 0; b < bits; b++) {
      const uint64_t m = __ballot(ok && ((dg >> b) & 1u));
      peers &= ((dg >> b) & 1u) ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
    if (ok && rank == 0) wcnt[wave][dg] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (ok) {
      uint32_t pre = 0u;
      for (int w = 0; w < wave; w++) pre += wcnt[w][dg];
      const uint32_t dst = base[dg] + pre + rank;
      keys_out[dst] = k;
      vals_out[dst] = v;
    }
    __syncthreads();
    for (int d = threadIdx.x; d < bins; d += blockDim.x) {
      uint32_t s = 0u;
      for (int w = 0; w < W; w++) s += wcnt[w][d];
      base[d] += s;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ binning
// Rank-order gather: records, tile counts and the inverse permutation.
__global__ void __launch_bounds__(256) k_rank_gather(const uint32_t* __restrict__ sidx,
                                                     const uint64_t* __restrict__ counters,
                                                     const uint4* __restrict__ rec_i,
                                                     const uint32_t* __restrict__ ntiles,
                                                     uint4* __restrict__ rec, uint32_t* __restrict__ cnt,
                                                     int32_t* __restrict__ rank_of) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= (int64_t)counters[C_VISIBLE]) return;
  const uint32_t i = sidx[r];
  const uint4* s = rec_i + 4 * (int64_t)i;
  uint4* d = rec + 4 * r;
  d[0] = s[0];
  d[1] = s[1];
  d[2] = s[2];
  d[3] = s[3];
  cnt[r] = ntiles[i];
  rank_of[i] = (int32_t)r;
}

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t* __restrict__ dst, uint32_t value, int64_t count) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count; j += (int64_t)gridDim.x * blockDim.x)
    dst[j] = value;
}

// Emit (tile, rank) pairs in rank-major order at the scanned offsets.
__global__ void __launch_bounds__(256) k_emit(const uint4* __restrict__ rec, const uint64_t* __restrict__ off,
                                              uint64_t* __restrict__ counters, int tile, int tx,
                                              uint32_t* __restrict__ pkey, uint32_t* __restrict__ pval) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= (int64_t)counters[C_VISIBLE] || counters[C_OVERFLOW]) return;
  const uint4 b = rec[4 * r + 3];
  const int x0 = (int)(b.y & 0xFFFFu) / tile, x1 = (int)(b.y >> 16) / tile;
  const int y0 = (int)(b.z & 0xFFFFu) / tile, y1 = (int)(b.z >> 16) / tile;
  uint64_t o = off[r];
  for (int ty = y0; ty <= y1; ty++)
    for (int txx = x0; txx <= x1; txx++) {
      pkey[o] = (uint32_t)(ty * tx + txx);
      pval[o] = (uint32_t)r;
      o++;
    }
}

__global__ void __launch_bounds__(256) k_ranges(const uint32_t* __restrict__ pkey,
                                                const uint64_t* __restrict__ counters,
                                                uint32_t* __restrict__ trange) {
  const int64_t K = counters[C_OVERFLOW] ? 0 : (int64_t)counters[C_PAIRS];
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t t = pkey[k];
    if (k == 0 || pkey[k - 1] != t) trange[2 * (int64_t)t] = (uint32_t)k;
    if (k == K - 1 || pkey[k + 1] != t) trange[2 * (int64_t)t + 1] = (uint32_t)(k + 1);
  }
}

// Stable LSD sort of (keys, vals) over bits [0, total_bits) in passes of at
// most 8 bits, ping-ponging between buffer a and buffer b. The data start in
// a; after an even number of passes they end in a, after an odd number in b
// (the caller places the input so that the result lands where it wants it).
hipError_t radix_sort(uint32_t* ak, uint32_t* av, uint32_t* bk, uint32_t* bv, const uint64_t* counters, int which,
                      int64_t limit, int total_bits, int nblocks, uint32_t* hist, hipStream_t st) {
  const int passes = sort_passes(total_bits);
  const int bits_per = passes > 0 ? (total_bits + passes - 1) / passes : 0;
  uint32_t *ki = ak, *vi = av, *ko = bk, *vo = bv;
  for (int p = 0, shift = 0; p < passes; p++, shift += bits_per) {
    const int bits = (shift + bits_per <= total_bits) ? bits_per : total_bits - shift;
    hipLaunchKernelGGL(k_radix_hist, dim3(nblocks), dim3(kSortThreads), 0, st, ki, counters, which, limit, shift,
                       bits, nblocks, hist);
    hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(1024), 0, st, hist, (1 << bits) * nblocks);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nblocks), dim3(kSortThreads), 0, st, ki, vi, ko, vo, counters, which,
                       limit, shift, bits, nblocks, hist);
    std::swap(ki, ko);
    std::swap(vi, vo);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* dst, uint32_t value, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, dst, value, count);
  return hipGetLastError();
}

hipError_t launch_bin(const Plan& p, char* ws, hipStream_t st) {
  uint64_t* counters = at<uint64_t>(ws, p.counters);
  uint32_t* trange = at<uint32_t>(ws, p.trange);
  hipError_t e = launch_fill_u32(trange, 0u, 2 * (int64_t)p.tiles, st);
  if (e != hipSuccess) return e;
  if (p.n == 0) return hipSuccess;
  // 1. compaction of the visible Gaussians, placed so that the depth sort
  //    ends in (ckey, cval)
  const bool dodd = sort_passes(32) & 1;
  uint32_t *ck = at<uint32_t>(ws, p.ckey), *cv = at<uint32_t>(ws, p.cval);
  uint32_t *ck2 = at<uint32_t>(ws, p.ckey2), *cv2 = at<uint32_t>(ws, p.cval2);
  uint32_t* vis = at<uint32_t>(ws, p.vis_pos);
  uint64_t* part = at<uint64_t>(ws, p.scan_part);
  hipLaunchKernelGGL((k_scan_partials<uint64_t>), dim3(p.scan_blocks_n), dim3(kScanThreads), 0, st, vis, p.n,
                     counters, -1, part);
  hipLaunchKernelGGL((k_scan_top<uint64_t>), dim3(1), dim3(kScanThreads), 0, st, part, p.scan_blocks_n, counters,
                     (int)C_VISIBLE, (int64_t)-1);
  hipLaunchKernelGGL((k_scan_apply<uint64_t, 1>), dim3(p.scan_blocks_n), dim3(kScanThreads), 0, st, vis, p.n,
                     counters, -1, part, (uint64_t*)nullptr, at<uint32_t>(ws, p.key), dodd ? ck2 : ck,
                     dodd ? cv2 : cv);
  // 2. depth sort (32-bit keys, index values)
  e = dodd ? radix_sort(ck2, cv2, ck, cv, counters, C_VISIBLE, p.n, 32, p.sort_blocks_v, at<uint32_t>(ws, p.hist), st)
           : radix_sort(ck, cv, ck2, cv2, counters, C_VISIBLE, p.n, 32, p.sort_blocks_v, at<uint32_t>(ws, p.hist), st);
  if (e != hipSuccess) return e;
  // 3. gather in rank order, scan tile counts, capacity check
  uint32_t* cnt = at<uint32_t>(ws, p.cnt);
  hipLaunchKernelGGL(k_rank_gather, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, st, cv, counters,
                     at<uint4>(ws, p.rec_i), at<uint32_t>(ws, p.ntiles), at<uint4>(ws, p.rec), cnt,
                     at<int32_t>(ws, p.rank_of));
  uint64_t* off = at<uint64_t>(ws, p.cnt_off);
  hipLaunchKernelGGL((k_scan_partials<uint64_t>), dim3(p.scan_blocks_n), dim3(kScanThreads), 0, st, cnt, p.n,
                     counters, (int)C_VISIBLE, part);
  hipLaunchKernelGGL((k_scan_top<uint64_t>), dim3(1), dim3(kScanThreads), 0, st, part, p.scan_blocks_n, counters,
                     (int)C_PAIRS, p.cap);
  hipLaunchKernelGGL((k_scan_apply<uint64_t, 0>), dim3(p.scan_blocks_n), dim3(kScanThreads), 0, st, cnt, p.n,
                     counters, (int)C_VISIBLE, part, off, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                     (uint32_t*)nullptr);
  // 4. emission, placed so that the tile sort ends in (pkey, pval)
  const int tbits = tile_bits(p.tiles);
  const bool podd = sort_passes(tbits) & 1;
  uint32_t *pk = at<uint32_t>(ws, p.pkey), *pv = at<uint32_t>(ws, p.pval);
  uint32_t *pk2 = at<uint32_t>(ws, p.pkey2), *pv2 = at<uint32_t>(ws, p.pval2);
  hipLaunchKernelGGL(k_emit, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, st, at<uint4>(ws, p.rec), off,
                     counters, p.tile, p.tx, podd ? pk2 : pk, podd ? pv2 : pv);
  // 5. stable sort of the pairs by tile id
  e = podd ? radix_sort(pk2, pv2, pk, pv, counters, C_PAIRS, p.cap, tbits, p.sort_blocks_p, at<uint32_t>(ws, p.hist), st)
           : radix_sort(pk, pv, pk2, pv2, counters, C_PAIRS, p.cap, tbits, p.sort_blocks_p, at<uint32_t>(ws, p.hist), st);
  if (e != hipSuccess) return e;
  // 6. tile ranges
  hipLaunchKernelGGL(k_ranges, dim3(2048), dim3(256), 0, st, pk, counters, trange);
  return hipGetLastError();
}

}  // namespace ms

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

// Emit the (tile, rank) pairs in rank-major order. Work is balanced over
// the output: each thread writes kEmitPerThread consecutive pairs, finding
// the rank that owns its first pair by binary search over the offsets, so a
// splat covering thousands of tiles is spread over many threads. Packed mode
// writes key = tile << rank_bits | rank; otherwise separate tile and rank
// arrays.
constexpr int kEmitPerThread = 8;

// Bins are global: a record's job (found from its virtual index) supplies the
// job's first bin and bins per row.
struct EmitJobs {
  int njobs;
  int64_t g0[kMaxJobs];
  int bin0[kMaxJobs], bx[kMaxJobs];
};

__device__ inline void emit_bin_base(const EmitJobs& ej, uint32_t vidx, int& bin0, int& bx) {
  int j = 0;
  for (int k = 1; k < ej.njobs; k++)
    if ((int64_t)vidx >= ej.g0[k]) j = k;
  bin0 = ej.bin0[j];
  bx = ej.bx[j];
}

__global__ void __launch_bounds__(256) k_emit(const uint4* __restrict__ rec, const uint64_t* __restrict__ off,
                                              const uint64_t* __restrict__ counters, int64_t cap, int tile,
                                              const JobDesc* __restrict__ jobs, int njobs, int rank_bits,
                                              uint32_t* __restrict__ pkey, uint32_t* __restrict__ pval) {
  __shared__ EmitJobs ej;
  if (threadIdx.x < (unsigned)njobs) {
    ej.g0[threadIdx.x] = jobs[threadIdx.x].g0;
    ej.bin0[threadIdx.x] = jobs[threadIdx.x].bin0;
    ej.bx[threadIdx.x] = jobs[threadIdx.x].bx;
  }
  if (threadIdx.x == 0) ej.njobs = njobs;
  __syncthreads();
  const int64_t nv = (int64_t)counters[C_VISIBLE];
  const int64_t K = (int64_t)counters[C_PAIRS];
  if (K > cap || nv == 0) return;
  for (int64_t o0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kEmitPerThread; o0 < K;
       o0 += (int64_t)gridDim.x * blockDim.x * kEmitPerThread) {
    // largest r with off[r] <= o0
    int64_t lo = 0, hi = nv - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if ((int64_t)off[mid] <= o0) lo = mid;
      else hi = mid - 1;
    }
    int64_t r = lo;
    int64_t base = (int64_t)off[r];
    int64_t next = r + 1 < nv ? (int64_t)off[r + 1] : K;
    uint4 b = rec[4 * r + 3];
    int x0 = (int)(b.y & 0xFFFFu) / tile, x1 = (int)(b.y >> 16) / tile;
    int y0 = (int)(b.z & 0xFFFFu) / tile;
    int w = x1 - x0 + 1;
    int bin0, tx;
    emit_bin_base(ej, b.w, bin0, tx);
    const int64_t oend = o0 + kEmitPerThread < K ? o0 + kEmitPerThread : K;
    for (int64_t o = o0; o < oend; o++) {
      while (o >= next) {
        r++;
        base = next;
        next = r + 1 < nv ? (int64_t)off[r + 1] : K;
        b = rec[4 * r + 3];
        x0 = (int)(b.y & 0xFFFFu) / tile;
        x1 = (int)(b.y >> 16) / tile;
        y0 = (int)(b.z & 0xFFFFu) / tile;
        w = x1 - x0 + 1;
        emit_bin_base(ej, b.w, bin0, tx);
      }
      const int pos = (int)(o - base);
      const uint32_t t = (uint32_t)(bin0 + (y0 + pos / w) * tx + x0 + pos % w);
      if (pval) {
        pkey[o] = t;
        pval[o] = (uint32_t)r;
      } else {
        pkey[o] = (t << rank_bits) | (uint32_t)r;
      }
    }
  }
}

__global__ void __launch_bounds__(256) k_ranges(const uint32_t* __restrict__ pkey,
                                                const uint64_t* __restrict__ counters, int shift,
                                                uint32_t* __restrict__ trange) {
  const int64_t K = counters[C_OVERFLOW] ? 0 : (int64_t)counters[C_PAIRS];
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t t = pkey[k] >> shift;
    if (k == 0 || (pkey[k - 1] >> shift) != t) trange[2 * (int64_t)t] = (uint32_t)k;
    if (k == K - 1 || (pkey[k + 1] >> shift) != t) trange[2 * (int64_t)t + 1] = (uint32_t)(k + 1);
  }
}

// ------------------------------------------------------- onesweep radix pass
// One launch per digit pass. Blocks take tiles of kOsTile keys in ticket
// order; each ranks its keys stably per digit in LDS, publishes its per-digit
// counts, and obtains the exclusive per-digit prefix of all earlier tiles by
// decoupled look-back: the predecessors' published words are summed until one
// carries an inclusive prefix. Every block publishes its aggregate before it
// waits, and only waits on tiles whose blocks are already running (they took
// earlier tickets), so the waits end; a spin limit turns a pathological wait
// into an error counter instead of a hang. Look-back words pack
// (epoch:8 | flag:2 | value:54); the region is zeroed at every forward and
// each pass uses its own epoch, so stale words never match.
constexpr int kOsThreads = 256;
#ifndef MS_OS_ITEMS
#define MS_OS_ITEMS 8
#endif
constexpr int kOsItems = MS_OS_ITEMS;   // keys per thread of a tile (the look-back region holds tiles of >= 2048)
constexpr int kOsTile = kOsThreads * kOsItems;
constexpr uint64_t kLbAgg = 1, kLbPre = 2;
constexpr uint64_t kLbValMask = (1ull << 54) - 1;
constexpr uint32_t kSpinLimit = 1u << 22;
constexpr int kLbWindow = 16;   // predecessors read per look-back round trip

__device__ inline uint64_t lb_word(uint32_t epoch, uint64_t flag, uint64_t v) {
  return ((uint64_t)epoch << 56) | (flag << 54) | v;
}

// Global digit histograms of every pass, in one read of the keys.
__global__ void __launch_bounds__(1024) k_digit_hist(const uint32_t* __restrict__ keys,
                                                     const uint64_t* __restrict__ counters, int which,
                                                     int64_t limit, int first_bit, int bits_per, int total_bits,
                                                     int passes, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[4][256];
  const int64_t count = sort_count(counters, which, limit);
  for (int d = threadIdx.x; d < 4 * 256; d += blockDim.x) (&h[0][0])[d] = 0u;
  __syncthreads();
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count; j += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t k = keys[j];
    for (int p = 0; p < passes; p++) {
      const int done = p * bits_per;
      const int bits = done + bits_per <= total_bits ? bits_per : total_bits - done;
      atomicAdd(&h[p][(k >> (first_bit + done)) & ((1u << bits) - 1u)], 1u);
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < passes * 256; d += blockDim.x) {
    const uint32_t v = (&h[0][0])[d];
    if (v) atomicAdd(&hist[d], v);
  }
}

// Persistent grid: each block repeatedly takes the next tile ticket. Within a
// tile, wave w owns the contiguous keys [w*512, (w+1)*512) in 8 rounds of 64,
// so (wave, round, lane) is the key order; a wave ranks its keys against a
// wave-private digit counter in LDS (ballot matching of the digit bits, no
// block barrier), and the waves are combined once per tile.
__global__ void __launch_bounds__(kOsThreads) k_onesweep(const uint32_t* __restrict__ keys_in,
                                                         const uint32_t* __restrict__ vals_in,
                                                         uint32_t* __restrict__ keys_out,
                                                         uint32_t* __restrict__ vals_out,
                                                         uint64_t* __restrict__ counters, int which, int64_t limit,
                                                         int shift, int bits, const uint32_t* __restrict__ hist,
                                                         uint64_t* __restrict__ lookback,
                                                         uint32_t* __restrict__ ticket, uint32_t epoch) {
  constexpr int NW = kOsThreads / 64;
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_scan[NW];
  __shared__ uint32_t goff[256];
  __shared__ uint32_t wcnt[NW][256];
  __shared__ uint32_t base[NW][256];
  const int64_t count = sort_count(counters, which, limit);
  const int64_t ntiles = (count + kOsTile - 1) / kOsTile;
  const int t = threadIdx.x;
  const int bins = 1 << bits;
  const uint32_t mask = (uint32_t)bins - 1u;
  const int lane = t & 63, wave = t >> 6;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  {
    const uint32_t h = t < bins ? hist[t] : 0u;
    uint32_t total;
    const uint32_t inc = block_inclusive_scan<uint32_t>(h, s_scan, total);
    goff[t] = inc - h;
  }
  while (true) {
    if (t == 0) s_tile = atomicAdd(ticket, 1u);
    for (int d = t; d < NW * 256; d += kOsThreads) (&wcnt[0][0])[d] = 0u;
    __syncthreads();
    const int64_t tile = s_tile;
    if (tile >= ntiles) break;
    const int64_t j0 = tile * kOsTile + (int64_t)wave * (kOsItems * 64);
    uint32_t k[kOsItems], v[kOsItems], rnk[kOsItems];
#pragma unroll
    for (int i = 0; i < kOsItems; i++) {
      const int64_t j = j0 + (int64_t)i * 64 + lane;
      const bool ok = j < count;
      k[i] = ok ? keys_in[j] : 0u;
      v[i] = (ok && vals_in) ? vals_in[j] : 0u;
    }
    uint32_t* my = wcnt[wave];
#pragma unroll
    for (int i = 0; i < kOsItems; i++) {
      const bool ok = j0 + (int64_t)i * 64 + lane < count;
      const uint32_t dg = (k[i] >> shift) & mask;
      uint64_t peers = __ballot(ok);
      for (int b = 0; b < bits; b++) {
        const uint64_t m = __ballot(ok && ((dg >> b) & 1u));
        peers &= ((dg >> b) & 1u) ? m : ~m;
      }
      // all lanes of a digit group read the wave's running count, then the
      // group's lowest lane advances it (same wave: LDS ops stay in order)
      const uint32_t old = ok ? my[dg] : 0u;
      const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
      rnk[i] = old + below;
      __builtin_amdgcn_wave_barrier();
      if (ok && below == 0) my[dg] = old + (uint32_t)__popcll(peers);
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit: prefix over waves, tile aggregate, publish, look back
    if (t < bins) {
      uint32_t run = 0u;
      for (int w = 0; w < NW; w++) {
        base[w][t] = run;
        run += wcnt[w][t];
      }
      const uint64_t agg = run;
      uint64_t* slot = lookback + tile * 256 + t;
      uint64_t excl = 0;
      if (tile == 0) {
        __hip_atomic_store(slot, lb_word(epoch, kLbPre, agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        __hip_atomic_store(slot, lb_word(epoch, kLbAgg, agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // walk back kLbWindow predecessors per round trip: issue the loads,
        // then consume them in order until one is not yet published
        int64_t jt = tile - 1;
        uint32_t spins = 0;
        bool found = false;
        while (!found) {
          uint64_t w8[kLbWindow];
#pragma unroll
          for (int q = 0; q < kLbWindow; q++) {
            const int64_t jq = jt - q >= 0 ? jt - q : 0;
            w8[q] = __hip_atomic_load(lookback + jq * 256 + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          int used = 0;
#pragma unroll
          for (int q = 0; q < kLbWindow; q++) {
            if (found || used != q || jt - q < 0) continue;
            const uint64_t flag = (w8[q] >> 54) & 3u;
            if ((uint32_t)(w8[q] >> 56) != epoch || flag == 0) continue;   // not ready: stop here
            excl += w8[q] & kLbValMask;
            used = q + 1;
            if (flag == kLbPre || jt - q == 0) found = true;
          }
          jt -= used;
          if (!found && used == 0 && ++spins > kSpinLimit) {
            atomicAdd((unsigned long long*)&counters[C_ERROR], 1ull);
            break;
          }
        }
        __hip_atomic_store(slot, lb_word(epoch, kLbPre, excl + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      const uint32_t g = goff[t] + (uint32_t)excl;
      for (int w = 0; w < NW; w++) base[w][t] += g;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kOsItems; i++) {
      const int64_t j = j0 + (int64_t)i * 64 + lane;
      if (j < count) {
        const uint32_t dst = base[wave][(k[i] >> shift) & mask] + rnk[i];
        keys_out[dst] = k[i];
        if (vals_out) vals_out[dst] = v[i];
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ per-bin path
// Used when all jobs together have at most kFastBins bins. A unit is a block
// of kUnitThreads threads covering kUnitThreads * R consecutive virtual
// Gaussians: wave w of the unit owns the R * 64 Gaussians starting at
// unit_base + w * R * 64, in R rounds of 64.
//   1. k_unit_count: pairs per (unit, bin), their sums over groups of
//      kGroupUnits consecutive units, and visible Gaussians per unit;
//   2. k_unit_scan (one block): exclusive offsets of every (group, bin) in
//      bin-major order, the bin ranges, the pair total and the capacity
//      check (a unit adds its predecessors in the group when it emits);
//   3. k_unit_emit: every pair (depth key, Gaussian index) written into its
//      bin's segment in Gaussian-index order;
//   4. k_bin_sort (one block per bin): stable LSD sort of the segment by
//      depth key, which leaves it ordered by (depth key, index).
// No step waits on another block, and every loop is bounded by the counts.

__device__ inline void gbin_decode(uint32_t w, int& ntx, int& nty, int& bx) {
  ntx = (int)(w & 1023u) + 1;
  nty = (int)((w >> 10) & 1023u) + 1;
  bx = (int)((w >> 20) & 1023u) + 1;
}

// Inclusive sum scan over the 64 lanes of a wave with DPP row shifts and
// row broadcasts (VALU only).
__device__ inline uint32_t wave_inclusive_scan(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);   // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);   // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);   // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);   // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);   // row_bcast:15 -> rows 1, 3
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);   // row_bcast:31 -> rows 2, 3
  return x;
}

// The pairs of one round of 64 Gaussians, listed in (lane, bin) order --
// Gaussian-index order -- and handed out 64 at a time so that lanes with
// large footprints do not serialise the wave. `RoundPairs` holds the round's
// per-lane exclusive pair offsets and footprints in LDS; pair q belongs to
// the lane with the largest offset <= q (a 6-step binary search).
struct RoundPairs {
  uint32_t pre[64];    // exclusive pair offset of each lane
  uint32_t first[64];  // first bin
  uint32_t word[64];   // packed footprint (gbin word 1)
};

// Publishes the footprint g of this lane's Gaussian in the round and returns
// the round's pair count (uniform).
__device__ inline uint32_t round_setup(RoundPairs& R, uint2 g, int lane) {
  uint32_t c = 0;
  if (g.x != kNoBin) {
    int ntx, nty, bx;
    gbin_decode(g.y, ntx, nty, bx);
    c = (uint32_t)(ntx * nty);
  }
  const uint32_t incl = wave_inclusive_scan(c);
  R.pre[lane] = incl - c;
  R.first[lane] = g.x;
  R.word[lane] = g.y;
  __builtin_amdgcn_wave_barrier();
  return (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
}

// Rounds are processed in groups of up to kRoundGroup whose footprints are
// loaded together, so a wave waits for memory once per group.
constexpr int kRoundGroup = 8;

__device__ inline void load_group(const uint2* __restrict__ gbin, int64_t i0, int64_t n, int nr, int lane,
                                  uint2 (&g)[kRoundGroup]) {
#pragma unroll
  for (int u = 0; u < kRoundGroup; u++) {
    const int64_t i = i0 + (int64_t)u * 64 + lane;
    g[u] = (u < nr && i < n) ? gbin[i] : make_uint2(kNoBin, 0u);
  }
}

// Bin of pair q (< the round's total) and its owning lane: the lane with the
// largest exclusive offset <= q.
__device__ inline uint32_t round_pair(const RoundPairs& R, uint32_t q, uint32_t& src) {
  uint32_t lo = 0;   // lo + step <= 63 at every step, and pre[0] = 0 <= q
#pragma unroll
  for (uint32_t step = 32; step > 0; step >>= 1)
    if (R.pre[lo + step] <= q) lo += step;
  src = lo;
  int ntx, nty, bx;
  gbin_decode(R.word[lo], ntx, nty, bx);
  const int j = (int)(q - R.pre[lo]);
  // j / ntx in binary32: j < 2^20 and the quotient's distance to an integer
  // is at least 0.5 / ntx, far above the rounding error; one correction step
  // guards the boundary anyway
  int y = (int)(((float)j + 0.5f) * __builtin_amdgcn_rcpf((float)ntx));
  int x = j - y * ntx;
  if (x < 0) {
    y--;
    x += ntx;
  } else if (x >= ntx) {
    y++;
    x -= ntx;
  }
  return R.first[lo] + (uint32_t)(y * bx + x);
}

__global__ void __launch_bounds__(kUnitThreads) k_unit_count(const uint2* __restrict__ gbin, int64_t n, int rounds,
                                                             int nbins, uint32_t* __restrict__ ucnt,
                                                             uint32_t* __restrict__ gcnt,
                                                             uint32_t* __restrict__ uvis) {
  constexpr int NW = kUnitThreads / 64;
  __shared__ uint32_t hw[NW][kFastBins];
  __shared__ RoundPairs RP[NW];
  __shared__ uint32_t s_vis;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  for (int k = t; k < NW * kFastBins; k += kUnitThreads) (&hw[0][0])[k] = 0u;
  uint32_t* h = hw[wave];
  if (t == 0) s_vis = 0u;
  __syncthreads();
  const int64_t wbase = (int64_t)blockIdx.x * kUnitThreads * rounds + (int64_t)wave * 64 * rounds;
  RoundPairs& R = RP[wave];
  uint32_t nvis = 0;
  for (int r0 = 0; r0 < rounds; r0 += kRoundGroup) {
    if (wbase + (int64_t)r0 * 64 >= n) break;   // uniform
    uint2 g[kRoundGroup];
    load_group(gbin, wbase + (int64_t)r0 * 64, n, rounds - r0, lane, g);
#pragma unroll
    for (int u = 0; u < kRoundGroup; u++) {
      if (r0 + u >= rounds) break;   // uniform
      nvis += g[u].x != kNoBin ? 1u : 0u;
      const uint32_t total = round_setup(R, g[u], lane);
      for (uint32_t q0 = 0; q0 < total; q0 += 64) {
        const uint32_t q = q0 + (uint32_t)lane;
        if (q < total) {
          uint32_t src;
          atomicAdd(&h[round_pair(R, q, src)], 1u);
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  for (int off = 32; off > 0; off >>= 1) nvis += __shfl_xor(nvis, off, 64);
  if (lane == 0) atomicAdd(&s_vis, nvis);
  __syncthreads();
  // per-wave counts (the emission places each wave's pairs from them) and
  // the unit's total into its group
  uint32_t* rows = ucnt + (int64_t)blockIdx.x * NW * nbins;
  uint32_t* grow = gcnt + (int64_t)(blockIdx.x / kGroupUnits) * nbins;
  for (int b = t; b < nbins; b += kUnitThreads) {
    uint32_t c = 0;
    for (int w = 0; w < NW; w++) {
      const uint32_t x = hw[w][b];
      rows[(int64_t)w * nbins + b] = x;
      c += x;
    }
    if (c) atomicAdd(&grow[b], c);
  }
  if (t == 0) uvis[blockIdx.x] = s_vis;
}

// One block of 1024 threads. gcnt[g][b] (group-major) becomes the exclusive
// offset of (unit group g, bin b) in the bin-major order of all pairs.
// Thread (chunk c, bin b) owns bin b over a contiguous chunk of groups.
constexpr int kUScanThreads = 1024;

__global__ void __launch_bounds__(kUScanThreads) k_unit_scan(uint32_t* __restrict__ gcnt,
                                                             const uint32_t* __restrict__ uvis, int units, int groups,
                                                             int nbins, int64_t cap, uint64_t* __restrict__ counters,
                                                             uint32_t* __restrict__ trange) {
  __shared__ uint32_t part[kUScanThreads];    // [chunk][bin] chunk sums, then chunk prefixes
  __shared__ uint32_t s_base[kFastBins];
  __shared__ uint32_t s_wsum[kUScanThreads / 64];
  __shared__ uint64_t s_vis[kUScanThreads / 64];
  const int t = threadIdx.x;
  const int chunks = kUScanThreads / nbins;           // >= 1 as nbins <= kFastBins = kUScanThreads
  const int b = t % nbins, c = t / nbins;
  const bool active = c < chunks;
  const int per = (groups + chunks - 1) / chunks;
  const int u0 = active ? c * per : 0;
  const int u1 = active ? min(groups, u0 + per) : 0;
  uint32_t sum = 0;
  for (int ub = u0; ub < u1; ub += 16) {   // sixteen independent loads in flight
    uint32_t x[16];
#pragma unroll
    for (int q = 0; q < 16; q++) x[q] = ub + q < u1 ? gcnt[(int64_t)(ub + q) * nbins + b] : 0u;
#pragma unroll
    for (int q = 0; q < 16; q++) sum += x[q];
  }
  if (active) part[c * nbins + b] = sum;
  // visible count
  uint64_t v = 0;
  for (int u = t; u < units; u += kUScanThreads) v += uvis[u];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((t & 63) == 0) s_vis[t >> 6] = v;
  __syncthreads();
  // per bin: exclusive prefix over chunks, and the bin total
  uint32_t total = 0;
  if (t < nbins) {
    for (int k = 0; k < chunks; k++) {
      const uint32_t x = part[k * nbins + t];
      part[k * nbins + t] = total;
      total += x;
    }
  }
  // exclusive scan of the totals over bins (thread t holds bin t)
  uint32_t inc = total;
  const int lane = t & 63, wave = t >> 6;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(inc, off, 64);
    if (lane >= off) inc += y;
  }
  if (lane == 63) s_wsum[wave] = inc;
  __syncthreads();
  uint32_t carry = 0;
  uint64_t grand = 0;
  for (int w = 0; w < kUScanThreads / 64; w++) {
    if (w < wave) carry += s_wsum[w];
    grand += s_wsum[w];
  }
  if (t < nbins) {
    const uint32_t start = carry + inc - total;
    s_base[t] = start;
    trange[2 * t] = start;
    trange[2 * t + 1] = start + total;
  }
  if (t == 0) {
    uint64_t nv = 0;
    for (int w = 0; w < kUScanThreads / 64; w++) nv += s_vis[w];
    counters[C_VISIBLE] = nv;
    counters[C_PAIRS] = grand;
    counters[C_OVERFLOW] = (int64_t)grand > cap ? 1ull : 0ull;
  }
  __syncthreads();
  if (active) {
    uint32_t run = s_base[b] + part[c * nbins + b];
    for (int ub = u0; ub < u1; ub += 16) {
      uint32_t x[16];
#pragma unroll
      for (int q = 0; q < 16; q++) x[q] = ub + q < u1 ? gcnt[(int64_t)(ub + q) * nbins + b] : 0u;
#pragma unroll
      for (int q = 0; q < 16; q++) {
        if (ub + q < u1) gcnt[(int64_t)(ub + q) * nbins + b] = run;
        run += x[q];
      }
    }
  }
}

// Emission. Each wave's start in every bin follows from the group offsets
// and the per-wave counts of k_unit_count. Then the pairs of each round, taken 64 at a
// time in Gaussian-index order, are ranked within their bins: a lane matches
// its pair's bin against the other lanes' with one ballot per bin bit, and
// the lowest lane of each group advances the wave's running count of that
// bin, as in the onesweep ranking. Each bin's pairs therefore come out in
// index order.
__global__ void __launch_bounds__(kUnitThreads) k_unit_emit(const uint2* __restrict__ gbin,
                                                            const uint32_t* __restrict__ key, int64_t n, int rounds,
                                                            int nbins, int bin_bits, const uint32_t* __restrict__ ucnt,
                                                            const uint32_t* __restrict__ goff,
                                                            const uint64_t* __restrict__ counters,
                                                            uint32_t* __restrict__ pkey, uint32_t* __restrict__ pval) {
  constexpr int NW = kUnitThreads / 64;
  __shared__ uint32_t wc[NW][kFastBins];
  __shared__ RoundPairs RP[NW];
  __shared__ uint32_t lkey[NW][64];
  if (counters[C_OVERFLOW]) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t wbase = (int64_t)blockIdx.x * kUnitThreads * rounds + (int64_t)wave * 64 * rounds;
  uint32_t* my = wc[wave];
  RoundPairs& R = RP[wave];
  // each wave's start in every bin: the group's offset, the earlier units of
  // the group and the earlier waves of this unit (counts from k_unit_count)
  const int grp = (int)blockIdx.x / kGroupUnits;
  const uint32_t* grow = goff + (int64_t)grp * nbins;
  for (int b = t; b < nbins; b += kUnitThreads) {
    uint32_t run = grow[b];
    for (int u = grp * kGroupUnits; u < (int)blockIdx.x; u++)
      for (int w = 0; w < NW; w++) run += ucnt[((int64_t)u * NW + w) * nbins + b];
    for (int w = 0; w < NW; w++) {
      wc[w][b] = run;
      run += ucnt[((int64_t)blockIdx.x * NW + w) * nbins + b];
    }
  }
  __syncthreads();
  const uint32_t lt_lo = lane >= 32 ? 0xFFFFFFFFu : ((1u << lane) - 1u);
  const uint32_t lt_hi = lane <= 32 ? 0u : ((1u << (lane - 32)) - 1u);
  for (int r0 = 0; r0 < rounds; r0 += kRoundGroup) {
    if (wbase + (int64_t)r0 * 64 >= n) break;   // uniform
    uint2 g[kRoundGroup];
    uint32_t kk[kRoundGroup];
    load_group(gbin, wbase + (int64_t)r0 * 64, n, rounds - r0, lane, g);
#pragma unroll
    for (int u = 0; u < kRoundGroup; u++)
      kk[u] = g[u].x != kNoBin ? key[wbase + (int64_t)(r0 + u) * 64 + lane] : 0u;
#pragma unroll
    for (int u = 0; u < kRoundGroup; u++) {
      if (r0 + u >= rounds) break;   // uniform
      const uint32_t total = round_setup(R, g[u], lane);
      lkey[wave][lane] = kk[u];
      __builtin_amdgcn_wave_barrier();
      const uint32_t ibase = (uint32_t)(wbase + (int64_t)(r0 + u) * 64);
      for (uint32_t q0 = 0; q0 < total; q0 += 64) {
        const uint32_t q = q0 + (uint32_t)lane;
        const bool ok = q < total;
        uint32_t src = 0, B = 0;
        if (ok) B = round_pair(R, q, src);
        const uint64_t v = __ballot(ok);
        uint32_t pl = (uint32_t)v, ph = (uint32_t)(v >> 32);
        for (int bit = 0; bit < bin_bits; bit++) {
          const uint32_t mine = (uint32_t)((int32_t)(B << (31 - bit)) >> 31);
          const uint64_t m = __ballot(mine != 0u);
          pl &= ~((uint32_t)m ^ mine);
          ph &= ~((uint32_t)(m >> 32) ^ mine);
        }
        const uint32_t old = ok ? my[B] : 0u;
        const uint32_t below = (uint32_t)(__popc(pl & lt_lo) + __popc(ph & lt_hi));
        __builtin_amdgcn_wave_barrier();
        if (ok && below == 0) my[B] = old + (uint32_t)(__popc(pl) + __popc(ph));
        __builtin_amdgcn_wave_barrier();
        if (ok) {
          pkey[old + below] = lkey[wave][src];
          pval[old + below] = ibase + src;
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
}

// Per-bin stable LSD sort by depth key of the segment trange[b] (keys in
// pkey, Gaussian indices in pval), in place. Segments of at most kSortMax
// pairs stay in registers and LDS: the keys are offset by the segment's
// minimum, and the bits that remain are sorted in as few passes of at most
// 9-bit digits as cover them (3 passes for a depth range below 2^27 key
// units). Longer segments are sorted chunk by chunk through (tkey, tval) in
// global memory, 4 passes of 8 bits. Item order within a chunk: wave w holds
// positions [w*ipt*64, (w+1)*ipt*64) in rounds of 64, so (wave, round, lane)
// is the segment order and a wave ranks its items against its own digit
// counters (peer masks, no block barrier).
constexpr int kSortThreads = 1024;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kSortItems = 16;
constexpr int kSortMax = kSortThreads * kSortItems;
constexpr int kSortDigits = 512;

struct alignas(16) SortShared {
  uint32_t buf[kSortMax];   // scatter/gather buffer; while ranking, the waves' peer masks
  uint32_t wcnt[kSortWaves][kSortDigits];
  uint32_t doff[kSortDigits];
  uint32_t wsum[kSortDigits / 64];
  uint32_t red[2][kSortWaves];
};

// Ranks the valid items of one chunk within each wave by the digit
// (k >> shift) & (2^dbits - 1); afterwards S.wcnt[w][d] holds wave w's count
// of digit d. A lane's peers (the lanes of its round with the same digit)
// come from a 64-bit mask per digit in LDS: every lane ORs its own bit into
// its digit's mask, reads the mask back, and the lowest peer clears it. The
// OR is order-independent, and a wave's LDS operations complete in program
// order, so the masks are exact. They live in S.buf, which is free while
// the waves rank.
static_assert(sizeof(uint32_t) * kSortMax >= sizeof(uint64_t) * kSortWaves * kSortDigits,
              "peer masks must fit the scatter buffer");
__device__ inline void sort_rank(SortShared& S, const uint32_t (&k)[kSortItems], uint32_t (&rk)[kSortItems],
                                 int ipt, int chunk_n, int shift, int dbits) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const uint64_t bit = 1ull << lane, below_me = bit - 1ull;
  const uint32_t dmask = (1u << dbits) - 1u;
  uint32_t* my = S.wcnt[wave];
  uint64_t* peers = reinterpret_cast<uint64_t*>(S.buf) + wave * kSortDigits;
  for (int d = lane; d < (1 << dbits); d += 64) {
    my[d] = 0u;
    peers[d] = 0ull;
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int r = 0; r < kSortItems; r++) {
    if (r < ipt) {   // uniform
      const int pos = wave * ipt * 64 + r * 64 + lane;
      const bool ok = pos < chunk_n;
      const uint32_t dg = (k[r] >> shift) & dmask;
      if (ok) atomicOr(&peers[dg], bit);
      __builtin_amdgcn_wave_barrier();
      const uint64_t pm = ok ? peers[dg] : 0ull;
      const uint32_t old = ok ? my[dg] : 0u;
      const uint32_t below = (uint32_t)__popcll(pm & below_me);
      rk[r] = old + below;
      __builtin_amdgcn_wave_barrier();
      if (ok && below == 0) {
        my[dg] = old + (uint32_t)__popcll(pm);
        peers[dg] = 0ull;
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
}

// Thread t < 2^dbits (digit d = t): per-wave starts of digit d from `run0`;
// returns the digit's total count.
__device__ inline uint32_t sort_wave_starts(SortShared& S, int t, uint32_t run0) {
  uint32_t run = run0;
  for (int w = 0; w < kSortWaves; w++) {
    const uint32_t x = S.wcnt[w][t];
    S.wcnt[w][t] = run;
    run += x;
  }
  return run - run0;
}

// Exclusive scan of `v` over threads 0 .. kSortDigits-1 (the digits); all
// threads must call it (it contains a block barrier).
__device__ inline uint32_t digit_exclusive_scan(SortShared& S, uint32_t v) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const uint32_t inc = wave_inclusive_scan(v);
  if (t < kSortDigits && lane == 63) S.wsum[wave] = inc;
  __syncthreads();
  uint32_t carry = 0;
  if (t < kSortDigits)
    for (int w = 0; w < wave; w++) carry += S.wsum[w];
  return carry + inc - v;
}

__global__ void __launch_bounds__(kSortThreads) k_bin_sort(uint32_t* __restrict__ pkey, uint32_t* __restrict__ pval,
                                                           uint32_t* __restrict__ tkey, uint32_t* __restrict__ tval,
                                                           const uint32_t* __restrict__ trange,
                                                           const uint64_t* __restrict__ counters) {
  __shared__ SortShared S;
  if (counters[C_OVERFLOW]) return;
  const uint32_t start = trange[2 * blockIdx.x], end = trange[2 * blockIdx.x + 1];
  const int seg = (int)(end - start);
  if (seg <= 1) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  uint32_t k[kSortItems], v[kSortItems], rk[kSortItems];
  if (seg <= kSortMax) {
    const int ipt = (seg + kSortThreads - 1) / kSortThreads;
    uint32_t kmin = 0xFFFFFFFFu, kmax = 0u;
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
      const int pos = wave * ipt * 64 + r * 64 + lane;
      const bool ok = r < ipt && pos < seg;
      k[r] = ok ? pkey[start + pos] : 0u;
      v[r] = ok ? pval[start + pos] : 0u;
      if (ok) {
        kmin = min(kmin, k[r]);
        kmax = max(kmax, k[r]);
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, off, 64));
      kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, off, 64));
    }
    if (lane == 0) {
      S.red[0][wave] = kmin;
      S.red[1][wave] = kmax;
    }
    __syncthreads();
    kmin = 0xFFFFFFFFu;
    kmax = 0u;
    for (int w = 0; w < kSortWaves; w++) {
      kmin = min(kmin, S.red[0][w]);
      kmax = max(kmax, S.red[1][w]);
    }
    const uint32_t range = kmax - kmin;
    const int bits = range == 0u ? 0 : 32 - __clz((int)range);
    const int passes = bits <= 27 ? (bits + 8) / 9 : 4;
    const int width = passes > 0 ? (bits + passes - 1) / passes : 0;
#pragma unroll
    for (int r = 0; r < kSortItems; r++) k[r] -= kmin;
    for (int q = 0; q < passes; q++) {
      const int shift = q * width;
      const int dbits = min(width, bits - shift);
      const int nd = 1 << dbits;
      sort_rank(S, k, rk, ipt, seg, shift, dbits);
      __syncthreads();
      // digit t: the waves' counts stay in registers between the scan and
      // the write of the waves' starts
      uint32_t wc[kSortWaves];
      uint32_t total = 0;
#pragma unroll
      for (int w = 0; w < kSortWaves; w++) {
        wc[w] = t < nd ? S.wcnt[w][t] : 0u;
        total += wc[w];
      }
      uint32_t run = digit_exclusive_scan(S, total);
      if (t < nd) {
#pragma unroll
        for (int w = 0; w < kSortWaves; w++) {
          S.wcnt[w][t] = run;
          run += wc[w];
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kSortItems; r++) {
        const int pos = wave * ipt * 64 + r * 64 + lane;
        if (r < ipt && pos < seg) rk[r] += S.wcnt[wave][(k[r] >> shift) & (uint32_t)(nd - 1)];
      }
      if (q + 1 < passes) {   // the last pass moves only the values
#pragma unroll
        for (int r = 0; r < kSortItems; r++) {
          const int pos = wave * ipt * 64 + r * 64 + lane;
          if (r < ipt && pos < seg) S.buf[rk[r]] = k[r];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSortItems; r++) {
          const int pos = wave * ipt * 64 + r * 64 + lane;
          if (r < ipt && pos < seg) k[r] = S.buf[pos];
        }
        __syncthreads();
      }
#pragma unroll
      for (int r = 0; r < kSortItems; r++) {
        const int pos = wave * ipt * 64 + r * 64 + lane;
        if (r < ipt && pos < seg) S.buf[rk[r]] = v[r];
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kSortItems; r++) {
        const int pos = wave * ipt * 64 + r * 64 + lane;
        if (r < ipt && pos < seg) v[r] = S.buf[pos];
      }
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
      const int pos = wave * ipt * 64 + r * 64 + lane;
      if (r < ipt && pos < seg) pval[start + pos] = v[r];
    }
    return;
  }
  // long segment: four passes of 8 bits through global memory, chunk by chunk
  uint32_t *sk = pkey, *sv = pval, *dk = tkey, *dv = tval;
  for (int shift = 0; shift < 32; shift += 8) {
    if (t < 256) S.doff[t] = 0u;
    __syncthreads();
    for (int pos = t; pos < seg; pos += kSortThreads) atomicAdd(&S.doff[(sk[start + pos] >> shift) & 255u], 1u);
    __syncthreads();
    const uint32_t h = t < 256 ? S.doff[t] : 0u;
    const uint32_t excl = digit_exclusive_scan(S, h);
    if (t < 256) S.doff[t] = excl;      // running start of every digit
    __syncthreads();
    for (int c0 = 0; c0 < seg; c0 += kSortMax) {
      const int cn = min(kSortMax, seg - c0);
      const int ipt = (cn + kSortThreads - 1) / kSortThreads;
#pragma unroll
      for (int r = 0; r < kSortItems; r++) {
        const int pos = wave * ipt * 64 + r * 64 + lane;
        k[r] = (r < ipt && pos < cn) ? sk[start + c0 + pos] : 0u;
        v[r] = (r < ipt && pos < cn) ? sv[start + c0 + pos] : 0u;
      }
      sort_rank(S, k, rk, ipt, cn, shift, 8);
      __syncthreads();
      if (t < 256) S.doff[t] += sort_wave_starts(S, t, S.doff[t]);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kSortItems; r++) {
        const int pos = wave * ipt * 64 + r * 64 + lane;
        if (r < ipt && pos < cn) {
          const uint32_t dst = S.wcnt[wave][(k[r] >> shift) & 255u] + rk[r];
          dk[start + dst] = k[r];
          dv[start + dst] = v[r];
        }
      }
      __syncthreads();
    }
    uint32_t* tmp = sk;
    sk = dk;
    dk = tmp;
    tmp = sv;
    sv = dv;
    dv = tmp;
  }
}

// Stable LSD sort of (keys, vals) over bits [0, total_bits) in passes of at
// most 8 bits, ping-ponging between buffer a and buffer b. The data start in
// a; after an even number of passes they end in a, after an odd number in b
// (the caller places the input so that the result lands where it wants it).
hipError_t radix_sort(uint32_t* ak, uint32_t* av, uint32_t* bk, uint32_t* bv, uint64_t* counters, int which,
                      int64_t limit, int first_bit, int total_bits, const Plan& p, char* ws, int slot,
                      hipStream_t st) {
  const int passes = sort_passes(total_bits);
  if (passes == 0) return hipSuccess;
  const int bits_per = (total_bits + passes - 1) / passes;
  uint32_t* hist = at<uint32_t>(ws, p.digit_hist) + (size_t)slot * 4 * 256;
  uint32_t* tickets = at<uint32_t>(ws, p.tickets) + (size_t)slot * 4;
  int64_t hblocks = (limit + 1024 * 16 - 1) / (1024 * 16);
  if (hblocks > 128) hblocks = 128;
  if (hblocks < 1) hblocks = 1;
  hipLaunchKernelGGL(k_digit_hist, dim3((unsigned)hblocks), dim3(1024), 0, st, ak, counters, which, limit, first_bit,
                     bits_per, total_bits, passes, hist);
  int64_t tiles = (limit + kOsTile - 1) / kOsTile;
  if (tiles > 2048) tiles = 2048;   // persistent blocks; tiles are taken by ticket
  uint32_t *ki = ak, *vi = av, *ko = bk, *vo = bv;
  for (int q = 0, done = 0; q < passes; q++, done += bits_per) {
    const int bits = (done + bits_per <= total_bits) ? bits_per : total_bits - done;
    hipLaunchKernelGGL(k_onesweep, dim3((unsigned)(tiles > 0 ? tiles : 1)), dim3(kOsThreads), 0, st, ki, vi, ko, vo,
                       counters, which, limit, first_bit + done, bits, hist + (size_t)q * 256,
                       at<uint64_t>(ws, p.lookback), tickets + q, (uint32_t)(slot * 4 + q + 1));
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
  uint32_t* trange = at<uint32_t>(ws, p.trange);   // zeroed with the control region
  hipError_t e = hipSuccess;
  if (p.n == 0) return hipSuccess;
  if (p.by_index) {
    uint2* gbin = at<uint2>(ws, p.gbin);
    uint32_t* ucnt = at<uint32_t>(ws, p.ucnt);
    uint32_t *pk = at<uint32_t>(ws, p.pkey), *pv = at<uint32_t>(ws, p.pval);
    uint32_t* gcnt = at<uint32_t>(ws, p.gcnt);   // zeroed with the control region
    {
      StageScope tm(MS_STAGE_BIN_COUNT, st);
      hipLaunchKernelGGL(k_unit_count, dim3((unsigned)p.units), dim3(kUnitThreads), 0, st, gbin, p.n, p.unit_rounds,
                         p.bins, ucnt, gcnt, at<uint32_t>(ws, p.uvis));
      hipLaunchKernelGGL(k_unit_scan, dim3(1), dim3(kUScanThreads), 0, st, gcnt, at<uint32_t>(ws, p.uvis), p.units,
                         p.groups, p.bins, p.cap, counters, trange);
    }
    {
      StageScope tm(MS_STAGE_BIN_EMIT, st);
      hipLaunchKernelGGL(k_unit_emit, dim3((unsigned)p.units), dim3(kUnitThreads), 0, st, gbin,
                         at<uint32_t>(ws, p.key), p.n, p.unit_rounds, p.bins, tile_bits(p.bins), ucnt, gcnt, counters,
                         pk, pv);
    }
    {
      StageScope tm(MS_STAGE_BIN_SORT, st);
      hipLaunchKernelGGL(k_bin_sort, dim3((unsigned)p.bins), dim3(kSortThreads), 0, st, pk, pv,
                         at<uint32_t>(ws, p.pkey2), at<uint32_t>(ws, p.pval2), trange, counters);
    }
    return hipGetLastError();
  }
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
  e = dodd ? radix_sort(ck2, cv2, ck, cv, counters, C_VISIBLE, p.n, 0, 32, p, ws, 0, st)
           : radix_sort(ck, cv, ck2, cv2, counters, C_VISIBLE, p.n, 0, 32, p, ws, 0, st);
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
  const int tbits = tile_bits(p.bins);
  const bool podd = sort_passes(tbits) & 1;
  uint32_t *pk = at<uint32_t>(ws, p.pkey), *pv = p.packed ? nullptr : at<uint32_t>(ws, p.pval);
  uint32_t *pk2 = at<uint32_t>(ws, p.pkey2), *pv2 = p.packed ? nullptr : at<uint32_t>(ws, p.pval2);
  int64_t emit_blocks = (p.cap + 256 * 8 - 1) / (256 * 8);
  if (emit_blocks > 4096) emit_blocks = 4096;
  if (emit_blocks < 1) emit_blocks = 1;
  hipLaunchKernelGGL(k_emit, dim3((unsigned)emit_blocks), dim3(256), 0, st, at<uint4>(ws, p.rec), off, counters,
                     p.cap, p.bin, at<JobTable>(ws, p.jobs)->job, p.njobs, p.rank_bits, podd ? pk2 : pk,
                     podd ? pv2 : pv);
  // 5. stable sort of the pairs by tile id (the bits above the rank when packed)
  const int first = p.packed ? p.rank_bits : 0;
  e = podd ? radix_sort(pk2, pv2, pk, pv, counters, C_PAIRS, p.cap, first, tbits, p, ws, 1, st)
           : radix_sort(pk, pv, pk2, pv2, counters, C_PAIRS, p.cap, first, tbits, p, ws, 1, st);
  if (e != hipSuccess) return e;
  // 6. tile ranges
  hipLaunchKernelGGL(k_ranges, dim3(2048), dim3(256), 0, st, pk, counters, first, trange);
  return hipGetLastError();
}

}  // namespace ms

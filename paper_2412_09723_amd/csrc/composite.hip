// Front-to-back compositing of colour, depth and silhouette (Eq. 2 of the
// paper and its depth / accumulated-opacity analogues), and its adjoint.
//
// Work decomposition (CDNA4, wave64). A workgroup owns one screen tile of
// TILE x TILE pixels; each of its (TILE/8)^2 wavefronts owns one 8x8 pixel
// sub-block (one pixel per lane) and walks the depth-ordered list of the bin
// tile containing it on its own, with no workgroup barrier. The list is read
// in chunks of 64 entries: each lane loads one pair word and one 64-byte
// record with vector loads, tests the record's pixel box against the
// sub-block, and a ballot plus a masked bit count packs the entries that meet
// it, in list order, into the wave's private LDS slot. The per-pixel loop then
// reads those entries as LDS broadcasts. The forward evaluates four entries at
// a time (their acceptance values and alphas are independent) and applies the
// sequential transmittance updates with predication rather than branches;
// each wave stops as soon as all 64 of its pixels are done (ballot).
//
// Per pixel and Gaussian the acceptance value q follows the pinned binary32
// recipe (two fused multiply-adds), so accept/reject decisions are
// bit-identical to any conforming implementation; alpha = min(0.99,
// 2^(log2 o - q)) uses the hardware exp2.
//
// Backward: no per-(pixel, Gaussian) state is stored. From the forward's
// final transmittance and last-composited list position, each lane walks its
// list back to front, recovering T_k = T_{k+1} / (1 - alpha_k) and the
// suffix sum of (G_rgb . c + G_depth z) alpha T, forms dL/dalpha, and the
// wave reduces the 10 per-Gaussian screen-space sums before one set of
// atomics per (wave, Gaussian).
#include "ms_internal.h"

#pragma clang fp contract(off)

// v_writelane_b32 (the compiler intrinsic; HIP exposes no builtin for it):
// returns `old` with lane `lane` replaced by the wave-uniform `value`
__device__ int writelane_u(int value, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

namespace ms {
namespace {

struct Staged {
  float4 geo;    // gx = X0 - ui, gy = Y0 - vi (exact), uf, vf
  float4 conic;  // a, b, c, qcut
  float4 app;    // log2 o, z, r, g
  float4 misc;   // b(lue), rank bits, list position + 1 (bits), 0
};

// An entry that accepts no pixel, with finite fields (pads a packed chunk to
// a multiple of the evaluation group).
__device__ inline Staged inert_entry() {
  Staged s;
  s.geo = make_float4(0.f, 0.f, 0.f, 0.f);
  s.conic = make_float4(0.f, 0.f, 0.f, -INFINITY);
  s.app = make_float4(0.f, 0.f, 0.f, 0.f);
  s.misc = make_float4(0.f, 0.f, 0.f, 0.f);
  return s;
}

// Conservative test that a record's acceptance ellipse can reach a pixel of
// the 8x8 sub-block at (X0, Y0), from the record's centre words ctr = (ui,
// vi, uf, vf) and conic words con = (a, b, c, qcut). The offsets the pixels use, dx = (x - ui) - uf rounded, lie in
// [x0, x1] (rounding is monotonic), likewise dy in [y0, y1]. Over that
// rectangle |a dx + b dy| >= m1 and |c dy| >= m2 (interval bounds). A pixel
// with q <= qcut has |t1|, |t2| within a few units in the last place of
// those exact forms, so reducing m1, m2 by 2^-20 (|a| |dx|max + |b| |dy|max + 3)
// and 2^-20 |c| |dy|max, and allowing qcut (1 + 2^-20), leaves no accepted
// pixel out: a record that fails composites nowhere in the sub-block.
__device__ inline bool ellipse_reaches(const uint4& ctr, const uint4& con, int X0, int Y0) {
  constexpr float kEps = 0x1p-20f;
  const float ui = __uint_as_float(ctr.x), vi = __uint_as_float(ctr.y);
  const float uf = __uint_as_float(ctr.z), vf = __uint_as_float(ctr.w);
  const float a = __uint_as_float(con.x), b = __uint_as_float(con.y), c = __uint_as_float(con.z),
              qc = __uint_as_float(con.w);
  const float gx = (float)X0 - ui, gy = (float)Y0 - vi;   // exact
  const float x0 = gx - uf, x1 = (7.f + gx) - uf;
  const float y0 = gy - vf, y1 = (7.f + gy) - vf;
  const float ax0 = a * x0, ax1 = a * x1, by0 = b * y0, by1 = b * y1;
  const float lo1 = fminf(ax0, ax1) + fminf(by0, by1);
  const float hi1 = fmaxf(ax0, ax1) + fmaxf(by0, by1);
  const float ym = fmaxf(fabsf(y0), fabsf(y1));
  const float m1 = fmaxf(fmaxf(lo1, -hi1), 0.f);
  const float m2 = fabsf(c) * fmaxf(fmaxf(y0, -y1), 0.f);
  const float e1 = kEps * ((fabsf(a) * fmaxf(fabsf(x0), fabsf(x1)) + fabsf(b) * ym) + 3.f);
  const float e2 = kEps * (fabsf(c) * ym);
  const float r1 = fmaxf(m1 - e1, 0.f), r2 = fmaxf(m2 - e2, 0.f);
  return __builtin_fmaf(r1, r1, r2 * r2) <= qc * (1.f + kEps);
}

// The pair words of one chunk of a bin list, one per lane and 64-entry
// round: lane j of round h holds the word of list position lo + 64 h + j, 0
// past the chunk. Loaded one chunk ahead, so that staging the next chunk
// waits for its records only.
template <int WB>
struct PairWords {
  uint32_t w[(WB + 63) / 64];
};

template <int WB>
__device__ inline PairWords<WB> load_pair_words(const uint32_t* __restrict__ pval, uint32_t base, int nb, int lane) {
  PairWords<WB> pw;
#pragma unroll
  for (int h = 0; h < (WB + 63) / 64; h++) {
    const int j = 64 * h + lane;
    pw.w[h] = j < nb ? pval[base + (uint32_t)j] : 0u;
  }
  return pw;
}

// Packs the bin-list entries at list positions [lo, lo + n) (1 <= n <= 64),
// whose pair words lane j holds in `pw`, that can composite in the 8x8
// sub-block at (X0, Y0) into dst[0 ..), in list order, and returns how many
// there are (wave-uniform). Every record load is issued at once: lane j
// reads the centre and conic words of record j for the ellipse test, and a
// lane quad reads each 64-byte record with one 16-byte load per lane (each
// load instruction covers 16 whole records); lanes past n read list entry
// 0's record instead, which is never packed. A record is packed when its
// pixel box meets the sub-block and its ellipse can reach a pixel of it; a
// ballot plus a masked bit count gives each packed record its slot.
__device__ inline int stage_chunk(const uint4* __restrict__ rec, uint32_t pw, uint32_t rank_mask, uint32_t lo, int n,
                                  int X0, int Y0, int lane, Staged* __restrict__ dst) {
  const uint32_t rank = pw & rank_mask;
  const uint32_t r0 = __builtin_amdgcn_readfirstlane(rank);   // entry 0 (n >= 1): a valid record
  const uint32_t rs = lane < n ? rank : r0;
  const uint4 ctr = rec[4 * (int64_t)rs], con = rec[4 * (int64_t)rs + 1];
  const int part = lane & 3, sub = lane >> 2;
  uint4 v[4];
  uint32_t rk[4];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    rk[k] = (uint32_t)__shfl((int)rs, 16 * k + sub, 64);
    v[k] = rec[4 * (int64_t)rk[k] + part];
  }
  const bool reach = lane < n && ellipse_reaches(ctr, con, X0, Y0);
  const uint64_t rm = __builtin_amdgcn_ballot_w64(reach);
  int base = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    if (16 * k < n) {   // uniform
      const int e = 16 * k + sub;
      bool touch = false;
      // a record is packed when its box meets the sub-block and its ellipse can
      // reach a pixel centre of it
      if (part == 3 && e < n && ((rm >> e) & 1u)) {
        const int bx0 = (int)(v[k].y & 0xFFFFu), bx1 = (int)(v[k].y >> 16);
        const int by0 = (int)(v[k].z & 0xFFFFu), by1 = (int)(v[k].z >> 16);
        touch = bx0 <= X0 + 7 && bx1 >= X0 && by0 <= Y0 + 7 && by1 >= Y0;
      }
      const uint64_t m = __builtin_amdgcn_ballot_w64(touch);
      if ((m >> (4 * sub + 3)) & 1u) {
        // packed records before this one: their box lanes lie below this quad
        const int slot =
            base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        float4 o = make_float4(__uint_as_float(v[k].x), __uint_as_float(v[k].y), __uint_as_float(v[k].z),
                               __uint_as_float(v[k].w));
        if (part == 0) {
          o.x = (float)X0 - o.x;   // exact: both are integers below 2^24
          o.y = (float)Y0 - o.y;
        } else if (part == 3) {
          o = make_float4(o.x, __uint_as_float(rk[k]), __uint_as_float(lo + (uint32_t)e + 1u), 0.f);
        }
        reinterpret_cast<float4*>(dst + slot)[part] = o;
      }
      base += __builtin_popcountll(m);
    }
  }
  return base;
}

// Packs a chunk of nb <= WB entries at list positions [lo, lo + nb) (WB / 64
// rounds of stage_chunk) and pads the packed count to a multiple of `group`
// with inert entries; returns the padded count.
template <int WB>
__device__ inline int stage_chunk_padded(const uint4* __restrict__ rec, const PairWords<WB>& pw, uint32_t rank_mask,
                                         uint32_t lo, int nb, int X0, int Y0, int lane, Staged* __restrict__ dst,
                                         int group, int& packed) {
  int cnt = 0;
#pragma unroll
  for (int h = 0; h < (WB + 63) / 64; h++) {
    const int n = nb - 64 * h;
    if (n > 0)
      cnt += stage_chunk(rec, pw.w[h], rank_mask, lo + (uint32_t)(64 * h), n < 64 ? n : 64, X0, Y0, lane,
                         dst + cnt);
  }
  const int padded = (cnt + group - 1) / group * group;
  if (lane < padded - cnt) dst[cnt + lane] = inert_entry();
  packed = cnt;
  return padded;
}

// Pinned acceptance value (binary32; the fused operations are explicit).
__device__ inline float accept_q(const Staged& s, float xf, float yf, float& dx, float& dy, float& t1, float& t2) {
  dx = (xf + s.geo.x) - s.geo.z;   // (x - ui) exactly, then - uf
  dy = (yf + s.geo.y) - s.geo.w;
  t1 = __builtin_fmaf(s.conic.x, dx, s.conic.y * dy);
  t2 = s.conic.z * dy;
  return __builtin_fmaf(t1, t1, t2 * t2);
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t o = (uint32_t)__shfl_xor((int)v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

// ------------------------------------------------------------- tile queue
// Persistent compositing: the launch holds as many workgroups G as fit on
// the device at once (G <= tiles), and each takes tiles from a queue until
// it is empty. The queue is a permutation of the tiles sorted by expected
// work, longest first (k_tile_order), so that the long tiles of a batch's
// large maps start at once rather than after the short ones, and the launch
// ends on short tiles. Workgroup g starts on queue position g without a
// claim; only the positions from G on are handed out by atomic claims.
//
// With nq = 8 the positions are dealt to eight queues, one per XCD (the
// hardware sends workgroup i to XCD i mod 8), in runs of kDeal consecutive
// positions (consecutive positions are tiles of one bin, which read the
// same list); a workgroup drains its own XCD's queue first and then takes
// from the others in turn, so no single counter is hit by every workgroup.
struct TileQueue {
  const uint32_t* order;   // tile ids, longest expected work first
  uint32_t* ctr;           // nq claim counters, kQueueStride words apart (zeroed by k_tile_order)
  int n;                   // tiles
  int nq;                  // queues: 1, or 8
  int grid;                // workgroups of the launch
};
constexpr int kQueueStride = 16;   // words: one 64-byte line per counter
constexpr int kMaxQueues = 8;
constexpr int kDeal = 8;           // consecutive positions dealt to one queue

// Number of the positions below `count` that queue q holds, and the
// position of its slot s (slots in position order).
__device__ inline int queue_count(int nq, int q, int count) {
  const int run = kDeal * nq;
  const int full = count / run, rem = count - full * run;
  return full * kDeal + min(max(rem - q * kDeal, 0), kDeal);
}
__device__ inline int queue_size(const TileQueue& tq, int q) { return queue_count(tq.nq, q, tq.n); }
__device__ inline int queue_position(const TileQueue& tq, int q, int s) {
  return ((s / kDeal) * tq.nq + q) * kDeal + s % kDeal;
}
// Slots of queue q taken without a claim: its positions below G.
__device__ inline int queue_static(const TileQueue& tq, int q) { return queue_count(tq.nq, q, tq.grid); }

// Issues a claim on queue q, unless a plain read already shows it exhausted
// (then returns 0xFFFFFFFF).
__device__ inline uint32_t queue_claim(const TileQueue& tq, int q) {
  uint32_t* c = tq.ctr + kQueueStride * q;
  const uint32_t seen = __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if ((int)seen + queue_static(tq, q) >= queue_size(tq, q)) return 0xFFFFFFFFu;
  return atomicAdd(c, 1u);
}

// Position of the claim `s` on queue q, moving on to the next queue while
// the current one is exhausted; n when every queue is. `tries` counts the
// queues given up so far (the caller keeps q and tries across calls).
__device__ inline int queue_resolve(const TileQueue& tq, uint32_t s, int& q, int& tries) {
  for (;;) {
    if (tries >= tq.nq) return tq.n;
    if (s != 0xFFFFFFFFu) {
      const int slot = (int)s + queue_static(tq, q);
      if (slot < queue_size(tq, q)) return queue_position(tq, q, slot);
    }
    tries++;
    q = q + 1 == tq.nq ? 0 : q + 1;
    if (tries < tq.nq) s = queue_claim(tq, q);
  }
}

// Runs body(b) for the tiles this workgroup takes from the queue. Thread 0
// claims one tile ahead, and reads the next tile's id one tile ahead: the
// claim for the tile after next and the id of the next are in flight while
// the current tile is composited, so their latency overlaps the tile's own
// first loads. Every thread of the workgroup runs each body and the barrier
// after it.
template <class F>
__device__ inline void for_queued_tiles(const TileQueue& tq, F&& body) {
  __shared__ int next[2];
  const int g = (int)blockIdx.x;
  int q = g % tq.nq, tries = 0;   // the home queue: this workgroup's XCD
  uint32_t claim = 0xFFFFFFFFu;
  if (threadIdx.x == 0) {
    claim = queue_claim(tq, q);
    next[0] = (int)tq.order[g];   // the static first position (g < G <= n)
  }
  __syncthreads();
  for (int it = 0;; it ^= 1) {
    const int b = next[it];
    if (b < 0) break;   // uniform
    int nb = -1;
    if (threadIdx.x == 0) {
      const int i = queue_resolve(tq, claim, q, tries);
      if (i < tq.n) {
        nb = (int)tq.order[i];
        claim = queue_claim(tq, q);
      }
    }
    body(b);
    if (threadIdx.x == 0) next[it ^ 1] = nb;
    __syncthreads();
  }
}

// Expected-work class: 0 for none, else 1 + 4 floor(log2 c) plus the two
// bits below the leading one (quarter-octave classes, at most 128).
__device__ inline int cost_class(uint32_t c) {
  if (c == 0u) return 0;
  const int l = 31 - __builtin_clz(c);
  const uint32_t f = l >= 2 ? (c >> (l - 2)) & 3u : (c << (2 - l)) & 3u;
  return 1 + 4 * l + (int)f;
}

constexpr int kOrderThreads = 1024;
constexpr int kOrderPer = 4;       // bins per thread per pass
constexpr int kCostClasses = 192;  // three per lane of the scanning wave (129 used)
constexpr int kOrderLdsBins = 4096;   // bins whose backward costs are summed in LDS

// Sorts the tiles by expected work, longest first, into `order`, and zeroes
// the queue counters. The unit of the sort is the bin: its tiles read the
// same list, so they stay together, row-major, in the queue. One workgroup:
// a histogram of the bins' cost classes weighted by their tile counts, in
// LDS, an exclusive scan of it from the top class down, and a scatter in
// which each bin reserves its run of positions (the order of the bins
// within a class is arbitrary). The expected work of a bin is its list
// length for the forward (nw = 0), and for the backward the sum over its
// tiles of the per-wave list depths the forward left in wcost (nw waves per
// tile).
__global__ void __launch_bounds__(kOrderThreads)
    k_tile_order(const uint32_t* __restrict__ trange, const uint32_t* __restrict__ wcost, int nw,
                 const JobDesc* __restrict__ jobs, int njobs, int bshift, int nbins, uint32_t* __restrict__ order,
                 uint32_t* __restrict__ qctr) {
  __shared__ uint32_t hist[kCostClasses];
  __shared__ int jt[kMaxJobs][6];   // bin0, bins per row, tile0, tiles per row, tile rows
  __shared__ uint32_t bcost[kOrderLdsBins];   // backward: per-bin sums of the tiles' list depths
  const bool lds_sum = nw > 0 && nbins <= kOrderLdsBins;
  for (int i = threadIdx.x; i < kCostClasses; i += kOrderThreads) hist[i] = 0u;
  if (lds_sum)
    for (int i = threadIdx.x; i < nbins; i += kOrderThreads) bcost[i] = 0u;
  if (threadIdx.x < kMaxQueues) qctr[kQueueStride * threadIdx.x] = 0u;
  if ((int)threadIdx.x < njobs) {
    const JobDesc& J = jobs[threadIdx.x];
    jt[threadIdx.x][0] = J.bin0;
    jt[threadIdx.x][1] = J.bx;
    jt[threadIdx.x][2] = J.tile0;
    jt[threadIdx.x][3] = J.tx;
    jt[threadIdx.x][4] = J.tx > 0 ? J.tiles / J.tx : 0;
  }
  __syncthreads();
  // the bin's tiles: columns [x0, x1) and rows [y0, y1) of its job's tile
  // grid, whose first tile is t0 and which has tx tiles per row
  struct BinTiles {
    int t0, tx, x0, x1, y0, y1;
  };
  auto tiles_of = [&](int g) -> BinTiles {
    int j = 0;
    for (int k = 1; k < njobs; k++)
      if (g >= jt[k][0]) j = k;
    const int lb = g - jt[j][0];
    const int bxi = lb % jt[j][1], byi = lb / jt[j][1];
    BinTiles r;
    r.t0 = jt[j][2];
    r.tx = jt[j][3];
    r.x0 = bxi << bshift;
    r.x1 = min((bxi + 1) << bshift, jt[j][3]);
    r.y0 = byi << bshift;
    r.y1 = min((byi + 1) << bshift, jt[j][4]);
    return r;
  };
  if (lds_sum) {   // tile-parallel sums of the list depths into the bins (few bins)
    int ntiles = 0;
    for (int k = 0; k < njobs; k++) ntiles = max(ntiles, jt[k][2] + jt[k][3] * jt[k][4]);
    for (int t = threadIdx.x; t < ntiles; t += kOrderThreads) {
      int j = 0;
      for (int k = 1; k < njobs; k++)
        if (t >= jt[k][2]) j = k;
      const int id = t - jt[j][2];
      const int tx = id % jt[j][3], ty = id / jt[j][3];
      uint32_t c = 0u;
      for (int w = 0; w < nw; w++) c += wcost[(int64_t)t * nw + w];
      if (c != 0u) atomicAdd(&bcost[jt[j][0] + (tx >> bshift) + (ty >> bshift) * jt[j][1]], c);
    }
    __syncthreads();
  }
  // class index counted from the top class down (longest first)
  auto rank_of = [&](int g, const BinTiles& bt) -> int {
    uint32_t c = 0u;
    if (nw == 0) {
      c = trange[2 * g + 1] - trange[2 * g];
    } else if (lds_sum) {
      c = bcost[g];
    } else {
      for (int y = bt.y0; y < bt.y1; y++)
        for (int x = bt.x0; x < bt.x1; x++) {
          const int64_t t = bt.t0 + (int64_t)y * bt.tx + x;
          for (int w = 0; w < nw; w++) c += wcost[t * nw + w];
        }
    }
    return 128 - cost_class(c);
  };
  for (int g0 = 0; g0 < nbins; g0 += kOrderThreads * kOrderPer) {
#pragma unroll
    for (int u = 0; u < kOrderPer; u++) {
      const int g = g0 + u * kOrderThreads + (int)threadIdx.x;
      if (g < nbins) {
        const BinTiles bt = tiles_of(g);
        atomicAdd(&hist[rank_of(g, bt)], (uint32_t)((bt.x1 - bt.x0) * (bt.y1 - bt.y0)));
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int l = (int)threadIdx.x;
    const uint32_t a = hist[3 * l], b = hist[3 * l + 1], c = hist[3 * l + 2];
    uint32_t incl = a + b + c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t o = (uint32_t)__shfl_up((int)incl, off, 64);
      if (l >= off) incl += o;
    }
    const uint32_t excl = incl - (a + b + c);
    hist[3 * l] = excl;
    hist[3 * l + 1] = excl + a;
    hist[3 * l + 2] = excl + a + b;
  }
  __syncthreads();
  for (int g0 = 0; g0 < nbins; g0 += kOrderThreads * kOrderPer) {
#pragma unroll
    for (int u = 0; u < kOrderPer; u++) {
      const int g = g0 + u * kOrderThreads + (int)threadIdx.x;
      if (g < nbins) {
        const BinTiles bt = tiles_of(g);
        const uint32_t m = (uint32_t)((bt.x1 - bt.x0) * (bt.y1 - bt.y0));
        uint32_t pos = atomicAdd(&hist[rank_of(g, bt)], m);
        for (int y = bt.y0; y < bt.y1; y++)
          for (int x = bt.x0; x < bt.x1; x++) order[pos++] = (uint32_t)(bt.t0 + y * bt.tx + x);
      }
    }
  }
}

constexpr int kFwdGroup = 4;   // entries evaluated together in the forward
#ifndef MS_FWD_WAVES
#define MS_FWD_WAVES 8
#endif
#ifndef MS_BWDM_WAVES
#define MS_BWDM_WAVES 4
#endif

#define MS_FWD_PARAMS                                                                                          \
  const uint4 *__restrict__ rec, const uint32_t *__restrict__ pval, uint32_t rank_mask,                        \
      const uint32_t *__restrict__ trange, uint64_t *__restrict__ counters_rw, const JobDesc *__restrict__ jobs, \
      int njobs, int bshift, float *__restrict__ tfinal, uint32_t *__restrict__ last, uint32_t *__restrict__ wcost
#define MS_FWD_ARGS rec, pval, rank_mask, trange, counters_rw, jobs, njobs, bshift, tfinal, last, wcost

// Forward of compositing tile b. Each wave also leaves in wcost[b NW + wave]
// the deepest list position any of its pixels composited (0 for none): the
// length of the list walk the backward will make for its sub-block.
template <int TILE, int WB>
__device__ __forceinline__ void fwd_tile(int b, MS_FWD_PARAMS) {
  // the thread index, opaque to the compiler: in the persistent loop this
  // keeps the values derived from it from being hoisted and held live
  // across tiles
  int tid = (int)threadIdx.x;
  __asm__ volatile("" : "+v"(tid));
  constexpr int SB = TILE / 8;
  constexpr int NW = SB * SB;
  __shared__ Staged stage[NW][WB];
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const JobDesc& J = jobs[job_of_tile(jobs, njobs, b)];
  const int W = J.W, H = J.H;
  const int tile_id = b - J.tile0;
  const int tx = tile_id % J.tx, ty = tile_id / J.tx;
  const int bin_id = J.bin0 + (tx >> bshift) + (ty >> bshift) * J.bx;
  const auto rgb = global_ptr(J.rgb);
  const auto depth = global_ptr(J.depth);
  const auto sil = global_ptr(J.sil);
  const int X0 = tx * TILE + (wave % SB) * 8, Y0 = ty * TILE + (wave / SB) * 8;
  if (X0 >= W || Y0 >= H) {   // whole sub-block outside the image (wave-uniform)
    if (lane == 0) wcost[b * NW + wave] = 0u;
    return;
  }
  const int xl = lane & 7, yl = lane >> 3;
  const int x = X0 + xl, y = Y0 + yl;
  const bool inside = x < W && y < H;
  const bool overflow = counters_rw[C_OVERFLOW] != 0;
  const uint32_t start = overflow ? 0u : trange[2 * bin_id];
  const uint32_t end = overflow ? 0u : trange[2 * bin_id + 1];
  const float xf = (float)xl, yf = (float)yl;
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
  uint32_t lastpos = 0u, ncomp = 0u, staged = 0u;
  bool done = !inside;
  Staged* my = stage[wave];
  PairWords<WB> pw = load_pair_words<WB>(pval, start, (int)min((uint32_t)WB, end - start), lane);
  for (uint32_t b0 = start; b0 < end; b0 += WB) {
    if (__builtin_amdgcn_ballot_w64(!done) == 0) break;
    const int nb = (int)min((uint32_t)WB, end - b0);
    staged += (uint32_t)nb;
    wave_sync();
    int packed;
    const int cnt = stage_chunk_padded<WB>(rec, pw, rank_mask, b0 - start, nb, X0, Y0, lane, my, kFwdGroup, packed);
    wave_sync();
    if (b0 + WB < end)   // uniform: the next chunk's pair words, while this one composites
      pw = load_pair_words<WB>(pval, b0 + WB, (int)min((uint32_t)WB, end - (b0 + WB)), lane);
    for (int g = 0; g < cnt; g += kFwdGroup) {
      // acceptance values and alphas of the group: independent of each other
      float al[kFwdGroup];
      bool ac[kFwdGroup];
#pragma unroll
      for (int i = 0; i < kFwdGroup; i++) {
        const float4 ge = my[g + i].geo;
        const float4 cn = my[g + i].conic;
        const float lo2 = my[g + i].app.x;
        const float dx = (xf + ge.x) - ge.z;   // (x - ui) exactly, then - uf
        const float dy = (yf + ge.y) - ge.w;
        const float t1 = __builtin_fmaf(cn.x, dx, cn.y * dy);
        const float t2 = cn.z * dy;
        const float q = __builtin_fmaf(t1, t1, t2 * t2);
        ac[i] = q <= cn.w;
        al[i] = fminf(kAlphaMax, __builtin_amdgcn_exp2f(lo2 - q));
      }
      // front-to-back updates in list order; colours and depths are finite
      // (non-finite Gaussians are culled), so a zero weight leaves the sums
      // unchanged
#pragma unroll
      for (int i = 0; i < kFwdGroup; i++) {
        const float4 ap = my[g + i].app;
        const float2 mi = make_float2(my[g + i].misc.x, my[g + i].misc.z);
        const bool a = ac[i] && !done;
        const float Tn = T * (1.f - al[i]);
        const bool low = Tn < kTMin;
        const bool upd = a && !low;
        const float w = upd ? al[i] * T : 0.f;
        C0 = __builtin_fmaf(w, ap.z, C0);
        C1 = __builtin_fmaf(w, ap.w, C1);
        C2 = __builtin_fmaf(w, mi.x, C2);
        D = __builtin_fmaf(w, ap.y, D);
        T = upd ? Tn : T;
        lastpos = upd ? __float_as_uint(mi.y) : lastpos;
        ncomp += upd ? 1u : 0u;
        done = done || (a && low);
      }
      if (__builtin_amdgcn_ballot_w64(!done) == 0) break;
    }
  }
  const uint32_t deepest = wave_max_u32(lastpos);
  if (lane == 0) wcost[b * NW + wave] = deepest;
  // work counters: one atomic per wave
  uint32_t wsum = ncomp;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) wsum += (uint32_t)__shfl_xor((int)wsum, off, 64);
  if (lane == 0) {
    work_add(counters_rw, b * NW + wave, W_COMPOSITED, wsum);
    work_add(counters_rw, b * NW + wave, W_STAGED, staged);
  }
  if (!inside) return;
  const int64_t P = (int64_t)W * H;
  const int64_t pix = (int64_t)y * W + x;
  if (overflow) {
    const float nanv = __builtin_nanf("");
    rgb[pix] = rgb[P + pix] = rgb[2 * P + pix] = nanv;
    depth[pix] = sil[pix] = nanv;
    tfinal[J.pix0 + pix] = 1.f;
    last[J.pix0 + pix] = 0u;
    return;
  }
  rgb[pix] = C0;
  rgb[P + pix] = C1;
  rgb[2 * P + pix] = C2;
  depth[pix] = D;
  sil[pix] = 1.f - T;
  tfinal[J.pix0 + pix] = T;
  last[J.pix0 + pix] = lastpos;
}

template <int TILE, int WB>
__global__ void __launch_bounds__(64 * (TILE / 8) * (TILE / 8), MS_FWD_WAVES) k_composite_fwd(MS_FWD_PARAMS) {
  fwd_tile<TILE, WB>((int)blockIdx.x, MS_FWD_ARGS);
}

// Persistent form: as many workgroups as fit on the device at once, each
// taking tiles from the queue until it is empty.
template <int TILE, int WB>
__global__ void __launch_bounds__(64 * (TILE / 8) * (TILE / 8), MS_FWD_WAVES)
    k_composite_fwd_q(MS_FWD_PARAMS, const TileQueue tq) {
  for_queued_tiles(tq, [&](int b) { fwd_tile<TILE, WB>(b, MS_FWD_ARGS); });
}

// Scalar-record variant of the forward. The 64-byte record of the Gaussian
// the wave is evaluating is the same for all 64 lanes, so it is read with
// wave-uniform (scalar) loads into SGPRs and used directly as the scalar
// operand of the per-pixel VALU instructions: no LDS staging, no LDS
// broadcast traffic, and the sub-block skip test runs on the scalar unit.
// Ranks are read eight at a time.
struct RecS {
  float ui, vi, uf, vf, a, b, c, qcut, lo2, z, cr, cg, cb;
  uint32_t bx, by, idx;
};

__device__ inline RecS load_rec_uniform(const uint4* __restrict__ rec, uint32_t r) {
  const uint4* g = rec + 4 * (int64_t)r;
  const uint4 q0 = g[0], q1 = g[1], q2 = g[2], q3 = g[3];
  RecS s;
  s.ui = __uint_as_float(q0.x);
  s.vi = __uint_as_float(q0.y);
  s.uf = __uint_as_float(q0.z);
  s.vf = __uint_as_float(q0.w);
  s.a = __uint_as_float(q1.x);
  s.b = __uint_as_float(q1.y);
  s.c = __uint_as_float(q1.z);
  s.qcut = __uint_as_float(q1.w);
  s.lo2 = __uint_as_float(q2.x);
  s.z = __uint_as_float(q2.y);
  s.cr = __uint_as_float(q2.z);
  s.cg = __uint_as_float(q2.w);
  s.cb = __uint_as_float(q3.x);
  s.bx = q3.y;
  s.by = q3.z;
  s.idx = q3.w;
  return s;
}

__device__ inline bool box_misses(const RecS& s, int X0, int Y0) {
  const int bx0 = (int)(s.bx & 0xFFFFu), bx1 = (int)(s.bx >> 16);
  const int by0 = (int)(s.by & 0xFFFFu), by1 = (int)(s.by >> 16);
  return bx0 > X0 + 7 || bx1 < X0 || by0 > Y0 + 7 || by1 < Y0;
}

// Pinned acceptance value with absolute integer-valued pixel coordinates:
// (xa - ui) is exact, so dx is bit-identical to (float)(x - ui) - uf.
__device__ inline float accept_q_abs(const RecS& s, float xa, float ya, float& dx, float& dy, float& t1, float& t2) {
  dx = (xa - s.ui) - s.uf;
  dy = (ya - s.vi) - s.vf;
  t1 = __builtin_fmaf(s.a, dx, s.b * dy);
  t2 = s.c * dy;
  return __builtin_fmaf(t1, t1, t2 * t2);
}

template <int TILE>
__global__ void __launch_bounds__(64 * (TILE / 8) * (TILE / 8))
    k_composite_fwd_s(const uint4* __restrict__ rec, const uint32_t* __restrict__ pval, uint32_t rank_mask,
                      const uint32_t* __restrict__ trange, uint64_t* __restrict__ counters_rw, const JobDesc* __restrict__ jobs, int njobs, int bshift,
                      float* __restrict__ tfinal, uint32_t* __restrict__ last) {
  constexpr int SB = TILE / 8;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const JobDesc& J = jobs[job_of_tile(jobs, njobs, (int)blockIdx.x)];
  const int W = J.W, H = J.H;
  const int tile_id = (int)blockIdx.x - J.tile0;
  const int tx = tile_id % J.tx, ty = tile_id / J.tx;
  const int bin_id = J.bin0 + (tx >> bshift) + (ty >> bshift) * J.bx;
  const auto rgb = global_ptr(J.rgb);
  const auto depth = global_ptr(J.depth);
  const auto sil = global_ptr(J.sil);
  const int X0 = tx * TILE + (wave % SB) * 8, Y0 = ty * TILE + (wave / SB) * 8;
  if (X0 >= W || Y0 >= H) return;
  const int x = X0 + (lane & 7), y = Y0 + (lane >> 3);
  const bool inside = x < W && y < H;
  const bool overflow = counters_rw[C_OVERFLOW] != 0;
  const uint32_t start = overflow ? 0u : trange[2 * bin_id];
  const uint32_t end = overflow ? 0u : trange[2 * bin_id + 1];
  const float xa = (float)x, ya = (float)y;
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
  uint32_t lastpos = 0u, ncomp = 0u, staged = 0u;
  bool done = !inside;
  for (uint32_t k0 = start; k0 < end; k0 += 8) {
    if (__builtin_amdgcn_ballot_w64(!done) == 0) break;
    uint32_t rk[8];
#pragma unroll
    for (int i = 0; i < 8; i++) {
      const uint32_t k = k0 + i < end ? k0 + i : end - 1;
      rk[i] = pval[k] & rank_mask;
    }
    const int nb = (int)min(8u, end - k0);
    staged += (uint32_t)nb;
    for (int i = 0; i < nb; i++) {
      const RecS s = load_rec_uniform(rec, rk[i]);
      if (box_misses(s, X0, Y0)) continue;
      float dx, dy, t1, t2;
      const float q = accept_q_abs(s, xa, ya, dx, dy, t1, t2);
      if (!done && q <= s.qcut) {
        const float at = __builtin_amdgcn_exp2f(s.lo2 - q);
        const float alpha = fminf(kAlphaMax, at);
        const float Tn = T * (1.f - alpha);
        if (Tn < kTMin) {
          done = true;
        } else {
          const float w = alpha * T;
          C0 = __builtin_fmaf(w, s.cr, C0);
          C1 = __builtin_fmaf(w, s.cg, C1);
          C2 = __builtin_fmaf(w, s.cb, C2);
          D = __builtin_fmaf(w, s.z, D);
          T = Tn;
          lastpos = (k0 - start) + (uint32_t)i + 1u;
          ncomp++;
        }
      }
    }
  }
  uint32_t wsum = ncomp;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) wsum += (uint32_t)__shfl_xor((int)wsum, off, 64);
  if (lane == 0) {
    work_add(counters_rw, blockIdx.x * (SB * SB) + wave, W_COMPOSITED, wsum);
    work_add(counters_rw, blockIdx.x * (SB * SB) + wave, W_STAGED, staged);
  }
  if (!inside) return;
  const int64_t P = (int64_t)W * H;
  const int64_t pix = (int64_t)y * W + x;
  if (overflow) {
    const float nanv = __builtin_nanf("");
    rgb[pix] = rgb[P + pix] = rgb[2 * P + pix] = nanv;
    depth[pix] = sil[pix] = nanv;
    tfinal[J.pix0 + pix] = 1.f;
    last[J.pix0 + pix] = 0u;
    return;
  }
  rgb[pix] = C0;
  rgb[P + pix] = C1;
  rgb[2 * P + pix] = C2;
  depth[pix] = D;
  sil[pix] = 1.f - T;
  tfinal[J.pix0 + pix] = T;
  last[J.pix0 + pix] = lastpos;
}

template <int TILE, int WB>
__global__ void __launch_bounds__(64 * (TILE / 8) * (TILE / 8))
    k_composite_bwd(const uint4* __restrict__ rec, const uint32_t* __restrict__ pval, uint32_t rank_mask,
                    const uint32_t* __restrict__ trange, const uint64_t* __restrict__ counters, const JobDesc* __restrict__ jobs, int njobs, int bshift, const float* __restrict__ tfinal,
                    const uint32_t* __restrict__ last, float* __restrict__ g2d) {
  constexpr int SB = TILE / 8;
  constexpr int NW = SB * SB;
  __shared__ Staged stage[NW][WB];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const JobDesc& J = jobs[job_of_tile(jobs, njobs, (int)blockIdx.x)];
  const int W = J.W, H = J.H;
  const int tile_id = (int)blockIdx.x - J.tile0;
  const int tx = tile_id % J.tx, ty = tile_id / J.tx;
  const int bin_id = J.bin0 + (tx >> bshift) + (ty >> bshift) * J.bx;
  const int X0 = tx * TILE + (wave % SB) * 8, Y0 = ty * TILE + (wave / SB) * 8;
  if (X0 >= W || Y0 >= H) return;
  if (counters[C_OVERFLOW] != 0) return;
  const int xl = lane & 7, yl = lane >> 3;
  const int x = X0 + xl, y = Y0 + yl;
  const bool inside = x < W && y < H;
  const int64_t P = (int64_t)W * H;
  const int64_t pix = (int64_t)y * W + x;
  float G0 = 0.f, G1 = 0.f, G2 = 0.f, GD = 0.f, GS = 0.f, Tf = 1.f;
  uint32_t L = 0u;
  if (inside) {
    load_upstream(J, pix, P, G0, G1, G2, GD, GS);
    Tf = tfinal[J.pix0 + pix];
    L = last[J.pix0 + pix];
  }
  const uint32_t Lmax = wave_max_u32(L);
  const uint32_t start = trange[2 * bin_id];
  const float xf = (float)xl, yf = (float)yl;
  const float GST = GS * Tf;
  float T = Tf;      // transmittance after the current entry
  float R = 0.f;     // suffix sum of (G . c + G_D z) alpha T over later entries
  Staged* my = stage[wave];
  PairWords<WB> pw = load_pair_words<WB>(pval, start + (Lmax > (uint32_t)WB ? Lmax - WB : 0u),
                                         (int)min(Lmax, (uint32_t)WB), lane);
  for (uint32_t hi = Lmax; hi > 0;) {
    const uint32_t lo = hi > (uint32_t)WB ? hi - WB : 0u;
    const int nb = (int)(hi - lo);
    wave_sync();
    int packed;
    stage_chunk_padded<WB>(rec, pw, rank_mask, lo, nb, X0, Y0, lane, my, 1, packed);
    wave_sync();
    if (lo > 0)   // uniform: the next (earlier) chunk's pair words
      pw = load_pair_words<WB>(pval, start + (lo > (uint32_t)WB ? lo - WB : 0u), (int)min(lo, (uint32_t)WB), lane);
    for (int j = packed - 1; j >= 0; j--) {
      const Staged s = my[j];
      const uint32_t pos1 = __float_as_uint(s.misc.z);   // list position + 1
      float dx, dy, t1, t2;
      const float q = accept_q(s, xf, yf, dx, dy, t1, t2);
      const bool acc = pos1 <= L && q <= s.conic.w;
      if (!__any(acc)) continue;
      float f[kGradFields];
#pragma unroll
      for (int k = 0; k < kGradFields; k++) f[k] = 0.f;
      if (acc) {
        const float at = __builtin_amdgcn_exp2f(s.app.x - q);
        const float alpha = fminf(kAlphaMax, at);
        const float oma = 1.f - alpha;
        const float Tk = T / oma;
        const float w = alpha * Tk;
        const float gcz = __builtin_fmaf(G0, s.app.z, __builtin_fmaf(G1, s.app.w, __builtin_fmaf(G2, s.misc.x, GD * s.app.y)));
        const float dalpha = __builtin_fmaf(Tk, gcz, -(R - GST) / oma);
        const float e = at > kAlphaMax ? 0.f : dalpha * at;
        f[0] = e;
        f[1] = t1 * e;
        f[2] = t2 * e;
        f[3] = f[1] * dx;
        f[4] = f[1] * dy;
        f[5] = f[2] * dy;
        f[6] = G0 * w;
        f[7] = G1 * w;
        f[8] = G2 * w;
        f[9] = GD * w;
        R = __builtin_fmaf(gcz, w, R);
        T = Tk;
      }
#pragma unroll
      for (int k = 0; k < kGradFields; k++) f[k] = wave_sum(f[k]);
      if (lane < kGradFields) {
        float v = f[0];
#pragma unroll
        for (int k = 1; k < kGradFields; k++) v = lane == k ? f[k] : v;
        const uint32_t r = __float_as_uint(s.misc.y);
        unsafeAtomicAdd(&g2d[(int64_t)r * kGradFields + lane], v);
      }
    }
    hi = lo;
  }
}

// Full 64-lane sum, every lane receiving the total: DPP row steps (quad
// swaps, half-row and row mirrors) fused into the adds, then the gfx950
// row-pair and half-wave swaps.
__device__ inline float wave_sum_dpp(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false));
  const auto r16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  v = __uint_as_float(r16[0]) + __uint_as_float(r16[1]);
  const auto r32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r32[0]) + __uint_as_float(r32[1]);
}

// Scalar-record backward: records in SGPRs as in the forward; the list is
// walked back to front in groups of eight ranks.
template <int TILE>
__global__ void __launch_bounds__(64 * (TILE / 8) * (TILE / 8))
    k_composite_bwd_s(const uint4* __restrict__ rec, const uint32_t* __restrict__ pval, uint32_t rank_mask,
                      const uint32_t* __restrict__ trange, uint64_t* __restrict__ counters_rw, const JobDesc* __restrict__ jobs, int njobs, int bshift, const float* __restrict__ tfinal,
                      const uint32_t* __restrict__ last, float* __restrict__ g2d) {
  constexpr int SB = TILE / 8;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const JobDesc& J = jobs[job_of_tile(jobs, njobs, (int)blockIdx.x)];
  const int W = J.W, H = J.H;
  const int tile_id = (int)blockIdx.x - J.tile0;
  const int tx = tile_id % J.tx, ty = tile_id / J.tx;
  const int bin_id = J.bin0 + (tx >> bshift) + (ty >> bshift) * J.bx;
  const int X0 = tx * TILE + (wave % SB) * 8, Y0 = ty * TILE + (wave / SB) * 8;
  if (X0 >= W || Y0 >= H) return;
  if (counters_rw[C_OVERFLOW] != 0) return;
  const int x = X0 + (lane & 7), y = Y0 + (lane >> 3);
  const bool inside = x < W && y < H;
  const int64_t P = (int64_t)W * H;
  const int64_t pix = (int64_t)y * W + x;
  float G0 = 0.f, G1 = 0.f, G2 = 0.f, GD = 0.f, GS = 0.f, Tf = 1.f;
  uint32_t L = 0u;
  if (inside) {
    load_upstream(J, pix, P, G0, G1, G2, GD, GS);
    Tf = tfinal[J.pix0 + pix];
    L = last[J.pix0 + pix];
  }
  const uint32_t Lmax = __builtin_amdgcn_readfirstlane(wave_max_u32(L));
  const uint32_t start = trange[2 * bin_id];
  const float xa = (float)x, ya = (float)y;
  const float GST = GS * Tf;
  float T = Tf;
  float R = 0.f;
  uint32_t reduced = 0u;
  for (uint32_t hi = Lmax; hi > 0;) {
    const uint32_t nb = hi < 8u ? hi : 8u;
    const uint32_t lo = hi - nb;
    uint32_t rk[8];
#pragma unroll
    for (int i = 0; i < 8; i++) {
      const uint32_t k = (uint32_t)i < nb ? start + lo + (uint32_t)i : start + lo;
      rk[i] = pval[k] & rank_mask;
    }
    for (int i = (int)nb - 1; i >= 0; i--) {
      const RecS s = load_rec_uniform(rec, rk[i]);
      if (box_misses(s, X0, Y0)) continue;
      const uint32_t pos = lo + (uint32_t)i;
      float dx, dy, t1, t2;
      const float q = accept_q_abs(s, xa, ya, dx, dy, t1, t2);
      const bool acc = pos < L && q <= s.qcut;
      if (__builtin_amdgcn_ballot_w64(acc) == 0) continue;
      reduced++;
      float f[kGradFields];
#pragma unroll
      for (int k = 0; k < kGradFields; k++) f[k] = 0.f;
      if (acc) {
        const float at = __builtin_amdgcn_exp2f(s.lo2 - q);
        const float alpha = fminf(kAlphaMax, at);
        const float inv = __builtin_amdgcn_rcpf(1.f - alpha);
        const float Tk = T * inv;
        const float w = alpha * Tk;
        const float gcz = __builtin_fmaf(G0, s.cr, __builtin_fmaf(G1, s.cg, __builtin_fmaf(G2, s.cb, GD * s.z)));
        const float dalpha = __builtin_fmaf(Tk, gcz, -(R - GST) * inv);
        const float e = at > kAlphaMax ? 0.f : dalpha * at;
        f[0] = e;
        f[1] = t1 * e;
        f[2] = t2 * e;
        f[3] = f[1] * dx;
        f[4] = f[1] * dy;
        f[5] = f[2] * dy;
        f[6] = G0 * w;
        f[7] = G1 * w;
        f[8] = G2 * w;
        f[9] = GD * w;
        R = __builtin_fmaf(gcz, w, R);
        T = Tk;
      }
#pragma unroll
      for (int k = 0; k < kGradFields; k++) f[k] = wave_sum_dpp(f[k]);
      if (lane < kGradFields) {
        float v = f[0];
#pragma unroll
        for (int k = 1; k < kGradFields; k++) v = lane == k ? f[k] : v;
        unsafeAtomicAdd(&g2d[(int64_t)rk[i] * kGradFields + lane], v);
      }
    }
    hi = lo;
  }
  if (lane == 0) work_add(counters_rw, blockIdx.x * (SB * SB) + wave, W_REDUCED, reduced);
}

// Backward with the per-Gaussian reduction over the wave's 64 pixels done on
// the matrix cores. All ten screen-space sums of a Gaussian are linear in the
// moments
//   sum_p e_p (1, x, y, x^2, xy, y^2)   and   sum_p w_p (G_r, G_g, G_b, G_D)
// of e = dL/dalpha * alpha~ and w = alpha T over the pixels p (x, y pixel
// coordinates about the sub-block centre). For a group of 8 Gaussians, each
// pixel lane writes its e values to rows 0-7 and its w values to rows 8-15 of
// a 16 x 64 LDS matrix A; the moment matrix M (16 x 64) holds the six
// monomials in rows 0-5 and the four upstream values in rows 6-9, so the
// product M A^T yields both sets of sums: per 32-pixel half, three
// v_mfma_f32_16x16x32_bf16 on high and low bf16 parts (about 16 significant
// bits per term). One lane per Gaussian then shifts the moments to the
// Gaussian's centre and forms the ten sums, as the binary32 kernel below
// does (its error bound holds here with the bf16 product error, about
// 2^-15 per term, in place of u). The sums leave as whole-Gaussian atomics,
// through the workgroup's LDS accumulator where the list position allows.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int kGrp = 8;                        // Gaussians per product
constexpr int kRow = 68;                       // padded row of 64 pixel values (bank spread)
constexpr int kWaveLds = 16 * kRow;            // floats per wave: the A matrix
// One staging round covers a full wave of list entries (every lane tests
// one record). With the LDS accumulator at 176 rows a 16-px tile's
// workgroup needs 40832 bytes of LDS, so four still fit on a CU.
#ifndef MS_BWD_CHUNK
#define MS_BWD_CHUNK 64
#endif
constexpr int kBwdChunk = MS_BWD_CHUNK;        // list entries packed per staging round
#define MS_BWD_PARAMS                                                                                     \
  const uint4 *__restrict__ rec, const uint32_t *__restrict__ pval, uint32_t rank_mask,                   \
      const uint32_t *__restrict__ trange, uint64_t *__restrict__ counters_rw, const JobTable &tbl,       \
      JobTable *__restrict__ tbl_dst, int bshift, const float *__restrict__ tfinal,                       \
      const uint32_t *__restrict__ last, float *__restrict__ g2d
#define MS_BWD_ARGS rec, pval, rank_mask, trange, counters_rw, tbl, tbl_dst, bshift, tfinal, last, g2d
// kernels take the job table by value
#define MS_BWD_KPARAMS                                                                                    \
  const uint4 *__restrict__ rec, const uint32_t *__restrict__ pval, uint32_t rank_mask,                   \
      const uint32_t *__restrict__ trange, uint64_t *__restrict__ counters_rw, const JobTable tbl,        \
      JobTable *__restrict__ tbl_dst, int bshift, const float *__restrict__ tfinal,                       \
      const uint32_t *__restrict__ last, float *__restrict__ g2d

constexpr int kBwdStep = 4;                    // entries whose alphas are evaluated together
#ifndef MS_ACC_ROWS
#define MS_ACC_ROWS 176
#endif
constexpr int kAccRows = MS_ACC_ROWS;          // list positions aggregated in LDS per workgroup
static_assert(kBwdChunk % kBwdStep == 0 && kBwdChunk <= 64, "a staging round pads to whole evaluation groups in one wave");

template <int TILE>
__device__ __forceinline__ void bwd_m_tile(int b, MS_BWD_PARAMS) {
  // the thread index, opaque to the compiler: in the persistent loop this
  // keeps the values derived from it from being hoisted and held live
  // across tiles
  int tid = (int)threadIdx.x;
  __asm__ volatile("" : "+v"(tid));
  constexpr int SB = TILE / 8;
  constexpr int NW = SB * SB;
  // the job table arrives by value; the first workgroup leaves a copy in the
  // workspace for the projection adjoint
  const JobDesc* jobs = tbl.job;
  const int njobs = tbl.njobs;
  if (b == 0) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&tbl);
    uint32_t* d = reinterpret_cast<uint32_t*>(tbl_dst);
    for (int i = tid; i < (int)(sizeof(JobTable) / 4); i += 64 * NW) d[i] = src[i];
  }
  __shared__ __attribute__((aligned(16))) float lds[NW * kWaveLds];
  __shared__ Staged stage[NW][kBwdChunk];
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const JobDesc& J = jobs[job_of_tile(jobs, njobs, b)];
  const int W = J.W, H = J.H;
  const int tile_id = b - J.tile0;
  const int tx = tile_id % J.tx, ty = tile_id / J.tx;
  const int bin_id = J.bin0 + (tx >> bshift) + (ty >> bshift) * J.bx;
  const int X0 = tx * TILE + (wave % SB) * 8, Y0 = ty * TILE + (wave / SB) * 8;
  if (counters_rw[C_OVERFLOW] != 0) return;   // uniform over the launch
  // Sums of the block's waves for the same Gaussian meet in LDS, indexed by
  // the entry's position in the bin list (the same in every wave of the
  // block); the block then issues one global atomic per (tile, Gaussian,
  // field) instead of one per wave. Positions past kAcc go straight to HBM.
  constexpr int kAcc = NW > 1 ? kAccRows : 0;
  __shared__ float acc[kAcc > 0 ? kAcc * kGradFields : 1];
  if (kAcc > 0) {
    for (int i = tid; i < kAcc * kGradFields; i += 64 * NW) acc[i] = 0.f;
    __syncthreads();
  }
  if (X0 < W && Y0 < H) {   // wave-uniform: sub-blocks wholly outside the image do nothing
  float* A = lds + wave * kWaveLds;    // [16 rows][4 k][16 s] (row stride kRow), pixel p = 4 s + k
  Staged* my = stage[wave];
  const int xl = lane & 7, yl = lane >> 3;
  const int x = X0 + xl, y = Y0 + yl;
  const bool inside = x < W && y < H;
  const int64_t P = (int64_t)W * H;
  const int64_t pix = (int64_t)y * W + x;
  float G0 = 0.f, G1 = 0.f, G2 = 0.f, GD = 0.f, GS = 0.f, Tf = 1.f;
  uint32_t L = 0u;
  if (inside) {
    load_upstream(J, pix, P, G0, G1, G2, GD, GS);
    Tf = tfinal[J.pix0 + pix];
    L = last[J.pix0 + pix];
  }
  // First product operand (constant per wave): the moment rows M^T. Lane
  // (k, j) = (lane / 16, lane % 16) holds row j at the pixels 32 h + 8 k + t,
  // t < 8, of the two 32-pixel halves h, split into bf16 high and low parts
  // (the monomial rows are exact in bf16; the upstream rows are not).
  const int pk = lane >> 4, pj = lane & 15;
  bf16x8 Mhi[2], Mlo[2];
  A[lane * 4 + 0] = G0;
  A[lane * 4 + 1] = G1;
  A[lane * 4 + 2] = G2;
  A[lane * 4 + 3] = GD;
  wave_sync();
#pragma unroll
  for (int h = 0; h < 2; h++) {
#pragma unroll
    for (int t = 0; t < 8; t++) {
      const int p = 32 * h + 8 * pk + t;
      const float px = (float)(p & 7) - 3.5f, py = (float)(p >> 3) - 3.5f;
      float m = 0.f;
      m = pj == 0 ? 1.f : m;
      m = pj == 1 ? px : m;
      m = pj == 2 ? py : m;
      m = pj == 3 ? px * px : m;
      m = pj == 4 ? px * py : m;
      m = pj == 5 ? py * py : m;
      m = (pj >= 6 && pj < 10) ? A[p * 4 + (pj - 6)] : m;
      const __bf16 mh = (__bf16)m;
      Mhi[h][t] = mh;
      Mlo[h][t] = (__bf16)(m - (float)mh);
    }
  }
  wave_sync();
  const uint32_t Lmax = __builtin_amdgcn_readfirstlane(wave_max_u32(L));
  const uint32_t start = trange[2 * bin_id];
  const float xf = (float)xl, yf = (float)yl;
  float T = Tf;
  float Rs = -(GS * Tf);   // suffix sum of (G_rgb . c + G_depth z) alpha T, minus G_sil T_final
  uint32_t reduced = 0u;
  const int eaddr = lane;   // pixel-contiguous rows of A
  // Rows g < count of A (e values) and 8 + g (w values) belong to the packed
  // entry held in lane g's `rowent`; only entries that some pixel of the wave
  // composites get a row, so every product reduces contributing entries only.
  // The product is formed transposed (moments x entries): lane (k, j) then
  // holds moments 4k .. 4k+3 of row j, so lane g gathers its entry's six
  // moments and four weighted sums from three other lanes with shuffles and
  // issues the ten accumulations itself.
  int rowent = 0;
  float* Fg = A;                                                  // [kGrp][10] sums bound for HBM
  uint32_t* Fslot = reinterpret_cast<uint32_t*>(A + kGrp * kGradFields);   // [kGrp] their accumulator rows
  auto flush = [&](int count) {
    bool to_global = false;
    wave_sync();
    // second operand: lane (k, j) holds row j of A at the pixels 32 h + 8 k + t;
    // three bf16 products (hi.hi + hi.lo + lo.hi) per half keep about 16
    // significant bits of every term
    f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int h = 0; h < 2; h++) {
      const float4* r4 = reinterpret_cast<const float4*>(A + pj * kRow + 32 * h + 8 * pk);
      const float4 x0 = r4[0], x1 = r4[1];
      const float v[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
      // high parts by truncation (a byte permute packs two of them), low
      // parts rounded from the exact remainders
      bf16x8 rh, rl;
      u32x4 hw;
#pragma unroll
      for (int t = 0; t < 8; t += 2) {
        const uint32_t u0 = __float_as_uint(v[t]), u1 = __float_as_uint(v[t + 1]);
        hw[t / 2] = __builtin_amdgcn_perm(u1, u0, 0x07060302u);   // high halves, truncated
        rl[t] = (__bf16)(v[t] - __uint_as_float(u0 & 0xFFFF0000u));
        rl[t + 1] = (__bf16)(v[t + 1] - __uint_as_float(u1 & 0xFFFF0000u));
      }
      rh = __builtin_bit_cast(bf16x8, hw);
      d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Mhi[h], rh, d, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Mhi[h], rl, d, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Mlo[h], rh, d, 0, 0, 0);
    }
    // lane g < 8: moments 0-3 in d[0..3]; moments 4, 5 in lane 16 + g; weighted
    // sums 6, 7 in lane 24 + g (d[2], d[3]) and 8, 9 in lane 40 + g (d[0], d[1])
    const int l = lane & 7;
    const float S4 = __shfl(d[0], 16 + l, 64), S5 = __shfl(d[1], 16 + l, 64);
    const float W6 = __shfl(d[2], 24 + l, 64), W7 = __shfl(d[3], 24 + l, 64);
    const float W8 = __shfl(d[0], 40 + l, 64), W9 = __shfl(d[1], 40 + l, 64);
    if (lane < count) {
      const Staged& sg = my[rowent];
      const float S1 = d[0], Sx = d[1], Sy = d[2], Sxx = d[3], Sxy = S4, Syy = S5;
      const float U = ((-sg.geo.x) - 3.5f) + sg.geo.z;   // ui - X0 - 3.5 + uf
      const float V = ((-sg.geo.y) - 3.5f) + sg.geo.w;
      const float a = sg.conic.x, b = sg.conic.y, c = sg.conic.z;
      // the moments shift to the Gaussian's centre through k1 = a U + b V,
      // which stays bounded for any Gaussian composited in the sub-block (see
      // the binary32 kernel below for the bound)
      const float k1 = __builtin_fmaf(a, U, b * V);
      const float P1 = __builtin_fmaf(a, Sx, __builtin_fmaf(b, Sy, -(k1 * S1)));
      float f[kGradFields];
      f[0] = S1;
      f[1] = P1;
      f[2] = c * __builtin_fmaf(-V, S1, Sy);
      f[3] = __builtin_fmaf(a, Sxx, __builtin_fmaf(b, Sxy, -(k1 * Sx))) - U * P1;
      f[4] = __builtin_fmaf(a, Sxy, __builtin_fmaf(b, Syy, -(k1 * Sy))) - V * P1;
      f[5] = c * __builtin_fmaf(V * V, S1, __builtin_fmaf(-2.f * V, Sy, Syy));
      f[6] = W6;
      f[7] = W7;
      f[8] = W8;
      f[9] = W9;
      const uint32_t pos = __float_as_uint(sg.misc.z) - 1u;   // list position
      to_global = !(kAcc > 0 && pos < (uint32_t)kAcc);
      if (!to_global) {
        float* dst = &acc[pos * kGradFields];
#pragma unroll
        for (int k = 0; k < kGradFields; k++) atomicAdd(dst + k, f[k]);
      } else {
        // global sums go through LDS so that each atomic instruction covers
        // whole Gaussians (ten consecutive floats), which the memory side
        // serves far better than ten instructions of scattered lanes
#pragma unroll
        for (int k = 0; k < kGradFields; k++) Fg[lane * kGradFields + k] = f[k];
        Fslot[lane] = __float_as_uint(sg.misc.y);
      }
    }
    const uint64_t gmask = __builtin_amdgcn_ballot_w64(lane < count && to_global);
    if (gmask != 0) {   // uniform
      wave_sync();
      for (int idx = lane; idx < count * kGradFields; idx += 64) {
        const int g = idx / kGradFields, fi = idx - g * kGradFields;
        if ((gmask >> g) & 1u) {
          const float v = Fg[idx];
          if (v != 0.f) unsafeAtomicAdd(g2d + (int64_t)Fslot[g] * kGradFields + fi, v);
        }
      }
    }
    wave_sync();   // the next rows of A overwrite Fg
  };
  PairWords<kBwdChunk> pw = load_pair_words<kBwdChunk>(
      pval, start + (Lmax > (uint32_t)kBwdChunk ? Lmax - kBwdChunk : 0u), (int)min(Lmax, (uint32_t)kBwdChunk), lane);
  for (uint32_t hi = Lmax; hi > 0;) {
    const uint32_t lo = hi > (uint32_t)kBwdChunk ? hi - kBwdChunk : 0u;
    const int nb = (int)(hi - lo);
    wave_sync();
    int packed;
    const int cnt = stage_chunk_padded<kBwdChunk>(rec, pw, rank_mask, lo, nb, X0, Y0, lane, my, kBwdStep, packed);
    wave_sync();
    if (lo > 0)   // uniform: the next (earlier) chunk's pair words, while this one is reduced
      pw = load_pair_words<kBwdChunk>(pval, start + (lo > (uint32_t)kBwdChunk ? lo - kBwdChunk : 0u),
                                      (int)min(lo, (uint32_t)kBwdChunk), lane);
    reduced += (uint32_t)packed;
    int rows = 0;   // uniform: rows of A filled since the last product
    for (int top = cnt - 1; top >= 0; top -= kBwdStep) {   // cnt is a multiple of kBwdStep
      if (rows > kGrp - kBwdStep) {   // room for a whole step of entries
        flush(rows);
        rows = 0;
      }
      float at[kBwdStep], alpha[kBwdStep], inv[kBwdStep], gcz[kBwdStep];
      bool acc[kBwdStep];
      // the step's entries from one base address in a VGPR, so that the four
      // reads use immediate offsets
      int lo_slot = top - (kBwdStep - 1);
      __asm__ volatile("" : "+v"(lo_slot));
      const Staged* sp = my + lo_slot;
#pragma unroll
      for (int k = 0; k < kBwdStep; k++) {
        const Staged& sk = sp[kBwdStep - 1 - k];
        const float4 ge = sk.geo, cn = sk.conic, ap = sk.app;
        const float2 mi = make_float2(sk.misc.x, sk.misc.z);
        const float dx = (xf + ge.x) - ge.z;
        const float dy = (yf + ge.y) - ge.w;
        const float t1 = __builtin_fmaf(cn.x, dx, cn.y * dy);
        const float t2 = cn.z * dy;
        const float q = __builtin_fmaf(t1, t1, t2 * t2);
        acc[k] = __float_as_uint(mi.y) <= L && q <= cn.w;   // list position < last
        // a pixel that does not composite the entry takes alpha~ = 0: its
        // weight, its e and its share of the suffix sum are then exactly zero
        at[k] = acc[k] ? __builtin_amdgcn_exp2f(ap.x - q) : 0.f;
        alpha[k] = fminf(kAlphaMax, at[k]);
        inv[k] = __builtin_amdgcn_rcpf(1.f - alpha[k]);
        gcz[k] = __builtin_fmaf(G0, ap.z, __builtin_fmaf(G1, ap.w, __builtin_fmaf(G2, mi.x, GD * ap.y)));
      }
      // back-to-front recursion; only the transmittance needs the predicate
#pragma unroll
      for (int k = 0; k < kBwdStep; k++) {
        const float Tk = T * inv[k];
        const float w = alpha[k] * Tk;
        const float dalpha = __builtin_fmaf(Tk, gcz[k], -Rs * inv[k]);
        const float e = at[k] > kAlphaMax ? 0.f : dalpha * at[k];
        Rs = __builtin_fmaf(gcz[k], w, Rs);
        T = acc[k] ? Tk : T;
        if (__builtin_amdgcn_ballot_w64(acc[k]) != 0) {   // uniform
          A[rows * kRow + eaddr] = e;
          A[(kGrp + rows) * kRow + eaddr] = w;
          rowent = writelane_u(top - k, rows, rowent);
          rows++;
        }
      }
    }
    if (rows > 0) flush(rows);
    hi = lo;
  }
  if (lane == 0) work_add(counters_rw, b * NW + wave, W_REDUCED, reduced);
  }
  if (kAcc > 0) {
    __syncthreads();
    const uint32_t start = trange[2 * bin_id];
    for (int i = tid; i < kAcc * kGradFields; i += 64 * NW) {
      const float v = acc[i];
      if (v != 0.f) {   // only rows of list entries some wave packed
        const int pos = i / kGradFields, fi = i - pos * kGradFields;
        const uint32_t r = pval[start + (uint32_t)pos] & rank_mask;
        unsafeAtomicAdd(g2d + (int64_t)r * kGradFields + fi, v);
      }
    }
  }
}

template <int TILE>
__global__ void __launch_bounds__(64 * (TILE / 8) * (TILE / 8), MS_BWDM_WAVES) k_composite_bwd_m(MS_BWD_KPARAMS) {
  bwd_m_tile<TILE>((int)blockIdx.x, MS_BWD_ARGS);
}

template <int TILE>
__global__ void __launch_bounds__(64 * (TILE / 8) * (TILE / 8), MS_BWDM_WAVES)
    k_composite_bwd_m_q(MS_BWD_KPARAMS, const TileQueue tq) {
  for_queued_tiles(tq, [&](int b) { bwd_m_tile<TILE>(b, MS_BWD_ARGS); });
}

// Backward with the per-Gaussian reduction over the wave's 64 pixels on the
// matrix cores in binary32 (v_mfma_f32_16x16x4_f32: fp32 operands, fp32
// accumulation). Each Gaussian the wave composites gets two columns of a
// wave-private 16-column LDS matrix, one value per pixel:
//   e = dL/dalpha * alpha~,   w = alpha T.
// The moment operand holds, per pixel, the rows
//   1, xi, eta, xi^2, xi eta, eta^2, G_r, G_g, G_b, G_D
// (xi, eta the pixel's offset from the sub-block centre), so one product
// yields, for eight Gaussians at a time, the moments
//   S = sum e (1, xi, eta, xi^2, xi eta, eta^2)   and   sum w (G_r, G_g, G_b, G_D).
// With (U, V) the Gaussian centre's offset from the sub-block centre, a pixel
// has dx = xi - U, dy = eta - V, t2 = c dy and
//   t1 = a dx + b dy = (a xi + b eta) - k1,   k1 = a U + b V,
// so the ten screen-space sums are
//   E = S1,  P1 = a Sx + b Sy - k1 S1,  P2 = c (Sy - V S1),
//   P1x = (a Sxx + b Sxy - k1 Sx) - U P1,  P1y = (a Sxy + b Syy - k1 Sy) - V P1,
//   P2y = c ((Syy - 2 V Sy) + V^2 S1),
// and the four weighted upstream sums.
//
// Error bound. The screen covariance carries the 0.3 px^2 dilation, which
// bounds the scaled Cholesky factors: |a|, |b|, |c| <= K / sqrt(0.3) ~ 1.55
// (K^2 = log2(e) / 2). A Gaussian that composites at some pixel of the
// sub-block has |t1| <= sqrt(qcut) there, and |xi|, |eta| <= 3.5, so
//   |k1| <= 3.5 (|a| + |b|) + sqrt(qcut),     |c V| <= 3.5 |c| + sqrt(qcut).
// Forming k1 first (one rounding of relative size u = 2^-24, the same
// rounding the pixel's own t1 carries) and with gamma the binary32 error of
// a 64-term sum, each moment errs by at most gamma sum |e| |monomial|, and
//   |dP1| <= (gamma + 3u) L sum|e|,        L = 3.5 (|a| + |b|) + |k1| <= 13.5,
//   |dP1x| <= (gamma + 4u) (3.5 + |U|) L sum|e|,   |dP1y| likewise with V,
//   |dP2| <= (gamma + 2u) (7 |c| + sqrt(qcut)) sum|e|,
//   |dP2y| <= (gamma + 4u) (7 |c| + sqrt(qcut)) (3.5 + |V|) sum|e|,
// while the sums themselves are bounded by sqrt(qcut) sum|e| times the same
// offset factors. Relative to that size the error is (gamma + 4u) times at
// most (13.5 + sqrt(qcut)) / sqrt(qcut): no Gaussian shape (elongation,
// distance of its centre from the sub-block) makes it grow; only opacity
// within a few per cent of the 1/255 floor (qcut near 0, where every sum is
// small) does, and there the absolute error stays below 16 (gamma + 4u)
// sum|e|. (Shifting by U and V separately, as Sx - U S1 and Sy - V S1, adds
// roundings of size u |a U| and u |b V|, which grow with the distance of an
// elongated Gaussian's centre; k1 does not.)
constexpr int kGrpF = 8;                       // Gaussians per product (two columns each)

template <int TILE>
__device__ __forceinline__ void bwd_f_tile(int b, MS_BWD_PARAMS) {
  // the thread index, opaque to the compiler: in the persistent loop this
  // keeps the values derived from it from being hoisted and held live
  // across tiles
  int tid = (int)threadIdx.x;
  __asm__ volatile("" : "+v"(tid));
  constexpr int SB = TILE / 8;
  constexpr int NW = SB * SB;
  const JobDesc* jobs = tbl.job;
  const int njobs = tbl.njobs;
  if (b == 0) {   // leave the job table for the projection adjoint
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&tbl);
    uint32_t* d = reinterpret_cast<uint32_t*>(tbl_dst);
    for (int i = tid; i < (int)(sizeof(JobTable) / 4); i += 64 * NW) d[i] = src[i];
  }
  __shared__ __attribute__((aligned(16))) float lds[NW * kWaveLds];
  __shared__ Staged stage[NW][kBwdChunk];
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const JobDesc& J = jobs[job_of_tile(jobs, njobs, b)];
  const int W = J.W, H = J.H;
  const int tile_id = b - J.tile0;
  const int tx = tile_id % J.tx, ty = tile_id / J.tx;
  const int bin_id = J.bin0 + (tx >> bshift) + (ty >> bshift) * J.bx;
  const int X0 = tx * TILE + (wave % SB) * 8, Y0 = ty * TILE + (wave / SB) * 8;
  if (counters_rw[C_OVERFLOW] != 0) return;   // uniform over the launch
  // sums of the block's waves for one Gaussian meet in LDS, indexed by list
  // position (the same in every wave of the block); positions past kAcc go
  // straight to HBM
  constexpr int kAcc = NW > 1 ? kAccRows : 0;
  __shared__ float acc[kAcc > 0 ? kAcc * kGradFields : 1];
  if (kAcc > 0) {
    for (int i = tid; i < kAcc * kGradFields; i += 64 * NW) acc[i] = 0.f;
    __syncthreads();
  }
  if (X0 < W && Y0 < H) {   // wave-uniform: sub-blocks wholly outside the image do nothing
  float* A = lds + wave * kWaveLds;   // [16 columns][kRow]: column j, pixel p at j * kRow + p
  Staged* my = stage[wave];
  const int xl = lane & 7, yl = lane >> 3;
  const int x = X0 + xl, y = Y0 + yl;
  const bool inside = x < W && y < H;
  const int64_t P = (int64_t)W * H;
  const int64_t pix = (int64_t)y * W + x;
  float G0 = 0.f, G1 = 0.f, G2 = 0.f, GD = 0.f, GS = 0.f, Tf = 1.f;
  uint32_t L = 0u;
  if (inside) {
    load_upstream(J, pix, P, G0, G1, G2, GD, GS);
    Tf = tfinal[J.pix0 + pix];
    L = last[J.pix0 + pix];
  }
  // Moment operand of v_mfma_f32_16x16x4_f32, constant per wave. Product k
  // (0..15) covers the pixels 16 q + k, q = 0..3; lane (q, i) = (lane / 16,
  // lane % 16) supplies row i of the moment matrix at pixel 16 q + k, and
  // later column i of the value matrix at the same pixel.
  const int pq = lane >> 4, pi = lane & 15;
  float Mf[16];
  A[lane * 4 + 0] = G0;
  A[lane * 4 + 1] = G1;
  A[lane * 4 + 2] = G2;
  A[lane * 4 + 3] = GD;
  wave_sync();
#pragma unroll
  for (int k = 0; k < 16; k++) {
    const int p = 16 * pq + k;
    const float px = (float)(p & 7) - 3.5f, py = (float)(p >> 3) - 3.5f;
    float m = 0.f;
    m = pi == 0 ? 1.f : m;
    m = pi == 1 ? px : m;
    m = pi == 2 ? py : m;
    m = pi == 3 ? px * px : m;
    m = pi == 4 ? px * py : m;
    m = pi == 5 ? py * py : m;
    m = (pi >= 6 && pi < 10) ? A[p * 4 + (pi - 6)] : m;
    Mf[k] = m;
  }
  wave_sync();
  const uint32_t Lmax = __builtin_amdgcn_readfirstlane(wave_max_u32(L));
  const uint32_t start = trange[2 * bin_id];
  const float xf = (float)xl, yf = (float)yl;
  float T = Tf;
  float Rs = -(GS * Tf);   // suffix sum of (G_rgb . c + G_depth z) alpha T, minus G_sil T_final
  uint32_t reduced = 0u;
  // Lane g < count holds in `rowent` the staged slot of the product's entry
  // g, whose columns are g (e) and 8 + g (w).
  int rowent = 0;
  // sums bound for HBM and their accumulator rows, in columns 14 and 15 (w
  // columns, read into registers before these are written)
  float* Fg = A + 14 * kRow;                                              // [kGrpF][10]
  uint32_t* Fslot = reinterpret_cast<uint32_t*>(Fg + kGrpF * kGradFields);   // [kGrpF]
  static_assert(kGrpF * (kGradFields + 1) <= 2 * kRow, "HBM staging fits two columns");
  auto flush = [&](int count) {
    wave_sync();
    const float4* r4 = reinterpret_cast<const float4*>(A + pi * kRow + 16 * pq);
    const float4 v0 = r4[0], v1 = r4[1], v2 = r4[2], v3 = r4[3];
    f32x4 d0 = {0.f, 0.f, 0.f, 0.f}, d1 = {0.f, 0.f, 0.f, 0.f};
    d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(Mf[0], v0.x, d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(Mf[1], v0.y, d1, 0, 0, 0);
    d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(Mf[2], v0.z, d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(Mf[3], v0.w, d1, 0, 0, 0);
    d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(Mf[4], v1.x, d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(Mf[5], v1.y, d1, 0, 0, 0);
    d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(Mf[6], v1.z, d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(Mf[7], v1.w, d1, 0, 0, 0);
    d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(Mf[8], v2.x, d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(Mf[9], v2.y, d1, 0, 0, 0);
    d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(Mf[10], v2.z, d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(Mf[11], v2.w, d1, 0, 0, 0);
    d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(Mf[12], v3.x, d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(Mf[13], v3.y, d1, 0, 0, 0);
    d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(Mf[14], v3.z, d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(Mf[15], v3.w, d1, 0, 0, 0);
    // lane (q, i) holds rows 4q .. 4q + 3 of column i. Entry g: lane g has
    // S1, Sx, Sy, Sxx; lane 16 + g has Sxy, Syy; lane 24 + g the w-sums of
    // G_r, G_g (rows 6, 7); lane 40 + g those of G_b, G_D (rows 8, 9).
    const float s0 = d0[0] + d1[0], s1 = d0[1] + d1[1], s2 = d0[2] + d1[2], s3 = d0[3] + d1[3];
    const int l = lane & 7;
    const float Sxy = __shfl(s0, 16 + l, 64), Syy = __shfl(s1, 16 + l, 64);
    const int ent = __shfl(rowent, l, 64);   // entry l's staged slot
    bool to_global = false;
    int i0 = 0;
    float v0f = 0.f, v1f = 0.f;
    const bool is_e = lane < count;
    const bool is_w = (lane >= 24 && lane < 24 + count) || (lane >= 40 && lane < 40 + count);
    if (is_e || is_w) {
      const Staged& sg = my[ent];
      const uint32_t pos = __float_as_uint(sg.misc.z) - 1u;   // list position
      to_global = !(kAcc > 0 && pos < (uint32_t)kAcc);
      float f[6];
      if (is_e) {
        const float S1 = s0, Sx = s1, Sy = s2, Sxx = s3;
        const float U = ((-sg.geo.x) - 3.5f) + sg.geo.z;   // ui - X0 - 3.5 + uf
        const float V = ((-sg.geo.y) - 3.5f) + sg.geo.w;   // vi - Y0 - 3.5 + vf
        const float a = sg.conic.x, b = sg.conic.y, c = sg.conic.z;
        const float k1 = __builtin_fmaf(a, U, b * V);
        const float P1 = __builtin_fmaf(a, Sx, __builtin_fmaf(b, Sy, -(k1 * S1)));
        f[0] = S1;
        f[1] = P1;
        f[2] = c * __builtin_fmaf(-V, S1, Sy);
        f[3] = __builtin_fmaf(a, Sxx, __builtin_fmaf(b, Sxy, -(k1 * Sx))) - U * P1;
        f[4] = __builtin_fmaf(a, Sxy, __builtin_fmaf(b, Syy, -(k1 * Sy))) - V * P1;
        f[5] = c * __builtin_fmaf(V * V, S1, __builtin_fmaf(-2.f * V, Sy, Syy));
      } else {
        // rows 6, 7 in d[2], d[3] of lanes 24 + g; rows 8, 9 in d[0], d[1] of lanes 40 + g
        const bool hi = lane >= 40;
        v0f = hi ? s0 : s2;
        v1f = hi ? s1 : s3;
        i0 = hi ? 8 : 6;
      }
      if (!to_global) {
        float* dst = &acc[pos * kGradFields];
        if (is_e) {
#pragma unroll
          for (int k = 0; k < 6; k++) atomicAdd(dst + k, f[k]);
        } else {
          atomicAdd(dst + i0, v0f);
          atomicAdd(dst + i0 + 1, v1f);
        }
      } else {
        // global sums go through LDS so that each atomic instruction covers
        // whole Gaussians (ten consecutive floats)
        float* fg = Fg + l * kGradFields;
        if (is_e) {
#pragma unroll
          for (int k = 0; k < 6; k++) fg[k] = f[k];
          Fslot[l] = __float_as_uint(sg.misc.y);
        } else {
          fg[i0] = v0f;
          fg[i0 + 1] = v1f;
        }
      }
    }
    const uint64_t gmask = __builtin_amdgcn_ballot_w64(is_e && to_global);
    if (gmask != 0) {   // uniform
      wave_sync();
      for (int idx = lane; idx < count * kGradFields; idx += 64) {
        const int ge = idx / kGradFields, fi = idx - ge * kGradFields;
        if ((gmask >> ge) & 1u) {
          const float v = Fg[idx];
          if (v != 0.f) unsafeAtomicAdd(g2d + (int64_t)Fslot[ge] * kGradFields + fi, v);
        }
      }
    }
    wave_sync();   // the next columns overwrite Fg
  };
  PairWords<kBwdChunk> pw = load_pair_words<kBwdChunk>(
      pval, start + (Lmax > (uint32_t)kBwdChunk ? Lmax - kBwdChunk : 0u), (int)min(Lmax, (uint32_t)kBwdChunk), lane);
  for (uint32_t hi = Lmax; hi > 0;) {
    const uint32_t lo = hi > (uint32_t)kBwdChunk ? hi - kBwdChunk : 0u;
    const int nb = (int)(hi - lo);
    wave_sync();
    int packed;
    const int cnt = stage_chunk_padded<kBwdChunk>(rec, pw, rank_mask, lo, nb, X0, Y0, lane, my, kBwdStep, packed);
    wave_sync();
    if (lo > 0)   // uniform: the next (earlier) chunk's pair words, while this one is reduced
      pw = load_pair_words<kBwdChunk>(pval, start + (lo > (uint32_t)kBwdChunk ? lo - kBwdChunk : 0u),
                                      (int)min(lo, (uint32_t)kBwdChunk), lane);
    reduced += (uint32_t)packed;
    int rows = 0;   // uniform: entries with columns since the last product
    for (int top = cnt - 1; top >= 0; top -= kBwdStep) {   // cnt is a multiple of kBwdStep
      if (rows > kGrpF - kBwdStep) {   // room for a whole step of entries
        flush(rows);
        rows = 0;
      }
      float at[kBwdStep], alpha[kBwdStep], inv[kBwdStep], gcz[kBwdStep];
      bool acc_k[kBwdStep];
      int lo_slot = top - (kBwdStep - 1);
      __asm__ volatile("" : "+v"(lo_slot));
      const Staged* sp = my + lo_slot;
#pragma unroll
      for (int k = 0; k < kBwdStep; k++) {
        const Staged& sk = sp[kBwdStep - 1 - k];
        const float4 ge = sk.geo, cn = sk.conic, ap = sk.app;
        const float2 mi = make_float2(sk.misc.x, sk.misc.z);
        const float dx = (xf + ge.x) - ge.z;
        const float dy = (yf + ge.y) - ge.w;
        const float t1 = __builtin_fmaf(cn.x, dx, cn.y * dy);
        const float t2 = cn.z * dy;
        const float q = __builtin_fmaf(t1, t1, t2 * t2);
        acc_k[k] = __float_as_uint(mi.y) <= L && q <= cn.w;   // list position < last
        // a pixel that does not composite the entry takes alpha~ = 0: its
        // weight, its e and its share of the suffix sum are then exactly zero
        at[k] = acc_k[k] ? __builtin_amdgcn_exp2f(ap.x - q) : 0.f;
        alpha[k] = fminf(kAlphaMax, at[k]);
        inv[k] = __builtin_amdgcn_rcpf(1.f - alpha[k]);
        gcz[k] = __builtin_fmaf(G0, ap.z, __builtin_fmaf(G1, ap.w, __builtin_fmaf(G2, mi.x, GD * ap.y)));
      }
#pragma unroll
      for (int k = 0; k < kBwdStep; k++) {
        const float Tk = T * inv[k];
        const float w = alpha[k] * Tk;
        const float dalpha = __builtin_fmaf(Tk, gcz[k], -Rs * inv[k]);
        const float e = at[k] > kAlphaMax ? 0.f : dalpha * at[k];
        Rs = __builtin_fmaf(gcz[k], w, Rs);
        T = acc_k[k] ? Tk : T;
        if (__builtin_amdgcn_ballot_w64(acc_k[k]) != 0) {   // uniform
          A[rows * kRow + lane] = e;
          A[(kGrpF + rows) * kRow + lane] = w;
          rowent = writelane_u(top - k, rows, rowent);
          rows++;
        }
      }
    }
    if (rows > 0) flush(rows);
    hi = lo;
  }
  if (lane == 0) work_add(counters_rw, b * NW + wave, W_REDUCED, reduced);
  }
  if (kAcc > 0) {
    __syncthreads();
    const uint32_t start = trange[2 * bin_id];
    for (int i = tid; i < kAcc * kGradFields; i += 64 * NW) {
      const float v = acc[i];
      if (v != 0.f) {   // only rows of list entries some wave packed
        const int pos = i / kGradFields, fi = i - pos * kGradFields;
        const uint32_t r = pval[start + (uint32_t)pos] & rank_mask;
        unsafeAtomicAdd(g2d + (int64_t)r * kGradFields + fi, v);
      }
    }
  }
}

template <int TILE>
__global__ void __launch_bounds__(64 * (TILE / 8) * (TILE / 8), MS_BWDM_WAVES) k_composite_bwd_f(MS_BWD_KPARAMS) {
  bwd_f_tile<TILE>((int)blockIdx.x, MS_BWD_ARGS);
}

template <int TILE>
__global__ void __launch_bounds__(64 * (TILE / 8) * (TILE / 8), MS_BWDM_WAVES)
    k_composite_bwd_f_q(MS_BWD_KPARAMS, const TileQueue tq) {
  for_queued_tiles(tq, [&](int b) { bwd_f_tile<TILE>(b, MS_BWD_ARGS); });
}

template <int TILE>
hipError_t bwd_mfma32(const Plan& p, const JobTable& t, char* ws, hipStream_t st) {
  constexpr int threads = 64 * (TILE / 8) * (TILE / 8);
  hipLaunchKernelGGL((k_composite_bwd_f<TILE>), dim3(p.tiles), dim3(threads), 0, st, at<uint4>(ws, rec_slots(p)),
                     at<uint32_t>(ws, p.pval), rank_mask(p), at<uint32_t>(ws, p.trange), at<uint64_t>(ws, p.counters),
                     t, at<JobTable>(ws, p.jobs), p.bshift, at<float>(ws, p.tfinal), at<uint32_t>(ws, p.last),
                     at<float>(ws, p.g2d));
  return hipGetLastError();
}

template <int TILE>
hipError_t bwd_mfma(const Plan& p, const JobTable& t, char* ws, hipStream_t st) {
  constexpr int threads = 64 * (TILE / 8) * (TILE / 8);
  hipLaunchKernelGGL((k_composite_bwd_m<TILE>), dim3(p.tiles), dim3(threads), 0, st, at<uint4>(ws, rec_slots(p)),
                     at<uint32_t>(ws, p.pval), rank_mask(p), at<uint32_t>(ws, p.trange), at<uint64_t>(ws, p.counters),
                     t, at<JobTable>(ws, p.jobs), p.bshift, at<float>(ws, p.tfinal), at<uint32_t>(ws, p.last),
                     at<float>(ws, p.g2d));
  return hipGetLastError();
}

template <int TILE>
hipError_t bwd_scalar(const Plan& p, char* ws, hipStream_t st) {
  constexpr int threads = 64 * (TILE / 8) * (TILE / 8);
  hipLaunchKernelGGL((k_composite_bwd_s<TILE>), dim3(p.tiles), dim3(threads), 0, st, at<uint4>(ws, rec_slots(p)),
                     at<uint32_t>(ws, p.pval), rank_mask(p), at<uint32_t>(ws, p.trange), at<uint64_t>(ws, p.counters),
                     at<JobTable>(ws, p.jobs)->job, p.njobs, p.bshift, at<float>(ws, p.tfinal),
                     at<uint32_t>(ws, p.last), at<float>(ws, p.g2d));
  return hipGetLastError();
}

template <int TILE, int WB>
hipError_t fwd_one(const Plan& p, char* ws, hipStream_t st) {
  constexpr int threads = 64 * (TILE / 8) * (TILE / 8);
  hipLaunchKernelGGL((k_composite_fwd<TILE, WB>), dim3(p.tiles), dim3(threads), 0, st, at<uint4>(ws, rec_slots(p)),
                     at<uint32_t>(ws, p.pval), rank_mask(p), at<uint32_t>(ws, p.trange), at<uint64_t>(ws, p.counters),
                     at<JobTable>(ws, p.jobs)->job, p.njobs, p.bshift, at<float>(ws, p.tfinal),
                     at<uint32_t>(ws, p.last), at<uint32_t>(ws, p.wcost));
  return hipGetLastError();
}

// Workgroups of `kernel` (`threads` each) resident on the current device at
// once, at most `tiles`; 0 when the runtime cannot say.
int queue_grid(const void* kernel, int threads, int tiles) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess) return 0;
  const int64_t g = (int64_t)cus * per_cu;
  return (int)(g < tiles ? g : tiles);
}

// The queue of a persistent launch over the plan's tiles, sorted for the
// forward (nw = 0) or the backward (nw waves per tile).
hipError_t launch_order(const Plan& p, int nw, int nq, int grid, char* ws, hipStream_t st, TileQueue& tq) {
  hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(kOrderThreads), 0, st, at<uint32_t>(ws, p.trange),
                     at<uint32_t>(ws, p.wcost), nw, at<JobTable>(ws, p.jobs)->job, p.njobs, p.bshift, p.bins,
                     at<uint32_t>(ws, p.order), at<uint32_t>(ws, p.qctr));
  tq.order = at<uint32_t>(ws, p.order);
  tq.ctr = at<uint32_t>(ws, p.qctr);
  tq.n = p.tiles;
  tq.nq = nq;
  tq.grid = grid;
  return hipGetLastError();
}

template <int TILE, int WB>
hipError_t fwd_queue(const Plan& p, int nq, char* ws, hipStream_t st) {
  constexpr int threads = 64 * (TILE / 8) * (TILE / 8);
  const int grid = queue_grid(reinterpret_cast<const void*>(&k_composite_fwd_q<TILE, WB>), threads, p.tiles);
  if (grid <= 0) return hipErrorInvalidConfiguration;
  TileQueue tq;
  hipError_t e = launch_order(p, 0, nq, grid, ws, st, tq);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_composite_fwd_q<TILE, WB>), dim3(grid), dim3(threads), 0, st, at<uint4>(ws, rec_slots(p)),
                     at<uint32_t>(ws, p.pval), rank_mask(p), at<uint32_t>(ws, p.trange), at<uint64_t>(ws, p.counters),
                     at<JobTable>(ws, p.jobs)->job, p.njobs, p.bshift, at<float>(ws, p.tfinal),
                     at<uint32_t>(ws, p.last), at<uint32_t>(ws, p.wcost), tq);
  return hipGetLastError();
}

// The MFMA backward (fp32 or bf16x3 products) as a persistent launch.
template <int TILE, bool kBf16x3>
hipError_t bwd_queue(const Plan& p, int nq, const JobTable& t, char* ws, hipStream_t st) {
  constexpr int threads = 64 * (TILE / 8) * (TILE / 8);
  const void* k = kBf16x3 ? reinterpret_cast<const void*>(&k_composite_bwd_m_q<TILE>)
                          : reinterpret_cast<const void*>(&k_composite_bwd_f_q<TILE>);
  const int grid = queue_grid(k, threads, p.tiles);
  if (grid <= 0) return hipErrorInvalidConfiguration;
  TileQueue tq;
  hipError_t e = launch_order(p, (TILE / 8) * (TILE / 8), nq, grid, ws, st, tq);
  if (e != hipSuccess) return e;
  if (kBf16x3)
    hipLaunchKernelGGL((k_composite_bwd_m_q<TILE>), dim3(grid), dim3(threads), 0, st, at<uint4>(ws, rec_slots(p)),
                       at<uint32_t>(ws, p.pval), rank_mask(p), at<uint32_t>(ws, p.trange),
                       at<uint64_t>(ws, p.counters), t, at<JobTable>(ws, p.jobs), p.bshift, at<float>(ws, p.tfinal),
                       at<uint32_t>(ws, p.last), at<float>(ws, p.g2d), tq);
  else
    hipLaunchKernelGGL((k_composite_bwd_f_q<TILE>), dim3(grid), dim3(threads), 0, st, at<uint4>(ws, rec_slots(p)),
                       at<uint32_t>(ws, p.pval), rank_mask(p), at<uint32_t>(ws, p.trange),
                       at<uint64_t>(ws, p.counters), t, at<JobTable>(ws, p.jobs), p.bshift, at<float>(ws, p.tfinal),
                       at<uint32_t>(ws, p.last), at<float>(ws, p.g2d), tq);
  return hipGetLastError();
}

template <int TILE, int WB>
hipError_t bwd_one(const Plan& p, char* ws, hipStream_t st) {
  constexpr int threads = 64 * (TILE / 8) * (TILE / 8);
  hipLaunchKernelGGL((k_composite_bwd<TILE, WB>), dim3(p.tiles), dim3(threads), 0, st, at<uint4>(ws, rec_slots(p)),
                     at<uint32_t>(ws, p.pval), rank_mask(p), at<uint32_t>(ws, p.trange), at<uint64_t>(ws, p.counters),
                     at<JobTable>(ws, p.jobs)->job, p.njobs, p.bshift, at<float>(ws, p.tfinal),
                     at<uint32_t>(ws, p.last), at<float>(ws, p.g2d));
  return hipGetLastError();
}

template <int TILE>
hipError_t fwd_scalar(const Plan& p, char* ws, hipStream_t st) {
  constexpr int threads = 64 * (TILE / 8) * (TILE / 8);
  hipLaunchKernelGGL((k_composite_fwd_s<TILE>), dim3(p.tiles), dim3(threads), 0, st, at<uint4>(ws, rec_slots(p)),
                     at<uint32_t>(ws, p.pval), rank_mask(p), at<uint32_t>(ws, p.trange), at<uint64_t>(ws, p.counters),
                     at<JobTable>(ws, p.jobs)->job, p.njobs, p.bshift, at<float>(ws, p.tfinal),
                     at<uint32_t>(ws, p.last));
  return hipGetLastError();
}

}  // namespace

#define MS_DISPATCH(FN, ...)                                                            \
  switch (p.tile * 1000 + wave_batch) {                                                 \
    case 8032: return FN<8, 32>(__VA_ARGS__);                                           \
    case 8064: return FN<8, 64>(__VA_ARGS__);                                           \
    case 8128: return FN<8, 128>(__VA_ARGS__);                                          \
    case 16032: return FN<16, 32>(__VA_ARGS__);                                         \
    case 16064: return FN<16, 64>(__VA_ARGS__);                                         \
    case 16128: return FN<16, 128>(__VA_ARGS__);                                        \
    case 32032: return FN<32, 32>(__VA_ARGS__);                                         \
    case 32064: return FN<32, 64>(__VA_ARGS__);                                         \
    case 32128: return FN<32, 128>(__VA_ARGS__);                                        \
    default: return hipErrorInvalidValue;                                               \
  }

hipError_t launch_composite_fwd(const Plan& p, int wave_batch, uint32_t flags, char* ws, hipStream_t st) {
  if (p.tiles == 0) return hipSuccess;
  if (flags & MS_FLAG_SCALAR_FWD) {
    switch (p.tile) {
      case 8: return fwd_scalar<8>(p, ws, st);
      case 16: return fwd_scalar<16>(p, ws, st);
      case 32: return fwd_scalar<32>(p, ws, st);
      default: return hipErrorInvalidValue;
    }
  }
  if (flags & MS_FLAG_TILE_QUEUE) {
    const int nq = (flags & MS_FLAG_XCD_QUEUES) ? kMaxQueues : 1;
    MS_DISPATCH(fwd_queue, p, nq, ws, st)
  }
  MS_DISPATCH(fwd_one, p, ws, st)
}

hipError_t launch_composite_bwd(const Plan& p, int wave_batch, uint32_t flags, const JobTable& t, char* ws,
                                hipStream_t st) {
  if (p.tiles == 0) return hipSuccess;
  if ((flags & MS_FLAG_MFMA_BWD) && (flags & MS_FLAG_TILE_QUEUE)) {
    const int nq = (flags & MS_FLAG_XCD_QUEUES) ? kMaxQueues : 1;
    const bool x3 = (flags & MS_FLAG_BWD_BF16X3) != 0;
    switch (p.tile * 2 + (x3 ? 1 : 0)) {
      case 16: return bwd_queue<8, false>(p, nq, t, ws, st);
      case 17: return bwd_queue<8, true>(p, nq, t, ws, st);
      case 32: return bwd_queue<16, false>(p, nq, t, ws, st);
      case 33: return bwd_queue<16, true>(p, nq, t, ws, st);
      case 64: return bwd_queue<32, false>(p, nq, t, ws, st);
      case 65: return bwd_queue<32, true>(p, nq, t, ws, st);
      default: return hipErrorInvalidValue;
    }
  }
  if ((flags & MS_FLAG_MFMA_BWD) && (flags & MS_FLAG_BWD_BF16X3)) {
    switch (p.tile) {
      case 8: return bwd_mfma<8>(p, t, ws, st);
      case 16: return bwd_mfma<16>(p, t, ws, st);
      case 32: return bwd_mfma<32>(p, t, ws, st);
      default: return hipErrorInvalidValue;
    }
  }
  if (flags & MS_FLAG_MFMA_BWD) {
    switch (p.tile) {
      case 8: return bwd_mfma32<8>(p, t, ws, st);
      case 16: return bwd_mfma32<16>(p, t, ws, st);
      case 32: return bwd_mfma32<32>(p, t, ws, st);
      default: return hipErrorInvalidValue;
    }
  }
  if (flags & MS_FLAG_SCALAR_BWD) {
    switch (p.tile) {
      case 8: return bwd_scalar<8>(p, ws, st);
      case 16: return bwd_scalar<16>(p, ws, st);
      case 32: return bwd_scalar<32>(p, ws, st);
      default: return hipErrorInvalidValue;
    }
  }
  MS_DISPATCH(bwd_one, p, ws, st)
}

}  // namespace ms

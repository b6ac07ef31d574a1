// Generalized-ICP alignment of the consensus (Sec. 3.4 "3) Alignment", Eqs.
// 3-4; Sec. 3.5 "3) Alignment", Eq. 6): a rigid transform T = [R|t] taking
// source Gaussians (observed points, or another map's Gaussians) onto target
// (map) Gaussians, minimising
//   E(T) = sum_(k,l) r^T (R S_k R^T + S_l + eps I)^-1 r,   r = T x_k - y_l,
// over nearest-mean correspondences within d_max (0.02 m in the paper's
// experiments). Gauss-Newton on the left twist xi of T <- exp(xi^) T.
//
// Launches of one build and of each iteration:
//   build:   k_gicp_zero, k_gicp_count, k_gicp_bsum + block offsets +
//            k_gicp_bscan (bucket starts), k_gicp_fill -- a hashed uniform
//            grid of the target means, cells of d_max (1 + 2^-10), bucket
//            entries as float4 (x, y, z, target index);
//   iterate: k_gicp_correspond (per source, on eight lanes: the 27 neighbouring cells, the
//            nearest mean in the pinned binary32 distance, ties to the
//            smaller index), k_gicp_normal (per correspondence in binary64:
//            residual, (R S_k R^T + S_l + eps I)^-1, J = [I | -[T x]_x],
//            J^T M J and J^T M r; per-block partial sums), k_gicp_solve (one
//            workgroup: fixed-order parallel fold of the partials, Cholesky solve of
//            the 6x6 system, T <- exp(xi^) T, stored in binary32).
// The correspondence decision is an integer taken in binary32 in this
// order, without fused operations:
//   y_k = ((R_k0 x_0 + R_k1 x_1) + R_k2 x_2) + t_k,
//   d = y - mu (per component), d2 = (d_0 d_0 + d_1 d_1) + d_2 d_2 <= fl(d_max^2).
#include "ms_internal.h"

#pragma clang fp contract(off)

namespace ms {
namespace {

constexpr int kGThreads = 256;
constexpr int kBucketBlock = 1024;   // buckets per scan block

__device__ inline uint32_t cell_hash(int64_t ix, int64_t iy, int64_t iz, uint32_t mask) {
  const uint32_t h = ((uint32_t)ix * 73856093u) ^ ((uint32_t)iy * 19349663u) ^ ((uint32_t)iz * 83492791u);
  return h & mask;
}

__device__ inline int64_t cell_of(float v, double inv_cell) { return (int64_t)floor((double)v * inv_cell); }

__device__ inline bool finite3(float a, float b, float c) {
  return __builtin_isfinite(a) && __builtin_isfinite(b) && __builtin_isfinite(c);
}

__global__ void k_gicp_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_gicp_zero(uint32_t* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0u;
}

// target k of the (optionally indexed) set: map index and mean
__device__ inline int64_t target_index(const int32_t* __restrict__ idx, int64_t k) { return idx ? (int64_t)idx[k] : k; }

__global__ void __launch_bounds__(kGThreads) k_gicp_count(const float* __restrict__ mu, int64_t n, const int32_t* __restrict__ idx,
                                                          int64_t m, double inv_cell, uint32_t mask, uint32_t* __restrict__ bcount) {
  const int64_t k = (int64_t)blockIdx.x * kGThreads + threadIdx.x;
  if (k >= m) return;
  const int64_t j = target_index(idx, k);
  if (j < 0 || j >= n) return;   // an index outside the map takes no part
  const float x = mu[j], y = mu[n + j], z = mu[2 * n + j];
  if (!finite3(x, y, z)) return;
  atomicAdd(&bcount[cell_hash(cell_of(x, inv_cell), cell_of(y, inv_cell), cell_of(z, inv_cell), mask)], 1u);
}

// sums of each block of kBucketBlock buckets
__global__ void __launch_bounds__(kGThreads) k_gicp_bsum(const uint32_t* __restrict__ bcount, uint32_t* __restrict__ bsum) {
  __shared__ uint32_t red[kGThreads / 64];
  const int t = threadIdx.x;
  uint32_t s = 0;
  for (int i = t; i < kBucketBlock; i += kGThreads) s += bcount[(int64_t)blockIdx.x * kBucketBlock + i];
  for (int off = 32; off > 0; off >>= 1) s += (uint32_t)__shfl_xor((int)s, off, 64);
  if ((t & 63) == 0) red[t >> 6] = s;
  __syncthreads();
  if (t == 0) bsum[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// bucket starts: exclusive scan inside each block plus the block's offset
__global__ void __launch_bounds__(kBucketBlock) k_gicp_bscan(const uint32_t* __restrict__ bcount, const uint32_t* __restrict__ boff,
                                                             uint32_t* __restrict__ bstart, int64_t nbuckets, const int64_t* __restrict__ total) {
  __shared__ uint32_t ws[kBucketBlock / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t b = (int64_t)blockIdx.x * kBucketBlock + t;
  const uint32_t v = bcount[b];
  uint32_t inc = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)inc, off, 64);
    if (lane >= off) inc += y;
  }
  if (lane == 63) ws[wave] = inc;
  __syncthreads();
  uint32_t before = boff[blockIdx.x];
  for (int w = 0; w < wave; w++) before += ws[w];
  bstart[b] = before + inc - v;
  if (b == nbuckets - 1) bstart[nbuckets] = (uint32_t)*total;
}

__global__ void __launch_bounds__(kGThreads) k_gicp_fill(const float* __restrict__ mu, int64_t n, const int32_t* __restrict__ idx,
                                                         int64_t m, double inv_cell, uint32_t mask, const uint32_t* __restrict__ bstart,
                                                         uint32_t* __restrict__ fillpos, float4* __restrict__ entries,
                                                         int2* __restrict__ eslot) {
  const int64_t k = (int64_t)blockIdx.x * kGThreads + threadIdx.x;
  if (k >= m) return;
  const int64_t j = target_index(idx, k);
  if (j < 0 || j >= n) return;
  const float x = mu[j], y = mu[n + j], z = mu[2 * n + j];
  if (!finite3(x, y, z)) return;
  const uint32_t b = cell_hash(cell_of(x, inv_cell), cell_of(y, inv_cell), cell_of(z, inv_cell), mask);
  const uint32_t slot = bstart[b] + atomicAdd(&fillpos[b], 1u);
  entries[slot] = make_float4(x, y, z, __int_as_float((int32_t)j));
  eslot[k] = make_int2((int32_t)slot, (int32_t)j);   // the entry of listed target k (-1 where none)
}

struct Pose32 {
  float r[12];
};

__device__ inline Pose32 load_pose32(const float* __restrict__ T) {
  Pose32 P;
#pragma unroll
  for (int k = 0; k < 12; k++) P.r[k] = T[k];
  return P;
}

// Eight lanes per source, each probing every eighth of the 27 neighbouring
// cells; their nearest candidates meet by a butterfly. The order on
// (distance, index) is total, so the nearest is the same whatever lane
// finds it.
constexpr int kProbeLanes = 8;

__device__ inline bool closer(float dd, int32_t j, float bd, int32_t best) {
  return j >= 0 && (best < 0 || dd < bd || (dd == bd && j < best));
}

__global__ void __launch_bounds__(kGThreads) k_gicp_correspond(const float* __restrict__ src, int64_t n, const float* __restrict__ T,
                                                               double inv_cell, uint32_t mask, const uint32_t* __restrict__ bstart,
                                                               const float4* __restrict__ entries, float dmax2,
                                                               int32_t* __restrict__ corr, int32_t* __restrict__ cslot) {
  const int64_t g = (int64_t)blockIdx.x * kGThreads + threadIdx.x;
  const int64_t k = g / kProbeLanes;
  const int sub = (int)(g % kProbeLanes);
  const bool live = k < n;   // the lanes of one source are all live or all not (kGThreads % kProbeLanes == 0)
  int32_t best = -1, bslot = -1;   // target index and grid entry of the nearest mean
  float bd = 0.f;
  if (live) {
    const Pose32 P = load_pose32(T);
    const float x0 = src[k], x1 = src[n + k], x2 = src[2 * n + k];
    const float y0 = ((P.r[0] * x0 + P.r[1] * x1) + P.r[2] * x2) + P.r[3];
    const float y1 = ((P.r[4] * x0 + P.r[5] * x1) + P.r[6] * x2) + P.r[7];
    const float y2 = ((P.r[8] * x0 + P.r[9] * x1) + P.r[10] * x2) + P.r[11];
    if (finite3(y0, y1, y2)) {
      const int64_t cx = cell_of(y0, inv_cell), cy = cell_of(y1, inv_cell), cz = cell_of(y2, inv_cell);
      // the bucket ranges of this lane's cells, loaded together
      constexpr int kCells = (27 + kProbeLanes - 1) / kProbeLanes;
      uint32_t bs[kCells], be[kCells];
#pragma unroll
      for (int u = 0; u < kCells; u++) {
        const int c = sub + u * kProbeLanes;
        bs[u] = be[u] = 0u;
        if (c < 27) {
          const uint32_t b = cell_hash(cx + (c % 3 - 1), cy + ((c / 3) % 3 - 1), cz + (c / 9 - 1), mask);
          bs[u] = bstart[b];
          be[u] = bstart[b + 1];
        }
      }
      auto test = [&](const float4& q, uint32_t s) {
        const float d0 = y0 - q.x, d1 = y1 - q.y, d2 = y2 - q.z;
        const float dd = (d0 * d0 + d1 * d1) + d2 * d2;
        const int32_t j = __float_as_int(q.w);
        if (dd <= dmax2 && closer(dd, j, bd, best)) {
          best = j;
          bslot = (int32_t)s;
          bd = dd;
        }
      };
#pragma unroll
      for (int u = 0; u < kCells; u++) {
        uint32_t s = bs[u];
        for (; s + 1 < be[u]; s += 2) {   // two entries in flight
          const float4 qa = entries[s], qb = entries[s + 1];
          test(qa, s);
          test(qb, s + 1);
        }
        if (s < be[u]) test(entries[s], s);
      }
    }
  }
#pragma unroll
  for (int off = 1; off < kProbeLanes; off <<= 1) {
    const float od = __shfl_xor(bd, off, 64);
    const int32_t oj = __shfl_xor(best, off, 64);
    const int32_t os = __shfl_xor(bslot, off, 64);
    if (closer(od, oj, bd, best)) {
      best = oj;
      bslot = os;
      bd = od;
    }
  }
  if (live && sub == 0) {
    corr[k] = best;
    if (cslot) cslot[k] = bslot;
  }
}

// covariance R_q diag(s^2) R_q^T of Gaussian j in binary64 (upper triangle
// xx, xy, xz, yy, yz, zz), or zero without scales
__device__ inline void gauss_cov(const float* __restrict__ sc, const float* __restrict__ qt, int64_t n, int64_t j, double c[6]) {
  if (!sc) {
    for (int i = 0; i < 6; i++) c[i] = 0.0;
    return;
  }
  double w = qt[j], x = qt[n + j], y = qt[2 * n + j], z = qt[3 * n + j];
  const double r = 1.0 / sqrt(((w * w + x * x) + y * y) + z * z);
  w *= r, x *= r, y *= r, z *= r;
  const double R[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                          {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                          {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
  const double s0 = sc[j], s1 = sc[n + j], s2 = sc[2 * n + j];
  const double v[3] = {s0 * s0, s1 * s1, s2 * s2};
  int o = 0;
  for (int a = 0; a < 3; a++)
    for (int b = a; b < 3; b++) c[o++] = (R[a][0] * v[0] * R[b][0] + R[a][1] * v[1] * R[b][1]) + R[a][2] * v[2] * R[b][2];
}

constexpr int kSums = 29;   // H upper triangle (21), g (6), cost, count

// A target as the normal equations read it, one record per grid entry (64
// bytes, half a line): its binary64 covariance, its mean and its map index
// (-1 when the index lies outside the map given to the alignment, which
// then takes no part, as a correspondence outside the target map does).
struct TargetRec {
  double cov[6];
  float mu[3];
  int32_t idx;
};
static_assert(sizeof(TargetRec) == 64, "one target record per half line");

// The records of the grid's entries from the target map tgt: the same
// covariance (gauss_cov) and mean the normal equations would read at the map
// index, computed once per alignment instead of once per correspondence and
// iteration. Thread k takes the k-th listed target (map order, or the order
// of the index list), so that its reads of the map's planes are coalesced;
// eslot[k] holds its entry and map index, or -1.
__global__ void __launch_bounds__(kGThreads) k_gicp_records(const int2* __restrict__ eslot, int64_t count,
                                                            const float* __restrict__ tgt, const float* __restrict__ tsc,
                                                            const float* __restrict__ tqt, int64_t nt,
                                                            TargetRec* __restrict__ rec) {
  const int64_t k = (int64_t)blockIdx.x * kGThreads + threadIdx.x;
  if (k >= count) return;
  const int2 e = eslot[k];
  if (e.x < 0) return;
  const int64_t s = e.x;
  const int32_t l = e.y;
  TargetRec r;
  if (l >= 0 && l < nt) {
    gauss_cov(tsc, tqt, nt, l, r.cov);
    r.mu[0] = tgt[l];
    r.mu[1] = tgt[nt + l];
    r.mu[2] = tgt[2 * nt + l];
    r.idx = l;
  } else {
    for (int i = 0; i < 6; i++) r.cov[i] = 0.0;
    r.mu[0] = r.mu[1] = r.mu[2] = 0.f;
    r.idx = -1;
  }
  rec[s] = r;
}

__device__ inline double wave_sum_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// kRec: the target of source k is the grid entry cslot[k] (its record);
// otherwise the map index corr[k], read from the target map.
template <bool kRec>
__global__ void __launch_bounds__(kGThreads) k_gicp_normal(const float* __restrict__ src, const float* __restrict__ ssc,
                                                           const float* __restrict__ sqt, int64_t n, const float* __restrict__ tgt,
                                                           const float* __restrict__ tsc, const float* __restrict__ tqt, int64_t nt,
                                                           const float* __restrict__ T, const int32_t* __restrict__ corr,
                                                           const TargetRec* __restrict__ rec, double eps,
                                                           double* __restrict__ partial) {
  __shared__ double red[kGThreads / 64][kSums];
  const int64_t k = (int64_t)blockIdx.x * kGThreads + threadIdx.x;
  double acc[kSums];
#pragma unroll
  for (int i = 0; i < kSums; i++) acc[i] = 0.0;
  const int32_t l = k < n ? corr[k] : -1;
  double ct[6], tm[3];
  bool valid;
  if (kRec) {
    valid = l >= 0;
    if (valid) {
      const TargetRec& q = rec[l];
      valid = q.idx >= 0;
      for (int i = 0; i < 6; i++) ct[i] = q.cov[i];
      for (int i = 0; i < 3; i++) tm[i] = q.mu[i];
    }
  } else {
    valid = l >= 0 && l < nt;   // a correspondence outside the target map takes no part
    if (valid) {
      gauss_cov(tsc, tqt, nt, l, ct);
      for (int i = 0; i < 3; i++) tm[i] = tgt[i * nt + l];
    }
  }
  if (valid) {
    double V[12];
#pragma unroll
    for (int i = 0; i < 12; i++) V[i] = (double)T[i];
    const double x0 = src[k], x1 = src[n + k], x2 = src[2 * n + k];
    const double p[3] = {((V[0] * x0 + V[1] * x1) + V[2] * x2) + V[3], ((V[4] * x0 + V[5] * x1) + V[6] * x2) + V[7],
                         ((V[8] * x0 + V[9] * x1) + V[10] * x2) + V[11]};
    const double r[3] = {p[0] - tm[0], p[1] - tm[1], p[2] - tm[2]};
    double cs[6];
    gauss_cov(ssc, sqt, n, k, cs);
    // C = R S_k R^T + S_l + eps I
    const double S[3][3] = {{cs[0], cs[1], cs[2]}, {cs[1], cs[3], cs[4]}, {cs[2], cs[4], cs[5]}};
    double RS[3][3];
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) RS[a][b] = (V[4 * a] * S[0][b] + V[4 * a + 1] * S[1][b]) + V[4 * a + 2] * S[2][b];
    double C[3][3];
    int o = 0;
    for (int a = 0; a < 3; a++)
      for (int b = a; b < 3; b++) {
        const double rsr = (RS[a][0] * V[4 * b] + RS[a][1] * V[4 * b + 1]) + RS[a][2] * V[4 * b + 2];
        C[a][b] = C[b][a] = rsr + ct[o++] + (a == b ? eps : 0.0);
      }
    // M = C^-1 by cofactors
    const double c00 = C[1][1] * C[2][2] - C[1][2] * C[2][1], c01 = C[1][2] * C[2][0] - C[1][0] * C[2][2],
                 c02 = C[1][0] * C[2][1] - C[1][1] * C[2][0];
    const double det = (C[0][0] * c00 + C[0][1] * c01) + C[0][2] * c02;
    const double id = 1.0 / det;
    const double M00 = c00 * id, M01 = c01 * id, M02 = c02 * id;
    const double M11 = (C[0][0] * C[2][2] - C[0][2] * C[2][0]) * id;
    const double M12 = (C[0][2] * C[1][0] - C[0][0] * C[1][2]) * id;
    const double M22 = (C[0][0] * C[1][1] - C[0][1] * C[1][0]) * id;
    const double M[3][3] = {{M00, M01, M02}, {M01, M11, M12}, {M02, M12, M22}};
    // J = [I | -[p]_x]: column c of J (3 entries)
    double J[3][6];
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) J[a][b] = a == b ? 1.0 : 0.0;
    J[0][3] = 0.0, J[0][4] = p[2], J[0][5] = -p[1];
    J[1][3] = -p[2], J[1][4] = 0.0, J[1][5] = p[0];
    J[2][3] = p[1], J[2][4] = -p[0], J[2][5] = 0.0;
    double MJ[3][6], Mr[3];
    for (int a = 0; a < 3; a++) {
      for (int c = 0; c < 6; c++) MJ[a][c] = (M[a][0] * J[0][c] + M[a][1] * J[1][c]) + M[a][2] * J[2][c];
      Mr[a] = (M[a][0] * r[0] + M[a][1] * r[1]) + M[a][2] * r[2];
    }
    o = 0;
    for (int c = 0; c < 6; c++)
      for (int d = c; d < 6; d++) acc[o++] = (J[0][c] * MJ[0][d] + J[1][c] * MJ[1][d]) + J[2][c] * MJ[2][d];
    for (int c = 0; c < 6; c++) acc[21 + c] = (J[0][c] * Mr[0] + J[1][c] * Mr[1]) + J[2][c] * Mr[2];
    acc[27] = (r[0] * Mr[0] + r[1] * Mr[1]) + r[2] * Mr[2];
    acc[28] = 1.0;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < kSums; i++) {
    const double s = wave_sum_d(acc[i]);
    if (lane == 0) red[wave][i] = s;
  }
  __syncthreads();
  if (threadIdx.x < kSums) {
    const int i = threadIdx.x;
    partial[(int64_t)blockIdx.x * 32 + i] = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
  }
}

// One workgroup: fold the partials in a fixed order, solve, update T.
__global__ void __launch_bounds__(kGThreads) k_gicp_solve(const double* __restrict__ partial, int64_t nblocks, float* __restrict__ T,
                                                          double* __restrict__ out, double* __restrict__ hist) {
  // fixed-order fold of the partials: thread t sums blocks t, t + 256, ...;
  // each wave folds its lanes by a butterfly; the waves are added in order
  __shared__ double wsum[kGThreads / 64][32];
  __shared__ double tot[32];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  double acc[kSums];
#pragma unroll
  for (int i = 0; i < kSums; i++) acc[i] = 0.0;
  for (int64_t b = t; b < nblocks; b += kGThreads)
#pragma unroll
    for (int i = 0; i < kSums; i++) acc[i] += partial[b * 32 + i];
#pragma unroll
  for (int i = 0; i < kSums; i++) {
    double v = acc[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) wsum[wave][i] = v;
  }
  __syncthreads();
  if (t < kSums) {
    double s = 0.0;
    for (int w = 0; w < kGThreads / 64; w++) s += wsum[w][t];
    tot[t] = s;
  }
  __syncthreads();
  if (t != 0) return;
  for (int i = 0; i < kSums; i++) {
    out[i] = tot[i];
    if (hist) hist[i] = tot[i];
  }
  if (!T || tot[28] < 6.0) return;   // sums only, or too few correspondences: T stays
  double H[6][6], g[6];
  int o = 0;
  for (int c = 0; c < 6; c++)
    for (int d = c; d < 6; d++) H[c][d] = H[d][c] = tot[o++];
  for (int c = 0; c < 6; c++) g[c] = tot[21 + c];
  double tr = 0.0;
  for (int c = 0; c < 6; c++) tr += H[c][c];
  const double lam = 1e-12 * tr / 6.0;
  for (int c = 0; c < 6; c++) H[c][c] += lam;
  // Cholesky H = L L^T, then xi = -H^-1 g
  double L[6][6] = {};
  for (int i = 0; i < 6; i++)
    for (int j = 0; j <= i; j++) {
      double s = H[i][j];
      for (int k = 0; k < j; k++) s -= L[i][k] * L[j][k];
      if (i == j) {
        if (!(s > 0.0)) return;   // not positive definite: T stays
        L[i][i] = sqrt(s);
      } else {
        L[i][j] = s / L[j][j];
      }
    }
  double z[6], xi[6];
  for (int i = 0; i < 6; i++) {
    double s = -g[i];
    for (int k = 0; k < i; k++) s -= L[i][k] * z[k];
    z[i] = s / L[i][i];
  }
  for (int i = 5; i >= 0; i--) {
    double s = z[i];
    for (int k = i + 1; k < 6; k++) s -= L[k][i] * xi[k];
    xi[i] = s / L[i][i];
  }
  // exp of the twist (rho, phi), closed form
  const double px = xi[3], py = xi[4], pz = xi[5];
  const double th2 = px * px + py * py + pz * pz, th = sqrt(th2);
  double A, B, Cc;
  if (th < 1e-12) {
    A = 1.0, B = 0.5, Cc = 1.0 / 6.0;
  } else {
    A = sin(th) / th;
    B = (1.0 - cos(th)) / th2;
    Cc = (th - sin(th)) / (th2 * th);
  }
  const double K[3][3] = {{0, -pz, py}, {pz, 0, -px}, {-py, px, 0}};
  double K2[3][3], Rx[3][3], Vm[3][3];
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) K2[a][b] = K[a][0] * K[0][b] + K[a][1] * K[1][b] + K[a][2] * K[2][b];
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      const double I = a == b ? 1.0 : 0.0;
      Rx[a][b] = I + A * K[a][b] + B * K2[a][b];
      Vm[a][b] = I + B * K[a][b] + Cc * K2[a][b];
    }
  const double tx[3] = {Vm[0][0] * xi[0] + Vm[0][1] * xi[1] + Vm[0][2] * xi[2],
                        Vm[1][0] * xi[0] + Vm[1][1] * xi[1] + Vm[1][2] * xi[2],
                        Vm[2][0] * xi[0] + Vm[2][1] * xi[1] + Vm[2][2] * xi[2]};
  double V[12];
  for (int i = 0; i < 12; i++) V[i] = (double)T[i];
  float Tn[12];
  for (int a = 0; a < 3; a++) {
    for (int b = 0; b < 3; b++) Tn[4 * a + b] = (float)(Rx[a][0] * V[b] + Rx[a][1] * V[4 + b] + Rx[a][2] * V[8 + b]);
    Tn[4 * a + 3] = (float)(Rx[a][0] * V[3] + Rx[a][1] * V[7] + Rx[a][2] * V[11] + tx[a]);
  }
  for (int i = 0; i < 12; i++) T[i] = Tn[i];
}

}  // namespace

GicpPlan gicp_plan(int64_t max_src, int64_t max_tgt, float d_max) {
  GicpPlan p;
  int64_t M = kBucketBlock;
  while (M < 2 * max_tgt) M <<= 1;
  p.nbuckets = M;
  p.max_src = max_src;
  p.max_tgt = max_tgt;
  p.cell = (double)d_max * (1.0 + 1.0 / 1024.0);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += (bytes + 255) / 256 * 256;
    return at;
  };
  p.bcount = take((size_t)M * 4);
  p.fillpos = take((size_t)M * 4);
  p.bstart = take((size_t)(M + 1) * 4);
  p.bsum = take((size_t)(M / kBucketBlock) * 4);
  p.total = take(8);
  p.entries = take((size_t)(max_tgt > 0 ? max_tgt : 1) * 16);
  p.corr = take((size_t)(max_src > 0 ? max_src : 1) * 4);
  p.cslot = take((size_t)(max_src > 0 ? max_src : 1) * 4);
  p.rec = take((size_t)(max_tgt > 0 ? max_tgt : 1) * sizeof(TargetRec));
  p.eslot = take((size_t)(max_tgt > 0 ? max_tgt : 1) * 8);
  p.nblocks = (max_src + kGThreads - 1) / kGThreads;
  p.partial = take((size_t)(p.nblocks > 0 ? p.nblocks : 1) * 32 * 8);
  p.out = take(32 * 8);
  p.bytes = o;
  return p;
}

hipError_t gicp_build(const GicpPlan& p, const float* mu, int64_t n, const int32_t* idx, int64_t m, char* ws,
                      hipStream_t st) {
  uint32_t* bcount = at<uint32_t>(ws, p.bcount);
  uint32_t* fillpos = at<uint32_t>(ws, p.fillpos);
  const uint32_t mask = (uint32_t)(p.nbuckets - 1);
  const double inv = 1.0 / p.cell;
  hipLaunchKernelGGL(k_gicp_zero, dim3(1024), dim3(256), 0, st, bcount, p.nbuckets);
  hipLaunchKernelGGL(k_gicp_zero, dim3(1024), dim3(256), 0, st, fillpos, p.nbuckets);
  // every listed target's entry starts as none (-1 in both words)
  hipLaunchKernelGGL(k_gicp_fill_u32, dim3(1024), dim3(256), 0, st, at<uint32_t>(ws, p.eslot), 2 * p.max_tgt, 0xFFFFFFFFu);
  const unsigned tb = (unsigned)((m + kGThreads - 1) / kGThreads);
  if (m > 0) hipLaunchKernelGGL(k_gicp_count, dim3(tb), dim3(kGThreads), 0, st, mu, n, idx, m, inv, mask, bcount);
  const int64_t nb = p.nbuckets / kBucketBlock;
  hipLaunchKernelGGL(k_gicp_bsum, dim3((unsigned)nb), dim3(kGThreads), 0, st, bcount, at<uint32_t>(ws, p.bsum));
  hipError_t e = launch_block_offsets(at<uint32_t>(ws, p.bsum), nb, at<int64_t>(ws, p.total), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gicp_bscan, dim3((unsigned)nb), dim3(kBucketBlock), 0, st, bcount, at<uint32_t>(ws, p.bsum),
                     at<uint32_t>(ws, p.bstart), p.nbuckets, at<int64_t>(ws, p.total));
  if (m > 0)
    hipLaunchKernelGGL(k_gicp_fill, dim3(tb), dim3(kGThreads), 0, st, mu, n, idx, m, inv, mask, at<uint32_t>(ws, p.bstart),
                       fillpos, at<float4>(ws, p.entries), at<int2>(ws, p.eslot));
  return hipGetLastError();
}

hipError_t gicp_correspond(const GicpPlan& p, const float* src, int64_t n, const float* T, float d_max,
                           int32_t* corr, int32_t* cslot, char* ws, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const float dmax2 = d_max * d_max;
  static_assert(kGThreads % kProbeLanes == 0, "a source's lanes share one workgroup");
  hipLaunchKernelGGL(k_gicp_correspond, dim3((unsigned)((n * kProbeLanes + kGThreads - 1) / kGThreads)), dim3(kGThreads), 0, st, src, n, T,
                     1.0 / p.cell, (uint32_t)(p.nbuckets - 1), at<uint32_t>(ws, p.bstart), at<float4>(ws, p.entries), dmax2,
                     corr, cslot);
  return hipGetLastError();
}

hipError_t gicp_normal(const GicpPlan& p, const ms_map& src, const ms_map& tgt, const float* T, const int32_t* corr,
                       float eps, char* ws, hipStream_t st) {
  const int64_t nb = (src.n + kGThreads - 1) / kGThreads;
  if (nb > 0)
    hipLaunchKernelGGL(k_gicp_normal<false>, dim3((unsigned)nb), dim3(kGThreads), 0, st, src.means, src.scales, src.quats,
                       src.n, tgt.means, tgt.scales, tgt.quats, tgt.n, T, corr, (const TargetRec*)nullptr, (double)eps,
                       at<double>(ws, p.partial));
  return hipGetLastError();
}

hipError_t gicp_records(const GicpPlan& p, const ms_map& tgt, char* ws, hipStream_t st) {
  if (p.max_tgt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gicp_records, dim3((unsigned)((p.max_tgt + kGThreads - 1) / kGThreads)), dim3(kGThreads), 0, st,
                     at<int2>(ws, p.eslot), p.max_tgt, tgt.means, tgt.scales, tgt.quats, tgt.n, at<TargetRec>(ws, p.rec));
  return hipGetLastError();
}

hipError_t gicp_normal_records(const GicpPlan& p, const ms_map& src, const float* T, float eps, char* ws,
                               hipStream_t st) {
  const int64_t nb = (src.n + kGThreads - 1) / kGThreads;
  if (nb > 0)
    hipLaunchKernelGGL(k_gicp_normal<true>, dim3((unsigned)nb), dim3(kGThreads), 0, st, src.means, src.scales, src.quats,
                       src.n, (const float*)nullptr, (const float*)nullptr, (const float*)nullptr, (int64_t)0, T,
                       at<int32_t>(ws, p.cslot), at<TargetRec>(ws, p.rec), (double)eps, at<double>(ws, p.partial));
  return hipGetLastError();
}

hipError_t gicp_solve(const GicpPlan& p, int64_t n_src, float* T, double* out, double* hist, char* ws, hipStream_t st,
                      bool update) {
  const int64_t nb = (n_src + kGThreads - 1) / kGThreads;
  hipLaunchKernelGGL(k_gicp_solve, dim3(1), dim3(kGThreads), 0, st, at<double>(ws, p.partial), nb, update ? T : nullptr,
                     out, hist);
  return hipGetLastError();
}

}  // namespace ms

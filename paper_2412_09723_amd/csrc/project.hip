// Projection of 3D Gaussians to screen-space records (forward) and the chain
// rule back to the Gaussian parameters and the camera pose (backward).
//
// Forward: one thread per Gaussian, coalesced structure-of-arrays loads. The
// discrete structure (visibility, pixel box, depth key, per-pixel acceptance
// constants) follows the pinned binary64 recipe stated in macsplat.h; it is
// evaluated here with contraction disabled so that every product and sum is
// an individually rounded IEEE operation. The per-Gaussian setup is cheap next
// to compositing, so binary64 costs nothing measurable and keeps the conic
// factors accurate for elongated splats.
//
// Backward: one thread per Gaussian; binary64 chain rule through the
// Cholesky factors of the conic, Sigma' = V V^T + 0.3 I with V = J R M, and
// the quaternion normalisation; per-block binary64 reduction of the pose
// partials, then one block folds them in a fixed order (deterministic).
#include "ms_internal.h"

#pragma clang fp contract(off)

namespace ms {
namespace {

__device__ inline double pinned_log2(double x) {
  int e;
  double m = frexp(x, &e);
  m = m * 2.0;
  e = e - 1;
  if (m > 1.4142135623730951) {
    m = m * 0.5;
    e = e + 1;
  }
  double y = (m - 1.0) / (m + 1.0);
  double y2 = y * y;
  double P = 1.0 / 23.0;
  for (int k = 10; k >= 0; k--) P = P * y2 + 1.0 / (double)(2 * k + 1);
  return (double)e + (2.0 * y * P) * kLog2e;
}

__device__ inline double dmin(double a, double b) { return (b < a) ? b : a; }
__device__ inline double dmax(double a, double b) { return (a < b) ? b : a; }

struct Pose {
  double R[3][3], t[3];
};

template <class PtrT>
__device__ inline void load_pose(PtrT vm, Pose& P) {
#pragma unroll
  for (int i = 0; i < 3; i++) {
#pragma unroll
    for (int j = 0; j < 3; j++) P.R[i][j] = (double)vm[4 * i + j];
    P.t[i] = (double)vm[4 * i + 3];
  }
}

// One block of 256 virtual slots belongs to one job; slots past the job's n
// are padding and stay invisible. Outputs per slot: the depth key and the
// record (index order), and for the binning path in use either the bin
// footprint `gbin` plus a zeroed accumulator row (per-bin path) or the
// visibility flag, bin count and rank placeholder (global sort path); the
// pointers of the other path are null.
// The first kernel of a forward pass: it also writes the job table (passed
// by value) into the workspace for the kernels after it, and zeroes `zcount`
// words at `zero` (the control region), which no projection block reads.
__global__ void __launch_bounds__(256) k_project_fwd(const JobTable tbl, JobTable* __restrict__ tbl_dst,
                                                     uint32_t* __restrict__ zero, int64_t zcount, float near_z,
                                                     int tile, uint32_t* __restrict__ key,
                                                     uint32_t* __restrict__ vis, uint32_t* __restrict__ ntiles,
                                                     int32_t* __restrict__ rank_of, uint4* __restrict__ rec_i,
                                                     uint2* __restrict__ gbin, float* __restrict__ g2d) {
  __shared__ int s_list[256];
  __shared__ int s_wcnt[256 / 64];
  const JobDesc* jobs = tbl.job;
  const int njobs = tbl.njobs;
  if (blockIdx.x == 0) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&tbl);
    uint32_t* d = reinterpret_cast<uint32_t*>(tbl_dst);
    for (int i = threadIdx.x; i < (int)(sizeof(JobTable) / 4); i += 256) d[i] = src[i];
  }
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < zcount; j += (int64_t)gridDim.x * 256) zero[j] = 0u;
  const JobDesc& J = jobs[job_of_block(jobs, njobs, (int)blockIdx.x)];
  const int64_t n = J.n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  auto set_culled = [&](int64_t iv) {
    key[iv] = 0xFFFFFFFFu;
    if (gbin) {
      gbin[iv] = make_uint2(kNoBin, 0u);
    } else {
      vis[iv] = 0u;
      ntiles[iv] = 0u;
      rank_of[iv] = -1;
    }
  };
  // The Gaussians in front of the near plane are packed onto the block's
  // first threads, so the binary64 projection runs on as few waves as there
  // are such Gaussians. The owner of any other slot marks it culled.
  const int64_t li0 = (int64_t)((int)blockIdx.x - J.block0) * 256;   // block's first index within the job
  const int64_t li_own = li0 + threadIdx.x;
  bool front = false;
  if (li_own < n) {
    Pose P0;
    load_pose(J.viewmat, P0);
    const double m0 = J.means[li_own], m1 = J.means[n + li_own], m2 = J.means[2 * n + li_own];
    double pz[3];
#pragma unroll
    for (int r = 0; r < 3; r++) pz[r] = ((P0.R[r][0] * m0 + P0.R[r][1] * m1) + P0.R[r][2] * m2) + P0.t[r];
    front = pz[2] > (double)near_z && isfinite(pz[0]) && isfinite(pz[1]) && isfinite(pz[2]);
  }
  if (!front) set_culled(J.g0 + li_own);
  const uint64_t fm = __ballot(front);
  if (lane == 0) s_wcnt[wave] = __popcll(fm);
  __syncthreads();
  int fbase = 0, nfront = 0;
  for (int w = 0; w < 256 / 64; w++) {
    if (w < wave) fbase += s_wcnt[w];
    nfront += s_wcnt[w];
  }
  if (front)
    s_list[fbase + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(fm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)fm, 0u))] =
        (int)threadIdx.x;
  __syncthreads();
  if ((int)threadIdx.x >= nfront) return;
  const int64_t li = li0 + s_list[threadIdx.x];   // index within the job
  const int64_t i = J.g0 + li;                     // virtual index
  set_culled(i);   // until the projection below accepts it
  const float* __restrict__ means = J.means;
  const float* __restrict__ scales = J.scales;
  const float* __restrict__ quats = J.quats;
  const float* __restrict__ opac = J.opacity;
  const float* __restrict__ colors = J.colors;
  struct {
    int W, H;
    float fx, fy, cx, cy, near_z;
  } cam = {J.W, J.H, J.fx, J.fy, J.cx, J.cy, near_z};
  Pose P;
  load_pose(J.viewmat, P);
  const double m0 = means[li], m1 = means[n + li], m2 = means[2 * n + li];
  double p[3];
#pragma unroll
  for (int r = 0; r < 3; r++) p[r] = ((P.R[r][0] * m0 + P.R[r][1] * m1) + P.R[r][2] * m2) + P.t[r];
  if (!(p[2] > (double)cam.near_z)) return;
  if (!isfinite(p[0]) || !isfinite(p[1]) || !isfinite(p[2])) return;
  const double o = opac[li];
  const double s[3] = {scales[li], scales[n + li], scales[2 * n + li]};
  if (!isfinite(o) || !isfinite(s[0]) || !isfinite(s[1]) || !isfinite(s[2])) return;
  if (!isfinite(colors[li]) || !isfinite(colors[n + li]) || !isfinite(colors[2 * n + li])) return;
  const double qw = quats[li], qx = quats[n + li], qy = quats[2 * n + li], qz = quats[3 * n + li];
  const double n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
  if (!(n2 > 0.0) || !isfinite(n2)) return;
  const double rn = 1.0 / sqrt(n2);
  const double w = qw * rn, x = qx * rn, y = qy * rn, z = qz * rn;
  const double xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
  const double wx = w * x, wy = w * y, wz = w * z;
  const double Rq[3][3] = {{1.0 - 2.0 * (yy + zz), 2.0 * (xy - wz), 2.0 * (xz + wy)},
                           {2.0 * (xy + wz), 1.0 - 2.0 * (xx + zz), 2.0 * (yz - wx)},
                           {2.0 * (xz - wy), 2.0 * (yz + wx), 1.0 - 2.0 * (xx + yy)}};
  double M[3][3], Wm[3][3];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) M[a][b] = Rq[a][b] * s[b];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) Wm[a][b] = (P.R[a][0] * M[0][b] + P.R[a][1] * M[1][b]) + P.R[a][2] * M[2][b];
  const double fx = cam.fx, fy = cam.fy;
  const double rz = 1.0 / p[2];
  const double xn = p[0] * rz, yn = p[1] * rz;
  const double limx = (kGuard * (double)cam.W) / fx;
  const double limy = (kGuard * (double)cam.H) / fy;
  const double xc = dmin(dmax(xn, -limx), limx);
  const double yc = dmin(dmax(yn, -limy), limy);
  const double j00 = fx * rz, j02 = -((fx * xc) * rz);
  const double j11 = fy * rz, j12 = -((fy * yc) * rz);
  double V0[3], V1[3];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    V0[k] = j00 * Wm[0][k] + j02 * Wm[2][k];
    V1[k] = j11 * Wm[1][k] + j12 * Wm[2][k];
  }
  const double S00 = ((V0[0] * V0[0] + V0[1] * V0[1]) + V0[2] * V0[2]) + kDilation;
  const double S01 = (V0[0] * V1[0] + V0[1] * V1[1]) + V0[2] * V1[2];
  const double S11 = ((V1[0] * V1[0] + V1[1] * V1[1]) + V1[2] * V1[2]) + kDilation;
  if (!(S00 <= kSigma2Limit) || !(S11 <= kSigma2Limit) || !isfinite(S01)) return;
  const double u = fx * xn + (double)cam.cx;
  const double v = fy * yn + (double)cam.cy;
  if (!(fabs(u) <= kCentreLimit) || !(fabs(v) <= kCentreLimit)) return;
  const double rx = ceil(kBoxSigmas * sqrt(S00));
  const double ry = ceil(kBoxSigmas * sqrt(S11));
  const double xlo = ceil(u - rx), xhi = floor(u + rx);
  const double ylo = ceil(v - ry), yhi = floor(v + ry);
  if (!(xlo <= (double)(cam.W - 1)) || !(xhi >= 0.0) || !(ylo <= (double)(cam.H - 1)) || !(yhi >= 0.0)) return;
  const double det = S00 * S11 - S01 * S01;
  if (!(det > 0.0)) return;
  const float z32 = (float)p[2];
  if (!isfinite(z32)) return;
  const double sd = sqrt(det), s1 = sqrt(S11);
  const double l11 = s1 / sd;
  const double l12 = -S01 / (sd * s1);
  const double l22 = 1.0 / s1;
  const double ufl = floor(u), vfl = floor(v);
  const double lo255 = 255.0 * o;
  const double qc = (lo255 > 0.0) ? dmin(kQ9, pinned_log2(lo255)) : -INFINITY;

  const int bx0 = (int)dmax(xlo, 0.0), bx1 = (int)dmin(xhi, (double)(cam.W - 1));
  const int by0 = (int)dmax(ylo, 0.0), by1 = (int)dmin(yhi, (double)(cam.H - 1));
  const uint32_t ntx = (uint32_t)(bx1 / tile - bx0 / tile + 1);
  const uint32_t nty = (uint32_t)(by1 / tile - by0 / tile + 1);

  uint32_t zbits = __float_as_uint(z32);
  key[i] = zbits;
  if (gbin) {
    const uint32_t first = (uint32_t)(J.bin0 + (by0 / tile) * J.bx + bx0 / tile);
    gbin[i] = make_uint2(first, (ntx - 1u) | ((nty - 1u) << 10) | ((uint32_t)(J.bx - 1) << 20));
    float2* row = reinterpret_cast<float2*>(g2d + (int64_t)kGradFields * i);
#pragma unroll
    for (int f = 0; f < kGradFields / 2; f++) row[f] = make_float2(0.f, 0.f);
  } else {
    vis[i] = 1u;
    ntiles[i] = ntx * nty;
  }
  uint4 r0, r1, r2, r3;
  r0.x = __float_as_uint((float)ufl);   // integer-valued, |floor(u)| <= 2^22: exact
  r0.y = __float_as_uint((float)vfl);
  r0.z = __float_as_uint((float)(u - ufl));
  r0.w = __float_as_uint((float)(v - vfl));
  r1.x = __float_as_uint((float)(kKappa * l11));
  r1.y = __float_as_uint((float)(kKappa * l12));
  r1.z = __float_as_uint((float)(kKappa * l22));
  r1.w = __float_as_uint((float)qc);
  r2.x = __float_as_uint(log2f((float)o));
  r2.y = zbits;
  r2.z = __float_as_uint(colors[li]);
  r2.w = __float_as_uint(colors[n + li]);
  r3.x = __float_as_uint(colors[2 * n + li]);
  r3.y = (uint32_t)bx0 | ((uint32_t)bx1 << 16);
  r3.z = (uint32_t)by0 | ((uint32_t)by1 << 16);
  r3.w = (uint32_t)i;
  uint4* dst = rec_i + 4 * i;
  dst[0] = r0;
  dst[1] = r1;
  dst[2] = r2;
  dst[3] = r3;
}

// ------------------------------------------------------------------ backward

#pragma clang fp contract(fast)

// Reciprocal and reciprocal square root in binary64 for the adjoint: the
// hardware estimates (relative error about 2^-22) refined by two Newton
// steps, each of which squares the relative error, so the result is within a
// few units in the last place. The adjoint's outputs are binary32, so it
// needs neither correctly rounded quotients nor roots; each of these is a
// handful of dependent instructions where a correctly rounded division is
// about ten.
__device__ inline double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}
__device__ inline double rsq64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = __builtin_fma(0.5 * y, __builtin_fma(-x * y, y, 1.0), y);
  return __builtin_fma(0.5 * y, __builtin_fma(-x * y, y, 1.0), y);
}

__global__ void __launch_bounds__(256) k_project_bwd(const JobDesc* __restrict__ jobs, int njobs,
                                                     const uint32_t* __restrict__ key,
                                                     const int32_t* __restrict__ rank_of,
                                                     float* __restrict__ g2d,
                                                     const uint64_t* __restrict__ counters,
                                                     double* __restrict__ pose_part) {
  constexpr int kSub = kAdjSlots / 256;   // slots per thread
  __shared__ int s_list[kAdjSlots];
  __shared__ int s_wcnt[kSub][256 / 64];
  const JobDesc& J = jobs[job_of_block(jobs, njobs, (int)blockIdx.x * kSub)];
  const int64_t n = J.n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // The block's kAdjSlots slots (slot s * 256 + t belongs to thread t) are
  // checked for visibility, and the visible Gaussians are packed in index
  // order onto the block's threads, so every wave runs the long binary64
  // path with nearly all lanes busy (a quarter of the slots are visible in a
  // typical frame); each slot's owner writes the zero gradients of an
  // invisible Gaussian (and, through LDS, those computed for a visible one).
  const int64_t li0 = ((int64_t)blockIdx.x * kSub - J.block0) * 256;   // block's first index within the job
  bool own_vis[kSub];
  uint64_t vm[kSub];
#pragma unroll
  for (int u = 0; u < kSub; u++) {
    const int64_t li = li0 + u * 256 + threadIdx.x;
    own_vis[u] = li < n && key[J.g0 + li] != 0xFFFFFFFFu;
    vm[u] = __ballot(own_vis[u]);
    if (lane == 0) s_wcnt[u][wave] = __popcll(vm[u]);
  }
  __syncthreads();
  int vbase[kSub], nvis = 0;
#pragma unroll
  for (int u = 0; u < kSub; u++)
    for (int w = 0; w < 256 / 64; w++) {
      if (w == wave) vbase[u] = nvis;
      nvis += s_wcnt[u][w];
    }
#pragma unroll
  for (int u = 0; u < kSub; u++)
    if (own_vis[u])
      s_list[vbase[u] + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(vm[u] >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)vm[u], 0u))] =
          u * 256 + (int)threadIdx.x;
  __syncthreads();
  const auto means = global_ptr(J.means);
  const auto scales = global_ptr(J.scales);
  const auto quats = global_ptr(J.quats);
  const auto opac = global_ptr(J.opacity);
  struct {
    int W, H;
    float fx, fy;
  } cam = {J.W, J.H, J.fx, J.fy};
  const auto viewmat = global_ptr(J.viewmat);
  const auto gm_out = global_ptr(J.gm), gs_out = global_ptr(J.gs), gq_out = global_ptr(J.gq),
             go_out = global_ptr(J.go), gc_out = global_ptr(J.gc);
  const bool map_grads = !(J.flags & MS_FLAG_POSE_GRAD_ONLY);
  const bool pose_grads = !(J.flags & MS_FLAG_NO_POSE_GRAD);
  const bool accumulate = (J.flags & MS_FLAG_ACCUMULATE_MAP_GRADS) != 0;   // several views of one map
  const bool overflow = counters[C_OVERFLOW] != 0;
  // LDS shared by two phases: first it carries the gradients of the visible
  // Gaussians from the threads that computed them to the slots' owners, so
  // that every store of a gradient plane covers whole lines (64 consecutive
  // slots) instead of scattered parts of them; then it holds the pose
  // reduction. 56 KB per block: the adjoint's registers allow two blocks
  // per CU, whose LDS this leaves room for.
  __shared__ __attribute__((aligned(16))) float adj_lds[14 * kAdjSlots];
  float* xg = adj_lds;                                           // [14][kAdjSlots]: gm 3, gs 3, gc 3, gq 4, go
  double (*pr)[256] = reinterpret_cast<double (*)[256]>(adj_lds);   // [12][256]
  static_assert(12 * 256 * sizeof(double) <= 14 * kAdjSlots * sizeof(float), "pose reduction fits the exchange LDS");
  const bool exchange = map_grads && !accumulate;   // uniform; otherwise atomics, or no map gradients
  double GR[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, Gt[3] = {0, 0, 0};
  for (int h = threadIdx.x; h < nvis; h += 256) {
    const int64_t li = li0 + s_list[h];   // index within the job
    const int64_t i = J.g0 + li;          // virtual index
    float gm[3], gs[3], gq[4], go, gc[3];
    // accumulator row: by depth rank (global sort path) or by index (per-bin
    // path, where the row is cleared after use for the next backward)
    const int64_t r = rank_of ? (int64_t)rank_of[i] : i;
    float* acc = g2d + r * kGradFields;
    const double E = acc[0], P1 = acc[1], P2 = acc[2], P1x = acc[3], P1y = acc[4], P2y = acc[5];
    const double GZ = acc[9];
    gc[0] = acc[6];
    gc[1] = acc[7];
    gc[2] = acc[8];
    if (!rank_of) {
      float2* row = reinterpret_cast<float2*>(acc);
#pragma unroll
      for (int f = 0; f < kGradFields / 2; f++) row[f] = make_float2(0.f, 0.f);
    }
    Pose P;
    load_pose(viewmat, P);
    const double mu[3] = {means[li], means[n + li], means[2 * n + li]};
    const double s[3] = {scales[li], scales[n + li], scales[2 * n + li]};
    const double q[4] = {quats[li], quats[n + li], quats[2 * n + li], quats[3 * n + li]};
    const double o = opac[li];
    double p[3];
    for (int a = 0; a < 3; a++) p[a] = P.R[a][0] * mu[0] + P.R[a][1] * mu[1] + P.R[a][2] * mu[2] + P.t[a];
    const double qn2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    const double iq = rsq64(qn2);   // qn2 > 0 for every visible Gaussian
    const double w = q[0] * iq, x = q[1] * iq, y = q[2] * iq, z = q[3] * iq;
    const double Rq[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                             {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                             {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
    double M[3][3], Wm[3][3];
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) M[a][b] = Rq[a][b] * s[b];
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) Wm[a][b] = P.R[a][0] * M[0][b] + P.R[a][1] * M[1][b] + P.R[a][2] * M[2][b];
    const double fx = cam.fx, fy = cam.fy;
    const double Z = p[2], rz = rcp64(Z);   // Z > near plane > 0
    const double xn = p[0] * rz, yn = p[1] * rz;
    const double limx = kGuard * cam.W / fx, limy = kGuard * cam.H / fy;
    const int clx = xn < -limx ? -1 : (xn > limx ? 1 : 0);
    const int cly = yn < -limy ? -1 : (yn > limy ? 1 : 0);
    const double xc = clx ? clx * limx : xn, yc = cly ? cly * limy : yn;
    const double j00 = fx * rz, j02 = -fx * xc * rz, j11 = fy * rz, j12 = -fy * yc * rz;
    double V0[3], V1[3];
    for (int k = 0; k < 3; k++) {
      V0[k] = j00 * Wm[0][k] + j02 * Wm[2][k];
      V1[k] = j11 * Wm[1][k] + j12 * Wm[2][k];
    }
    const double s0 = V0[0] * V0[0] + V0[1] * V0[1] + V0[2] * V0[2] + kDilation;
    const double s1 = V0[0] * V1[0] + V0[1] * V1[1] + V0[2] * V1[2];
    const double s2 = V1[0] * V1[0] + V1[1] * V1[1] + V1[2] * V1[2] + kDilation;
    const double d = s0 * s2 - s1 * s1;   // >= 0.09: both diagonals carry the dilation
    const double r_sqd = rsq64(d), r_sqs2 = rsq64(s2);
    const double sqs2 = s2 * r_sqs2, r_d = r_sqd * r_sqd, r_s2 = r_sqs2 * r_sqs2;
    const double l11 = sqs2 * r_sqd, l22 = r_sqs2;
    const double l12 = -s1 * (r_sqd * r_sqs2);
    const double a_ = kKappa * l11, b_ = kKappa * l12, c_ = kKappa * l22;
    // record-level gradients; g_t = -2 ln2 t e collected as P-sums
    const double c2 = -2.0 * kLn2;
    const double gu = -a_ * c2 * P1;
    const double gv = -(b_ * c2 * P1 + c_ * c2 * P2);
    const double gl11 = kKappa * c2 * P1x, gl12 = kKappa * c2 * P1y, gl22 = kKappa * c2 * P2y;
    go = (float)(o > 0.0 ? E * rcp64(o) : 0.0);   // opacity 0 composites nowhere (E = 0)
    // Cholesky factors -> (S00, S01, S11)
    const double r_dsq = r_d * r_sqd * r_sqs2;   // 1 / (d sqrt(d s2))
    const double gS0 = gl11 * (-0.5 * l11 * s2 * r_d) + gl12 * (-0.5 * l12 * s2 * r_d);
    const double gS1 = gl11 * (l11 * s1 * r_d) + gl12 * (-(s0 * s2) * r_dsq);
    const double gS2 = gl11 * (0.5 * l11 * (r_s2 - s0 * r_d)) + gl12 * (-0.5 * l12 * (s0 * r_d + r_s2)) +
                       gl22 * (-0.5 * l22 * r_s2);
    // S = V V^T + 0.3 I
    double gV0[3], gV1[3];
    for (int k = 0; k < 3; k++) {
      gV0[k] = 2.0 * gS0 * V0[k] + gS1 * V1[k];
      gV1[k] = gS1 * V0[k] + 2.0 * gS2 * V1[k];
    }
    double gj00 = 0, gj02 = 0, gj11 = 0, gj12 = 0;
    double gW[3][3];
    for (int k = 0; k < 3; k++) {
      gj00 += gV0[k] * Wm[0][k];
      gj02 += gV0[k] * Wm[2][k];
      gj11 += gV1[k] * Wm[1][k];
      gj12 += gV1[k] * Wm[2][k];
      gW[0][k] = j00 * gV0[k];
      gW[1][k] = j11 * gV1[k];
      gW[2][k] = j02 * gV0[k] + j12 * gV1[k];
    }
    // Wm = R M
    double gM[3][3];
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) {
        gM[a][b] = P.R[0][a] * gW[0][b] + P.R[1][a] * gW[1][b] + P.R[2][a] * gW[2][b];
        GR[a][b] += gW[a][0] * M[b][0] + gW[a][1] * M[b][1] + gW[a][2] * M[b][2];
      }
    // M = Rq diag(s)
    double gRq[3][3];
    for (int b = 0; b < 3; b++) {
      gs[b] = (float)(gM[0][b] * Rq[0][b] + gM[1][b] * Rq[1][b] + gM[2][b] * Rq[2][b]);
      for (int a = 0; a < 3; a++) gRq[a][b] = gM[a][b] * s[b];
    }
    // Rq(w, x, y, z)
    double gw = 2 * (-z * gRq[0][1] + y * gRq[0][2] + z * gRq[1][0] - x * gRq[1][2] - y * gRq[2][0] + x * gRq[2][1]);
    double gx = 2 * (y * gRq[0][1] + z * gRq[0][2] + y * gRq[1][0] - 2 * x * gRq[1][1] - w * gRq[1][2] +
                     z * gRq[2][0] + w * gRq[2][1] - 2 * x * gRq[2][2]);
    double gy = 2 * (-2 * y * gRq[0][0] + x * gRq[0][1] + w * gRq[0][2] + x * gRq[1][0] + z * gRq[1][2] -
                     w * gRq[2][0] + z * gRq[2][1] - 2 * y * gRq[2][2]);
    double gz = 2 * (-2 * z * gRq[0][0] - w * gRq[0][1] + x * gRq[0][2] + w * gRq[1][0] - 2 * z * gRq[1][1] +
                     y * gRq[1][2] + x * gRq[2][0] + y * gRq[2][1]);
    const double dot = gw * w + gx * x + gy * y + gz * z;
    gq[0] = (float)((gw - w * dot) * iq);
    gq[1] = (float)((gx - x * dot) * iq);
    gq[2] = (float)((gy - y * dot) * iq);
    gq[3] = (float)((gz - z * dot) * iq);
    // J(p), (u, v)(p), direct depth
    double gp[3] = {0, 0, GZ};
    gp[2] += gj00 * (-fx * rz * rz) + gj11 * (-fy * rz * rz);
    if (clx == 0) {
      gp[0] += gj02 * (-fx * rz * rz);
      gp[2] += gj02 * (2.0 * fx * p[0] * rz * rz * rz);
    } else {
      gp[2] += gj02 * (fx * clx * limx * rz * rz);
    }
    if (cly == 0) {
      gp[1] += gj12 * (-fy * rz * rz);
      gp[2] += gj12 * (2.0 * fy * p[1] * rz * rz * rz);
    } else {
      gp[2] += gj12 * (fy * cly * limy * rz * rz);
    }
    gp[0] += gu * fx * rz;
    gp[2] += -gu * fx * p[0] * rz * rz;
    gp[1] += gv * fy * rz;
    gp[2] += -gv * fy * p[1] * rz * rz;
    // p = R mu + t
    for (int b = 0; b < 3; b++) gm[b] = (float)(P.R[0][b] * gp[0] + P.R[1][b] * gp[1] + P.R[2][b] * gp[2]);
    for (int a = 0; a < 3; a++) {
      for (int b = 0; b < 3; b++) GR[a][b] += gp[a] * mu[b];
      Gt[a] += gp[a];
    }
    if (overflow) {
      const float nanv = __builtin_nanf("");
      for (int k = 0; k < 3; k++) gm[k] = gs[k] = gc[k] = nanv;
      for (int k = 0; k < 4; k++) gq[k] = nanv;
      go = nanv;
    }
    if (map_grads && accumulate) {
      for (int k = 0; k < 3; k++) {
        __builtin_amdgcn_global_atomic_fadd_f32(gm_out + k * n + li, gm[k]);
        __builtin_amdgcn_global_atomic_fadd_f32(gs_out + k * n + li, gs[k]);
        __builtin_amdgcn_global_atomic_fadd_f32(gc_out + k * n + li, gc[k]);
      }
      for (int k = 0; k < 4; k++) __builtin_amdgcn_global_atomic_fadd_f32(gq_out + k * n + li, gq[k]);
      __builtin_amdgcn_global_atomic_fadd_f32(go_out + li, go);
    } else if (exchange) {
      for (int k = 0; k < 3; k++) {
        xg[k * kAdjSlots + h] = gm[k];
        xg[(3 + k) * kAdjSlots + h] = gs[k];
        xg[(6 + k) * kAdjSlots + h] = gc[k];
      }
      for (int k = 0; k < 4; k++) xg[(9 + k) * kAdjSlots + h] = gq[k];
      xg[13 * kAdjSlots + h] = go;
    }
  }
  // Every slot's owner stores its gradients (zero for an invisible
  // Gaussian). The stores come after all of the block's loads: one counter
  // covers a wave's loads and stores, so a load issued after stores would
  // wait for them.
  if (exchange) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kSub; u++) {
      const int64_t li = li0 + u * 256 + threadIdx.x;
      if (li < n) {
        const int h = vbase[u] + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(vm[u] >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)vm[u], 0u));
        const bool v = own_vis[u];
        for (int k = 0; k < 3; k++) {
          gm_out[k * n + li] = v ? xg[k * kAdjSlots + h] : 0.f;
          gs_out[k * n + li] = v ? xg[(3 + k) * kAdjSlots + h] : 0.f;
          gc_out[k * n + li] = v ? xg[(6 + k) * kAdjSlots + h] : 0.f;
        }
        for (int k = 0; k < 4; k++) gq_out[k * n + li] = v ? xg[(9 + k) * kAdjSlots + h] : 0.f;
        go_out[li] = v ? xg[13 * kAdjSlots + h] : 0.f;
      }
    }
    __syncthreads();   // the pose reduction below reuses the LDS
  }
  if (!pose_grads) return;   // uniform over the block (one job per block)
  // block reduction of the 12 pose partials of the threads: through LDS, in a
  // fixed order (16 partial sums of 16 threads each, then their sum)
  __shared__ double ps[12][16];
  for (int a = 0; a < 3; a++) {
    for (int b = 0; b < 3; b++) pr[3 * a + b][threadIdx.x] = GR[a][b];
    pr[9 + a][threadIdx.x] = Gt[a];
  }
  __syncthreads();
  if (threadIdx.x < 12 * 16) {
    const int k = threadIdx.x >> 4, seg = threadIdx.x & 15;
    double acc = 0.0;
    for (int j = seg * 16; j < seg * 16 + 16; j++) acc += pr[k][j];
    ps[k][seg] = acc;
  }
  __syncthreads();
  if (threadIdx.x < 12) {
    double acc = 0.0;
    for (int q = 0; q < 16; q++) acc += ps[threadIdx.x][q];
    pose_part[(int64_t)blockIdx.x * 12 + threadIdx.x] = acc;
  }
}

// One block per job: folds the job's per-block pose partials in a fixed
// order and writes dL/d[R|t] and the left-twist gradient.
constexpr int kPoseThreads = 256;

__global__ void __launch_bounds__(kPoseThreads) k_pose_final(const JobDesc* __restrict__ jobs,
                                                             const double* __restrict__ part,
                                                             const uint64_t* __restrict__ counters) {
  __shared__ double pr[12][kPoseThreads];
  __shared__ double ps[12][16];
  __shared__ double tot[12];
  const JobDesc& J = jobs[blockIdx.x];
  if (J.flags & MS_FLAG_NO_POSE_GRAD) return;   // uniform over the block
  const auto viewmat = global_ptr(J.viewmat);
  const auto gview = global_ptr(J.gview);
  const auto gtwist = global_ptr(J.gtwist);
  const int nblocks = (int)((J.n + kAdjSlots - 1) / kAdjSlots);   // adjoint blocks of this job
  part += (int64_t)(J.block0 / (kAdjSlots / 256)) * 12;
  // thread t folds partials t, t + 256, ...; then 16 sums of 16 threads and
  // their sum, all in a fixed order
  double acc[12];
  for (int k = 0; k < 12; k++) acc[k] = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kPoseThreads)
    for (int k = 0; k < 12; k++) acc[k] += part[(int64_t)b * 12 + k];
  for (int k = 0; k < 12; k++) pr[k][threadIdx.x] = acc[k];
  __syncthreads();
  if (threadIdx.x < 12 * 16) {
    const int k = threadIdx.x >> 4, seg = threadIdx.x & 15;
    double a = 0.0;
    for (int j = seg * 16; j < seg * 16 + 16; j++) a += pr[k][j];
    ps[k][seg] = a;
  }
  __syncthreads();
  if (threadIdx.x < 12) {
    double a = 0.0;
    for (int q = 0; q < 16; q++) a += ps[threadIdx.x][q];
    tot[threadIdx.x] = a;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const bool overflow = counters[C_OVERFLOW] != 0;
  const float nanv = __builtin_nanf("");
  double GR[3][3], Gt[3], R[3][3], t[3];
  for (int a = 0; a < 3; a++) {
    for (int b = 0; b < 3; b++) {
      GR[a][b] = tot[3 * a + b];
      R[a][b] = viewmat[4 * a + b];
    }
    Gt[a] = tot[9 + a];
    t[a] = viewmat[4 * a + 3];
  }
  if (gview) {
    for (int a = 0; a < 3; a++) {
      for (int b = 0; b < 3; b++) gview[4 * a + b] = overflow ? nanv : (float)GR[a][b];
      gview[4 * a + 3] = overflow ? nanv : (float)Gt[a];
    }
  }
  if (gtwist) {
    // left perturbation: d/drho = dL/dt; d/dphi = sum_k R[:,k] x GR[:,k] + t x dL/dt
    double phi[3] = {0, 0, 0};
    for (int k = 0; k < 3; k++) {
      phi[0] += R[1][k] * GR[2][k] - R[2][k] * GR[1][k];
      phi[1] += R[2][k] * GR[0][k] - R[0][k] * GR[2][k];
      phi[2] += R[0][k] * GR[1][k] - R[1][k] * GR[0][k];
    }
    phi[0] += t[1] * Gt[2] - t[2] * Gt[1];
    phi[1] += t[2] * Gt[0] - t[0] * Gt[2];
    phi[2] += t[0] * Gt[1] - t[1] * Gt[0];
    for (int k = 0; k < 3; k++) {
      gtwist[k] = overflow ? nanv : (float)Gt[k];
      gtwist[3 + k] = overflow ? nanv : (float)phi[k];
    }
  }
}

}  // namespace

hipError_t launch_project_fwd(const Plan& p, float near_z, const JobTable& t, uint32_t* zero, int64_t zcount,
                              char* ws, hipStream_t st) {
  if (p.n == 0) return hipSuccess;
  const bool bi = p.by_index;
  hipLaunchKernelGGL(k_project_fwd, dim3((unsigned)(p.n / 256)), dim3(256), 0, st, t, at<JobTable>(ws, p.jobs), zero,
                     zcount, near_z, p.bin, at<uint32_t>(ws, p.key),
                     bi ? nullptr : at<uint32_t>(ws, p.vis_pos), bi ? nullptr : at<uint32_t>(ws, p.ntiles),
                     bi ? nullptr : at<int32_t>(ws, p.rank_of), at<uint4>(ws, p.rec_i),
                     bi ? at<uint2>(ws, p.gbin) : nullptr, bi ? at<float>(ws, p.g2d) : nullptr);
  return hipGetLastError();
}

hipError_t launch_project_bwd(const Plan& p, bool any_pose, char* ws, hipStream_t st) {
  const JobDesc* jobs = at<JobTable>(ws, p.jobs)->job;
  if (p.n > 0) {
    hipLaunchKernelGGL(k_project_bwd, dim3((unsigned)(p.n / kAdjSlots)), dim3(256), 0, st, jobs, p.njobs,
                       at<uint32_t>(ws, p.key), p.by_index ? nullptr : at<int32_t>(ws, p.rank_of),
                       at<float>(ws, p.g2d),
                       at<uint64_t>(ws, p.counters), at<double>(ws, p.pose_part));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (any_pose) {
    StageScope tm(MS_STAGE_POSE, st);
    hipLaunchKernelGGL(k_pose_final, dim3((unsigned)p.njobs), dim3(kPoseThreads), 0, st, jobs, at<double>(ws, p.pose_part),
                       at<uint64_t>(ws, p.counters));
    return hipGetLastError();
  }
  return hipSuccess;
}

}  // namespace ms

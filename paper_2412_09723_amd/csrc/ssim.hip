// SSIM term of the mapping objective (Eq. 7), with the SSIM of the
// evaluation-metrics appendix: S = (2 mx my + C1)(2 sxy + C2) /
// ((mx^2 + my^2 + C1)(sx^2 + sy^2 + C2)) from local statistics under an
// 11x11 Gaussian window (std 1.5 px, weights summing to 1), zero outside the
// image. The loss is weight * (1 - mean S) over all channels and pixels and
// its gradient with respect to the rendered image x is
//   dL/dx(p) = sum_q w(q - p) (a(q) + 2 x(p) b(q) + y(p) c(q)),
// a = dS/dmx, b = dS/dE[x^2] = -S / B2, c = dS/dE[xy] = 2 S / A2, each times
// dL/dS = -weight / (channels * pixels).
//
// One workgroup of 512 threads per 32x32 output tile and channel, everything
// in LDS (65 KB: two workgroups per CU):
//   0. x and y on the 52x52 region the tile's gradient depends on;
//   1. row sums (11 taps) of x, y, x^2, y^2, xy on 52 rows x 42 columns;
//   2. column sums: the five statistics on the 42x42 region whose windows
//      reach the tile, then S and a, b, c there (zero outside the image);
//   3. row sums of a, b, c on 42 rows x 32 columns;
//   4. column sums on the 32x32 tile and the gradient.
// The tile's own pixels add their S to the loss (one atomic per workgroup).
// Every pass is separable and register-blocked along its direction.
#include "ms_internal.h"

namespace ms {
namespace {

constexpr int kSsimTile = 32;                         // output tile edge
constexpr int kSsimRad = 5;                           // window radius
constexpr int kSsimTaps = 2 * kSsimRad + 1;
constexpr int kSsimStat = kSsimTile + 2 * kSsimRad;   // 42: statistics region edge
constexpr int kSsimIn = kSsimTile + 4 * kSsimRad;     // 52: input region edge
constexpr int kSsimThreads = 512;
constexpr int kRunStat = 7;    // statistics pass: 42 columns x 6 runs, one per thread
constexpr int kRunGrad = 4;    // the two passes over a, b, c: 42 x 8 and 32 x 8 runs
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

// region 1: x, y (2 x 52 x 52), later a, b, c (3 x 42 x 42) and, in the
// pair form, a_y (4 x 42 x 42)
template <bool kPair>
constexpr int ssim_r1() {
  return kPair ? 4 * kSsimStat * kSsimStat : 2 * kSsimIn * kSsimIn;
}
static_assert(4 * kSsimStat * kSsimStat >= 2 * kSsimIn * kSsimIn, "x, y fit the pair form's region 1");
// region 2: five row-sum planes (5 x 52 x 42), later three or four (x 42 x 32)
constexpr int kR2 = 5 * kSsimIn * kSsimStat;
static_assert(3 * kSsimStat * kSsimStat <= 2 * kSsimIn * kSsimIn, "a, b, c fit region 1");
static_assert(4 * kSsimStat * kSsimTile <= kR2, "their row sums fit region 2");

// Pair form, depth part: the L1 term of the two depth planes on one 32x32
// tile (no window); returns the tile's share of the loss from thread 0.
__device__ inline float depth_l1_tile(const SsimArgs& A, int X0, int Y0, int t) {
  float acc = 0.f;
  for (int i = t; i < kSsimTile * kSsimTile; i += kSsimThreads) {
    const int gx = X0 + (i % kSsimTile), gy = Y0 + i / kSsimTile;
    if (gx >= A.W || gy >= A.H) continue;
    const int64_t q = (int64_t)gy * A.W + gx;
    const float d = A.dx[q] - A.dy[q];
    const float g = l1_sign(d, A.sgeom);
    A.gdx[q] = A.accumulate ? A.gdx[q] + g : g;
    A.gdy[q] = A.accumulate ? A.gdy[q] - g : -g;
    acc += fabsf(d) * A.sgeom;
  }
  return acc;
}

template <bool kPair>
__global__ void __launch_bounds__(kSsimThreads) k_ssim_grad(SsimArgs A) {
  constexpr int kR1 = ssim_r1<kPair>();
  constexpr int kPlanes = kPair ? 4 : 3;   // a (a_x), b, c, and a_y
  __shared__ float r1[kR1];
  __shared__ float r2[kR2];
  __shared__ float red[kSsimThreads / 64];
  const int t = threadIdx.x;
  const int W = A.W, H = A.H;
  const int64_t P = (int64_t)W * H;
  // workgroups go to the eight XCDs in turn: give each XCD a contiguous run
  // of tiles so that neighbouring tiles' halos meet in one L2
  const int gx = (W + kSsimTile - 1) / kSsimTile, gy = (H + kSsimTile - 1) / kSsimTile;
  const int total = gx * gy * (A.C + (kPair ? 1 : 0)), per = (total + 7) / 8;
  const int tile = ((int)blockIdx.x % 8) * per + (int)blockIdx.x / 8;
  if (tile >= total) return;
  if (kPair && tile >= gx * gy * A.C) {   // block-uniform: a depth tile
    const int rem = tile - gx * gy * A.C, by = rem / gx, bx = rem - by * gx;
    float acc = depth_l1_tile(A, bx * kSsimTile, by * kSsimTile, t);
    if (!A.loss) return;
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((t & 63) == 0) red[t >> 6] = acc;
    __syncthreads();
    if (t == 0) {
      float s = 0.f;
      for (int w = 0; w < kSsimThreads / 64; w++) s += red[w];
      unsafeAtomicAdd(A.loss, s);
    }
    return;
  }
  const int bz = tile / (gx * gy), rem = tile - bz * gx * gy, by = rem / gx, bx = rem - by * gx;
  const int X0 = bx * kSsimTile, Y0 = by * kSsimTile;
  const float* __restrict__ x = A.pred + (int64_t)bz * P;
  const float* __restrict__ y = A.target + (int64_t)bz * P;
  float* __restrict__ grad = A.grad + (int64_t)bz * P;
  float g[kSsimTaps];
#pragma unroll
  for (int k = 0; k < kSsimTaps; k++) g[k] = A.w[k];

  // 0. input region, origin (X0 - 2R, Y0 - 2R)
  float* xs = r1;
  float* ys = r1 + kSsimIn * kSsimIn;
  for (int i = t; i < kSsimIn * kSsimIn; i += kSsimThreads) {
    const int r = i / kSsimIn, c = i - r * kSsimIn;
    const int gx = X0 - 2 * kSsimRad + c, gy = Y0 - 2 * kSsimRad + r;
    const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
    const int64_t o = (int64_t)gy * W + gx;
    xs[i] = in ? x[o] : 0.f;
    ys[i] = in ? y[o] : 0.f;
  }
  __syncthreads();
  // Each thread produces a run of kRun consecutive outputs of a pass from the
  // kRun + 2R inputs it loads once, instead of 2R + 1 loads per output.
  // 1. row sums: plane q at (row r, column c) sums input columns c .. c + 2R
  constexpr int kP1 = kSsimIn * kSsimStat;
  {
    constexpr int kRun = 6, kGroups = kSsimStat / kRun, kLen = kRun + 2 * kSsimRad;
    static_assert(kGroups * kRun == kSsimStat, "row-sum runs tile the statistics columns");
    for (int it = t; it < kSsimIn * kGroups; it += kSsimThreads) {
      const int r = it / kGroups, c0 = (it - r * kGroups) * kRun;
      float xv[kLen], yv[kLen];
#pragma unroll
      for (int j = 0; j < kLen; j++) {
        xv[j] = xs[r * kSsimIn + c0 + j];
        yv[j] = ys[r * kSsimIn + c0 + j];
      }
#pragma unroll
      for (int o = 0; o < kRun; o++) {
        float sx = 0.f, sy = 0.f, sxx = 0.f, syy = 0.f, sxy = 0.f;
#pragma unroll
        for (int k = 0; k < kSsimTaps; k++) {
          const float xk = xv[o + k], yk = yv[o + k];
          sx = __builtin_fmaf(g[k], xk, sx);
          sy = __builtin_fmaf(g[k], yk, sy);
          sxx = __builtin_fmaf(g[k], xk * xk, sxx);
          syy = __builtin_fmaf(g[k], yk * yk, syy);
          sxy = __builtin_fmaf(g[k], xk * yk, sxy);
        }
        const int i = r * kSsimStat + c0 + o;
        r2[i] = sx;
        r2[kP1 + i] = sy;
        r2[2 * kP1 + i] = sxx;
        r2[3 * kP1 + i] = syy;
        r2[4 * kP1 + i] = sxy;
      }
    }
  }
  __syncthreads();
  // 2. statistics on the 42x42 region, origin (X0 - R, Y0 - R); S and a, b, c
  constexpr int kP2 = kSsimStat * kSsimStat;
  float* pa = r1;
  float* pb = r1 + kP2;
  float* pc = r1 + 2 * kP2;
  float* pay = r1 + 3 * kP2;   // pair form only
  float ssum = 0.f;
  {
    constexpr int kRun = kRunStat, kGroups = kSsimStat / kRun, kLen = kRun + 2 * kSsimRad;
    for (int it = t; it < kSsimStat * kGroups; it += kSsimThreads) {
      const int c = it % kSsimStat, r0 = (it / kSsimStat) * kRun;   // neighbouring threads: neighbouring columns
      float st[5][kRun];
#pragma unroll
      for (int q = 0; q < 5; q++) {
        float v[kLen];
#pragma unroll
        for (int j = 0; j < kLen; j++) v[j] = r2[q * kP1 + (r0 + j) * kSsimStat + c];
#pragma unroll
        for (int o = 0; o < kRun; o++) {
          float s = 0.f;
#pragma unroll
          for (int k = 0; k < kSsimTaps; k++) s = __builtin_fmaf(g[k], v[o + k], s);
          st[q][o] = s;
        }
      }
      const int gx = X0 - kSsimRad + c;
      const bool own_col = c >= kSsimRad && c < kSsimRad + kSsimTile;
#pragma unroll
      for (int o = 0; o < kRun; o++) {
        const int r = r0 + o, gy = Y0 - kSsimRad + r;
        float va = 0.f, vb = 0.f, vc = 0.f, vay = 0.f;
        if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
          const float mx = st[0][o], my = st[1][o];
          const float a1 = 2.f * mx * my + kC1;
          const float a2 = 2.f * (st[4][o] - mx * my) + kC2;
          const float b1 = mx * mx + my * my + kC1;
          const float b2 = (st[2][o] - mx * mx) + (st[3][o] - my * my) + kC2;
          // hardware reciprocals (about 1 ulp): the partials need no
          // correctly rounded quotients
          const float ra1 = __builtin_amdgcn_rcpf(a1), ra2 = __builtin_amdgcn_rcpf(a2);
          const float rb1 = __builtin_amdgcn_rcpf(b1), rb2 = __builtin_amdgcn_rcpf(b2);
          const float sv = (a1 * a2) * (rb1 * rb2);
          const float ds = A.dS * sv;
          va = ds * (2.f * my * (ra1 - ra2) + 2.f * mx * (rb2 - rb1));
          vb = -ds * rb2;
          vc = 2.f * ds * ra2;
          // S is symmetric in x and y: dS/dmy swaps their roles
          if (kPair) vay = ds * (2.f * mx * (ra1 - ra2) + 2.f * my * (rb2 - rb1));
          if (own_col && r >= kSsimRad && r < kSsimRad + kSsimTile) ssum += sv;
        }
        const int i = r * kSsimStat + c;
        pa[i] = va;
        pb[i] = vb;
        pc[i] = vc;
        if (kPair) pay[i] = vay;
      }
    }
  }
  __syncthreads();
  // 3. row sums of a, b, c: (row r of the statistics region, tile column c)
  constexpr int kP3 = kSsimStat * kSsimTile;
  {
    constexpr int kRun = kRunGrad, kGroups = kSsimTile / kRun, kLen = kRun + 2 * kSsimRad;
    for (int it = t; it < kSsimStat * kGroups; it += kSsimThreads) {
      const int r = it / kGroups, c0 = (it - r * kGroups) * kRun;
      float v[kPlanes][kLen];
#pragma unroll
      for (int j = 0; j < kLen; j++) {
        const int i = r * kSsimStat + c0 + j;
#pragma unroll
        for (int q = 0; q < kPlanes; q++) v[q][j] = r1[q * kP2 + i];
      }
#pragma unroll
      for (int o = 0; o < kRun; o++) {
        const int i = r * kSsimTile + c0 + o;
#pragma unroll
        for (int q = 0; q < kPlanes; q++) {
          float sq = 0.f;
#pragma unroll
          for (int k = 0; k < kSsimTaps; k++) sq = __builtin_fmaf(g[k], v[q][o + k], sq);
          r2[q * kP3 + i] = sq;
        }
      }
    }
  }
  __syncthreads();
  // 4. column sums on the tile and the gradient
  float l1sum = 0.f;
  {
    constexpr int kRun = kRunGrad, kGroups = kSsimTile / kRun, kLen = kRun + 2 * kSsimRad;
    for (int it = t; it < kSsimTile * kGroups; it += kSsimThreads) {
      const int c = it % kSsimTile, r0 = (it / kSsimTile) * kRun;
      const int gx = X0 + c;
      if (gx >= W) continue;
      float sum[kPlanes][kRun];
#pragma unroll
      for (int q = 0; q < kPlanes; q++) {
        float v[kLen];
#pragma unroll
        for (int j = 0; j < kLen; j++) v[j] = r2[q * kP3 + (r0 + j) * kSsimTile + c];
#pragma unroll
        for (int o = 0; o < kRun; o++) {
          float s = 0.f;
#pragma unroll
          for (int k = 0; k < kSsimTaps; k++) s = __builtin_fmaf(g[k], v[o + k], s);
          sum[q][o] = s;
        }
      }
#pragma unroll
      for (int o = 0; o < kRun; o++) {
        const int gy = Y0 + r0 + o;
        if (gy >= H) break;
        const int64_t q = (int64_t)gy * W + gx;
        const float xq = x[q], yq = y[q];
        const float v = sum[0][o] + 2.f * xq * sum[1][o] + yq * sum[2][o];
        if (kPair) {
          // the L1 term of the pair, and dL/dy by the same window sums
          const float d = xq - yq;
          const float l1 = l1_sign(d, A.sl1);
          const float vy = sum[3][o] + 2.f * yq * sum[1][o] + xq * sum[2][o];
          float* __restrict__ grad_y = A.grad_y + (int64_t)bz * P;
          grad[q] = A.accumulate ? grad[q] + (v + l1) : v + l1;
          grad_y[q] = A.accumulate ? grad_y[q] + (vy - l1) : vy - l1;
          l1sum += fabsf(d) * A.sl1;
        } else {
          grad[q] = A.accumulate ? grad[q] + v : v;
        }
      }
    }
  }
  if (!A.loss) return;
  ssum = A.dS * ssum + l1sum;   // this thread's share of the loss
  for (int off = 32; off > 0; off >>= 1) ssum += __shfl_xor(ssum, off, 64);
  if ((t & 63) == 0) red[t >> 6] = ssum;
  __syncthreads();
  if (t == 0) {
    float s = 0.f;
    for (int w = 0; w < kSsimThreads / 64; w++) s += red[w];
    // weight * (1 - mean S): the constant once, from the first workgroup
    const bool first = bx == 0 && by == 0 && bz == 0;
    unsafeAtomicAdd(A.loss, s + (first ? A.weight : 0.f));
  }
}

}  // namespace

hipError_t launch_ssim_grad(const SsimArgs& a, hipStream_t st) {
  if (a.W <= 0 || a.H <= 0 || a.C <= 0) return hipSuccess;
  // one workgroup per (tile, channel) -- and per depth tile in the pair form
  // -- rounded up to a multiple of the eight XCDs
  const bool pair = a.grad_y != nullptr;
  const int total = ((a.W + kSsimTile - 1) / kSsimTile) * ((a.H + kSsimTile - 1) / kSsimTile) * (a.C + (pair ? 1 : 0));
  const dim3 grid((unsigned)((total + 7) / 8 * 8));
  if (pair)
    hipLaunchKernelGGL(k_ssim_grad<true>, grid, dim3(kSsimThreads), 0, st, a);
  else
    hipLaunchKernelGGL(k_ssim_grad<false>, grid, dim3(kSsimThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace ms

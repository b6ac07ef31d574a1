// Tracking-loop helpers around the render: the gradient of the L1
// photometric/depth loss (the loss form of Eq. 7's L1 terms, used here for
// per-agent tracking), and one Adam step on the left SE(3) twist of the pose
// (Sec. 3.1 poses in SE(3)), applied as [R|t] <- exp(-step^) [R|t]. Both stay
// on the device so a tracking step needs no host round trip.
#include "ms_internal.h"

namespace ms {
namespace {

constexpr int kLossThreads = 256;

// The three planes of one L1 loss gradient in one launch: for the flat
// index j over rgb (3P entries), depth (P) and silhouette (P),
// grad = scale * sign(pred - target) with the plane's scale; optional loss
// sum (sum of scale |pred - target|) accumulated with one atomic per block.
struct L1Planes {
  const float* pred[3];
  const float* target[3];
  float* grad[3];
  float scale[3];
  int64_t end[3];   // cumulative flat end of each plane
};


// VEC: every plane length is a multiple of 4 and every plane 16-byte
// aligned, so j counts groups of four floats (L.end in groups).
template <bool VEC>
__global__ void __launch_bounds__(kLossThreads) k_l1_grad(L1Planes L, float* __restrict__ loss) {
  __shared__ float red[kLossThreads / 64];
  float acc = 0.f;
  const int64_t total = L.end[2];
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < total; j += (int64_t)gridDim.x * blockDim.x) {
    const int pl = j < L.end[0] ? 0 : (j < L.end[1] ? 1 : 2);
    const int64_t o = pl == 0 ? j : j - L.end[pl - 1];
    const float sc = L.scale[pl];
    if (VEC) {
      const float4 a = reinterpret_cast<const float4*>(L.pred[pl])[o];
      const float4 b = reinterpret_cast<const float4*>(L.target[pl])[o];
      const float4 d = make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
      reinterpret_cast<float4*>(L.grad[pl])[o] =
          make_float4(l1_sign(d.x, sc), l1_sign(d.y, sc), l1_sign(d.z, sc), l1_sign(d.w, sc));
      acc += (fabsf(d.x) + fabsf(d.y) + fabsf(d.z) + fabsf(d.w)) * sc;
    } else {
      const float d = L.pred[pl][o] - L.target[pl][o];
      L.grad[pl][o] = l1_sign(d, sc);
      acc += fabsf(d) * sc;
    }
  }
  if (!loss) return;
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int w = 0; w < kLossThreads / 64; w++) s += red[w];
    unsafeAtomicAdd(loss, s);
  }
}

__global__ void k_zero_f32(float* p) { *p = 0.f; }

// Writes the job table (passed by value) into the workspace and zeroes
// `count` words at `zero` (the first launch of a pass: one launch for both).
__global__ void __launch_bounds__(256) k_setup(JobTable t, JobTable* __restrict__ dst, uint32_t* __restrict__ zero,
                                               int64_t count) {
  if (blockIdx.x == 0) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&t);
    uint32_t* d = reinterpret_cast<uint32_t*>(dst);
    for (int i = threadIdx.x; i < (int)(sizeof(JobTable) / 4); i += blockDim.x) d[i] = src[i];
  }
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count; j += (int64_t)gridDim.x * blockDim.x)
    zero[j] = 0u;
}

// Adam on the twist xi = (rho, phi), then V <- exp(-step^) V in binary64.
// state: m[6], v[6], t.
// One wave: lane k < 6 takes twist component k, then lane 0 applies the step.
__global__ void k_pose_adam(float* __restrict__ viewmat, const float* __restrict__ g, float* __restrict__ state,
                            float lr, float b1, float b2, float eps) {
  if (blockIdx.x != 0 || threadIdx.x >= 64) return;
  const int k = (int)threadIdx.x;
  const float t = state[12] + 1.f;   // read by every lane before lane 0 stores it below
  double xk = 0.0;
  if (k < 6) {
    const float m = b1 * state[k] + (1.f - b1) * g[k];
    const float v = b2 * state[6 + k] + (1.f - b2) * g[k] * g[k];
    state[k] = m;
    state[6 + k] = v;
    const double mh = m / (1.0 - pow((double)b1, (double)t));
    const double vh = v / (1.0 - pow((double)b2, (double)t));
    xk = -(double)lr * mh / (sqrt(vh) + (double)eps);
  }
  double xi[6];
  for (int j = 0; j < 6; j++) xi[j] = __shfl(xk, j, 64);
  if (k != 0) return;
  state[12] = t;
  // exp of the se(3) element (rho = xi[0..2], phi = xi[3..5]), Rodrigues form
  const double px = xi[3], py = xi[4], pz = xi[5];
  const double th2 = px * px + py * py + pz * pz, th = sqrt(th2);
  double A, B, C;
  if (th < 1e-8) {
    A = 1.0 - th2 / 6.0;
    B = 0.5 - th2 / 24.0;
    C = 1.0 / 6.0 - th2 / 120.0;
  } else {
    A = sin(th) / th;
    B = (1.0 - cos(th)) / th2;
    C = (th - sin(th)) / (th2 * th);
  }
  const double K[3][3] = {{0, -pz, py}, {pz, 0, -px}, {-py, px, 0}};
  double K2[3][3], Rx[3][3], Vm[3][3];
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      K2[a][b] = K[a][0] * K[0][b] + K[a][1] * K[1][b] + K[a][2] * K[2][b];
      Rx[a][b] = (a == b ? 1.0 : 0.0) + A * K[a][b] + B * K2[a][b];
      Vm[a][b] = (a == b ? 1.0 : 0.0) + B * K[a][b] + C * K2[a][b];
    }
  double V[3][4], out[3][4];
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 4; b++) V[a][b] = viewmat[4 * a + b];
  for (int a = 0; a < 3; a++) {
    for (int b = 0; b < 4; b++) out[a][b] = Rx[a][0] * V[0][b] + Rx[a][1] * V[1][b] + Rx[a][2] * V[2][b];
    out[a][3] += Vm[a][0] * xi[0] + Vm[a][1] * xi[1] + Vm[a][2] * xi[2];
  }
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 4; b++) viewmat[4 * a + b] = (float)out[a][b];
}

}  // namespace

hipError_t launch_l1_grad(const float* const pred[3], const float* const target[3], float* const grad[3], int64_t P,
                          const float scale[3], float* loss, hipStream_t st) {
  if (P <= 0) return hipSuccess;
  L1Planes L;
  bool vec = P % 4 == 0;
  for (int k = 0; k < 3; k++)
    vec = vec && ((uintptr_t)pred[k] % 16 == 0) && ((uintptr_t)target[k] % 16 == 0) && ((uintptr_t)grad[k] % 16 == 0);
  const int64_t unit = vec ? 4 : 1;
  const int64_t counts[3] = {3 * P / unit, P / unit, P / unit};
  int64_t run = 0;
  for (int k = 0; k < 3; k++) {
    L.pred[k] = pred[k];
    L.target[k] = target[k];
    L.grad[k] = grad[k];
    L.scale[k] = scale[k];
    run += counts[k];
    L.end[k] = run;
  }
  int64_t blocks = (run + kLossThreads - 1) / kLossThreads;
  const int64_t max_blocks = loss ? 256 : 4096;   // one atomic per block on the loss
  if (blocks > max_blocks) blocks = max_blocks;
  if (vec)
    hipLaunchKernelGGL(k_l1_grad<true>, dim3((unsigned)blocks), dim3(kLossThreads), 0, st, L, loss);
  else
    hipLaunchKernelGGL(k_l1_grad<false>, dim3((unsigned)blocks), dim3(kLossThreads), 0, st, L, loss);
  return hipGetLastError();
}

hipError_t launch_setup(const JobTable& t, const Plan& p, char* ws, uint32_t* zero, int64_t count, hipStream_t st) {
  static_assert(sizeof(JobTable) % 4 == 0, "job table is copied in 32-bit words");
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_setup, dim3((unsigned)blocks), dim3(256), 0, st, t, at<JobTable>(ws, p.jobs), zero, count);
  return hipGetLastError();
}

hipError_t launch_zero_scalar(float* p, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(1), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_pose_adam(float* viewmat, const float* g, float* state, float lr, float b1, float b2, float eps,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_pose_adam, dim3(1), dim3(64), 0, st, viewmat, g, state, lr, b1, b2, eps);
  return hipGetLastError();
}

}  // namespace ms

// Front-to-back compositing of colour, depth and silhouette (Eq. 2 of the
// paper and its depth / accumulated-opacity analogues), and its adjoint.
//
// Work decomposition (CDNA4, wave64). A workgroup owns one screen tile of
// TILE x TILE pixels; each of its (TILE/8)^2 wavefronts owns one 8x8 pixel
// sub-block (one pixel per lane) and walks the tile's depth-ordered list on
// its own: it stages WB records at a time from HBM/L2 into its private LDS
// slot (one record per lane, converted to sub-block-local form), then every
// lane evaluates the staged Gaussians against its pixel with the staged
// values read as LDS broadcasts. There is no workgroup barrier: each wave
// stops as soon as all 64 of its pixels are done (ballot), and Gaussians
// whose pixel box misses the wave's sub-block are skipped with a scalar
// branch (their staged acceptance bound is -inf).
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

namespace ms {
namespace {

struct Staged {
  float4 geo;    // cu = X0 - ui, cv = Y0 - vi, uf, vf
  float4 conic;  // a, b, c, qcut (-inf when the box misses the sub-block)
  float4 app;    // log2 o, z, r, g
  float4 misc;   // b(lue), rank bits, 0, 0
};

__device__ inline void stage_record(const uint4* __restrict__ rec, uint32_t r, int X0, int Y0, Staged& s) {
  const uint4* src = rec + 4 * (int64_t)r;
  const uint4 q0 = src[0], q1 = src[1], q2 = src[2], q3 = src[3];
  const int ui = (int)q0.x, vi = (int)q0.y;
  const int bx0 = (int)(q3.y & 0xFFFFu), bx1 = (int)(q3.y >> 16);
  const int by0 = (int)(q3.z & 0xFFFFu), by1 = (int)(q3.z >> 16);
  const bool touch = bx0 <= X0 + 7 && bx1 >= X0 && by0 <= Y0 + 7 && by1 >= Y0;
  s.geo = make_float4((float)(X0 - ui), (float)(Y0 - vi), __uint_as_float(q0.z), __uint_as_float(q0.w));
  s.conic = make_float4(__uint_as_float(q1.x), __uint_as_float(q1.y), __uint_as_float(q1.z),
                        touch ? __uint_as_float(q1.w) : -INFINITY);
  s.app = make_float4(__uint_as_float(q2.x), __uint_as_float(q2.y), __uint_as_float(q2.z), __uint_as_float(q2.w));
  s.misc = make_float4(__uint_as_float(q3.x), __uint_as_float(r), 0.f, 0.f);
}

// Pinned acceptance value (binary32; the fused operations are explicit).
__device__ inline float accept_q(const Staged& s, float xf, float yf, float& dx, float& dy, float& t1, float& t2) {
  dx = (xf + s.geo.x) - s.geo.z;   // (x - ui) exactly, then - uf
  dy = (yf + s.geo.y) - s.geo.w;
  t1 = __builtin_fmaf(s.conic.x, dx, s.conic.y * dy);
  t2 = s.conic.z * dy;
  return __builtin_fmaf(t1, t1, t2 * t2);
}

__device__ inline bool wave_skips(const Staged& s) {
  // wave-uniform: all lanes read the same staged value
  return __builtin_amdgcn_readfirstlane(__float_as_int(s.conic.w)) == (int)0xFF800000u;
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int TILE, int WB>
__global__ void __launch_bounds__(64 * (TILE / 8) * (TILE / 8))
    k_composite_fwd(const uint4* __restrict__ rec, const uint32_t* __restrict__ pval,
                    const uint32_t* __restrict__ trange, const uint64_t* __restrict__ counters, int W, int H, int TX,
                    float* __restrict__ rgb, float* __restrict__ depth, float* __restrict__ sil,
                    float* __restrict__ tfinal, uint32_t* __restrict__ last) {
  constexpr int SB = TILE / 8;
  constexpr int NW = SB * SB;
  __shared__ Staged stage[NW][WB];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile_id = blockIdx.x;
  const int tx = tile_id % TX, ty = tile_id / TX;
  const int X0 = tx * TILE + (wave % SB) * 8, Y0 = ty * TILE + (wave / SB) * 8;
  if (X0 >= W || Y0 >= H) return;   // whole sub-block outside the image (wave-uniform)
  const int xl = lane & 7, yl = lane >> 3;
  const int x = X0 + xl, y = Y0 + yl;
  const bool inside = x < W && y < H;
  const bool overflow = counters[C_OVERFLOW] != 0;
  const uint32_t start = overflow ? 0u : trange[2 * tile_id];
  const uint32_t end = overflow ? 0u : trange[2 * tile_id + 1];
  const float xf = (float)xl, yf = (float)yl;
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
  uint32_t lastpos = 0u;
  bool done = !inside;
  Staged* my = stage[wave];
  for (uint32_t b0 = start; b0 < end; b0 += WB) {
    if (!__any(!done)) break;
    const int nb = (int)min((uint32_t)WB, end - b0);
    wave_sync();
    for (int j = lane; j < nb; j += 64) {
      Staged s;
      stage_record(rec, pval[b0 + j], X0, Y0, s);
      my[j] = s;
    }
    wave_sync();
    for (int j = 0; j < nb; j++) {
      const Staged s = my[j];
      if (wave_skips(s)) continue;
      float dx, dy, t1, t2;
      const float q = accept_q(s, xf, yf, dx, dy, t1, t2);
      if (!done && q <= s.conic.w) {
        const float at = __builtin_amdgcn_exp2f(s.app.x - q);
        const float alpha = fminf(kAlphaMax, at);
        const float Tn = T * (1.f - alpha);
        if (Tn < kTMin) {
          done = true;
        } else {
          const float w = alpha * T;
          C0 = __builtin_fmaf(w, s.app.z, C0);
          C1 = __builtin_fmaf(w, s.app.w, C1);
          C2 = __builtin_fmaf(w, s.misc.x, C2);
          D = __builtin_fmaf(w, s.app.y, D);
          T = Tn;
          lastpos = (b0 - start) + (uint32_t)j + 1u;
        }
      }
    }
    if (!__any(!done)) break;
  }
  if (!inside) return;
  const int64_t P = (int64_t)W * H;
  const int64_t pix = (int64_t)y * W + x;
  if (overflow) {
    const float nanv = __builtin_nanf("");
    rgb[pix] = rgb[P + pix] = rgb[2 * P + pix] = nanv;
    depth[pix] = sil[pix] = nanv;
    tfinal[pix] = 1.f;
    last[pix] = 0u;
    return;
  }
  rgb[pix] = C0;
  rgb[P + pix] = C1;
  rgb[2 * P + pix] = C2;
  depth[pix] = D;
  sil[pix] = 1.f - T;
  tfinal[pix] = T;
  last[pix] = lastpos;
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

template <int TILE, int WB>
__global__ void __launch_bounds__(64 * (TILE / 8) * (TILE / 8))
    k_composite_bwd(const uint4* __restrict__ rec, const uint32_t* __restrict__ pval,
                    const uint32_t* __restrict__ trange, const uint64_t* __restrict__ counters, int W, int H, int TX,
                    const float* __restrict__ g_rgb, const float* __restrict__ g_depth,
                    const float* __restrict__ g_sil, const float* __restrict__ tfinal,
                    const uint32_t* __restrict__ last, float* __restrict__ g2d) {
  constexpr int SB = TILE / 8;
  constexpr int NW = SB * SB;
  __shared__ Staged stage[NW][WB];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile_id = blockIdx.x;
  const int tx = tile_id % TX, ty = tile_id / TX;
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
    G0 = g_rgb[pix];
    G1 = g_rgb[P + pix];
    G2 = g_rgb[2 * P + pix];
    GD = g_depth[pix];
    GS = g_sil[pix];
    Tf = tfinal[pix];
    L = last[pix];
  }
  const uint32_t Lmax = wave_max_u32(L);
  const uint32_t start = trange[2 * tile_id];
  const float xf = (float)xl, yf = (float)yl;
  const float GST = GS * Tf;
  float T = Tf;      // transmittance after the current entry
  float R = 0.f;     // suffix sum of (G . c + G_D z) alpha T over later entries
  Staged* my = stage[wave];
  for (uint32_t hi = Lmax; hi > 0;) {
    const uint32_t lo = hi > (uint32_t)WB ? hi - WB : 0u;
    const int nb = (int)(hi - lo);
    wave_sync();
    for (int j = lane; j < nb; j += 64) {
      Staged s;
      stage_record(rec, pval[start + lo + j], X0, Y0, s);
      my[j] = s;
    }
    wave_sync();
    for (int j = nb - 1; j >= 0; j--) {
      const Staged s = my[j];
      if (wave_skips(s)) continue;
      const uint32_t pos = lo + (uint32_t)j;
      float dx, dy, t1, t2;
      const float q = accept_q(s, xf, yf, dx, dy, t1, t2);
      const bool acc = pos < L && q <= s.conic.w;
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

template <int TILE, int WB>
hipError_t fwd_one(const Camera& cam, const Plan& p, char* ws, const ms_images& out, hipStream_t st) {
  constexpr int threads = 64 * (TILE / 8) * (TILE / 8);
  hipLaunchKernelGGL((k_composite_fwd<TILE, WB>), dim3(p.tiles), dim3(threads), 0, st, at<uint4>(ws, p.rec),
                     at<uint32_t>(ws, p.pval), at<uint32_t>(ws, p.trange), at<uint64_t>(ws, p.counters), cam.W,
                     cam.H, p.tx, out.rgb, out.depth, out.silhouette, at<float>(ws, p.tfinal),
                     at<uint32_t>(ws, p.last));
  return hipGetLastError();
}

template <int TILE, int WB>
hipError_t bwd_one(const Camera& cam, const Plan& p, char* ws, const ms_images& g, hipStream_t st) {
  constexpr int threads = 64 * (TILE / 8) * (TILE / 8);
  hipLaunchKernelGGL((k_composite_bwd<TILE, WB>), dim3(p.tiles), dim3(threads), 0, st, at<uint4>(ws, p.rec),
                     at<uint32_t>(ws, p.pval), at<uint32_t>(ws, p.trange), at<uint64_t>(ws, p.counters), cam.W,
                     cam.H, p.tx, g.rgb, g.depth, g.silhouette, at<float>(ws, p.tfinal), at<uint32_t>(ws, p.last),
                     at<float>(ws, p.g2d));
  return hipGetLastError();
}

template <template <int, int> class F>
struct Dispatch;

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

hipError_t launch_composite_fwd(const Camera& cam, const Plan& p, int wave_batch, char* ws, const ms_images& out,
                                hipStream_t st) {
  MS_DISPATCH(fwd_one, cam, p, ws, out, st)
}

hipError_t launch_composite_bwd(const Camera& cam, const Plan& p, int wave_batch, char* ws, const ms_images& gout,
                                hipStream_t st) {
  MS_DISPATCH(bwd_one, cam, p, ws, gout, st)
}

}  // namespace ms

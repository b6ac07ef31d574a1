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
  const float ui = __uint_as_float(q0.x), vi = __uint_as_float(q0.y);
  const int bx0 = (int)(q3.y & 0xFFFFu), bx1 = (int)(q3.y >> 16);
  const int by0 = (int)(q3.z & 0xFFFFu), by1 = (int)(q3.z >> 16);
  const bool touch = bx0 <= X0 + 7 && bx1 >= X0 && by0 <= Y0 + 7 && by1 >= Y0;
  s.geo = make_float4((float)X0 - ui, (float)Y0 - vi, __uint_as_float(q0.z), __uint_as_float(q0.w));
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
    k_composite_fwd(const uint4* __restrict__ rec, const uint32_t* __restrict__ pval, uint32_t rank_mask,
                    const uint32_t* __restrict__ trange, uint64_t* __restrict__ counters_rw, int W, int H, int TX, int BX, int bshift,
                    float* __restrict__ rgb, float* __restrict__ depth, float* __restrict__ sil,
                    float* __restrict__ tfinal, uint32_t* __restrict__ last) {
  constexpr int SB = TILE / 8;
  constexpr int NW = SB * SB;
  __shared__ Staged stage[NW][WB];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile_id = blockIdx.x;
  const int tx = tile_id % TX, ty = tile_id / TX;
  const int bin_id = (tx >> bshift) + (ty >> bshift) * BX;
  const int X0 = tx * TILE + (wave % SB) * 8, Y0 = ty * TILE + (wave / SB) * 8;
  if (X0 >= W || Y0 >= H) return;   // whole sub-block outside the image (wave-uniform)
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
  for (uint32_t b0 = start; b0 < end; b0 += WB) {
    if (!__any(!done)) break;
    const int nb = (int)min((uint32_t)WB, end - b0);
    staged += (uint32_t)nb;
    wave_sync();
    for (int j = lane; j < nb; j += 64) {
      Staged s;
      stage_record(rec, pval[b0 + j] & rank_mask, X0, Y0, s);
      my[j] = s;
    }
    wave_sync();
    for (int j = 0; j < nb; j++) {
      // read only what each step needs: the bound (skip test), then the
      // geometry, then colour and depth when some lane accepted
      const float4 cn = my[j].conic;
      if (__builtin_amdgcn_readfirstlane(__float_as_int(cn.w)) == (int)0xFF800000u) continue;
      const float4 ge = my[j].geo;
      const float dx = (xf + ge.x) - ge.z;
      const float dy = (yf + ge.y) - ge.w;
      const float t1 = __builtin_fmaf(cn.x, dx, cn.y * dy);
      const float t2 = cn.z * dy;
      const float q = __builtin_fmaf(t1, t1, t2 * t2);
      const bool acc = !done && q <= cn.w;
      if (__builtin_amdgcn_ballot_w64(acc) == 0) continue;
      if (acc) {
        const float4 ap = my[j].app;
        const float cb = my[j].misc.x;
        const float at = __builtin_amdgcn_exp2f(ap.x - q);
        const float alpha = fminf(kAlphaMax, at);
        const float Tn = T * (1.f - alpha);
        if (Tn < kTMin) {
          done = true;
        } else {
          const float w = alpha * T;
          C0 = __builtin_fmaf(w, ap.z, C0);
          C1 = __builtin_fmaf(w, ap.w, C1);
          C2 = __builtin_fmaf(w, cb, C2);
          D = __builtin_fmaf(w, ap.y, D);
          T = Tn;
          lastpos = (b0 - start) + (uint32_t)j + 1u;
          ncomp++;
        }
      }
    }
    if (!__any(!done)) break;
  }
  // work counters: one atomic per wave
  uint32_t wsum = ncomp;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) wsum += (uint32_t)__shfl_xor((int)wsum, off, 64);
  if (lane == 0) {
    atomicAdd((unsigned long long*)&counters_rw[C_COMPOSITED], (unsigned long long)wsum);
    atomicAdd((unsigned long long*)&counters_rw[C_STAGED], (unsigned long long)staged);
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
                      const uint32_t* __restrict__ trange, uint64_t* __restrict__ counters_rw, int W, int H, int TX,
                      int BX, int bshift,
                      float* __restrict__ rgb, float* __restrict__ depth, float* __restrict__ sil,
                      float* __restrict__ tfinal, uint32_t* __restrict__ last) {
  constexpr int SB = TILE / 8;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int tile_id = blockIdx.x;
  const int tx = tile_id % TX, ty = tile_id / TX;
  const int bin_id = (tx >> bshift) + (ty >> bshift) * BX;
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
    atomicAdd((unsigned long long*)&counters_rw[C_COMPOSITED], (unsigned long long)wsum);
    atomicAdd((unsigned long long*)&counters_rw[C_STAGED], (unsigned long long)staged);
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
    k_composite_bwd(const uint4* __restrict__ rec, const uint32_t* __restrict__ pval, uint32_t rank_mask,
                    const uint32_t* __restrict__ trange, const uint64_t* __restrict__ counters, int W, int H, int TX, int BX, int bshift,
                    const float* __restrict__ g_rgb, const float* __restrict__ g_depth,
                    const float* __restrict__ g_sil, const float* __restrict__ tfinal,
                    const uint32_t* __restrict__ last, float* __restrict__ g2d) {
  constexpr int SB = TILE / 8;
  constexpr int NW = SB * SB;
  __shared__ Staged stage[NW][WB];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile_id = blockIdx.x;
  const int tx = tile_id % TX, ty = tile_id / TX;
  const int bin_id = (tx >> bshift) + (ty >> bshift) * BX;
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
  const uint32_t start = trange[2 * bin_id];
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
      stage_record(rec, pval[start + lo + j] & rank_mask, X0, Y0, s);
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
                      const uint32_t* __restrict__ trange, uint64_t* __restrict__ counters_rw, int W, int H,
                      int TX, int BX, int bshift, const float* __restrict__ g_rgb, const float* __restrict__ g_depth,
                      const float* __restrict__ g_sil, const float* __restrict__ tfinal,
                      const uint32_t* __restrict__ last, float* __restrict__ g2d) {
  constexpr int SB = TILE / 8;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int tile_id = blockIdx.x;
  const int tx = tile_id % TX, ty = tile_id / TX;
  const int bin_id = (tx >> bshift) + (ty >> bshift) * BX;
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
    G0 = g_rgb[pix];
    G1 = g_rgb[P + pix];
    G2 = g_rgb[2 * P + pix];
    GD = g_depth[pix];
    GS = g_sil[pix];
    Tf = tfinal[pix];
    L = last[pix];
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
  if (lane == 0) atomicAdd((unsigned long long*)&counters_rw[C_REDUCED], (unsigned long long)reduced);
}

// Backward with the per-Gaussian reduction over the wave's 64 pixels done on
// the matrix cores. For a group of 16 Gaussians with accepting pixels, each
// pixel lane stores e = dL/dalpha * alpha~ and w = alpha T to LDS. All ten
// screen-space sums of a Gaussian are linear in the moments
//   sum_p e_p (1, x, y, x^2, xy, y^2)   and   sum_p w_p (G_r, G_g, G_b, G_D)
// (x, y pixel coordinates about the sub-block centre), i.e. a (16 Gaussians x
// 64 pixels) x (64 pixels x 16 columns) product: sixteen
// v_mfma_f32_16x16x4_f32 steps per product, K = 4 pixels per step. One lane
// per Gaussian then forms the ten sums from the moments and issues the
// atomics. This replaces ten full-wave reductions per Gaussian.
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kGrp = 16;
constexpr int kRow = 68;                               // padded row of 64 pixel values (bank spread)
constexpr int kWaveLds = 2 * kGrp * kRow + kGrp * 8;   // floats per wave: E, W, parameters

template <int TILE>
__global__ void __launch_bounds__(64 * (TILE / 8) * (TILE / 8))
    k_composite_bwd_m(const uint4* __restrict__ rec, const uint32_t* __restrict__ pval, uint32_t rank_mask,
                      const uint32_t* __restrict__ trange, uint64_t* __restrict__ counters_rw, int W, int H,
                      int TX, int BX, int bshift, const float* __restrict__ g_rgb, const float* __restrict__ g_depth,
                      const float* __restrict__ g_sil, const float* __restrict__ tfinal,
                      const uint32_t* __restrict__ last, float* __restrict__ g2d) {
  constexpr int SB = TILE / 8;
  constexpr int NW = SB * SB;
  __shared__ __attribute__((aligned(16))) float lds[NW * kWaveLds];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int tile_id = blockIdx.x;
  const int tx = tile_id % TX, ty = tile_id / TX;
  const int bin_id = (tx >> bshift) + (ty >> bshift) * BX;
  const int X0 = tx * TILE + (wave % SB) * 8, Y0 = ty * TILE + (wave / SB) * 8;
  if (X0 >= W || Y0 >= H) return;
  if (counters_rw[C_OVERFLOW] != 0) return;
  float* Ew = lds + wave * kWaveLds;   // [16 Gaussians][4 k][16 s] (row stride kRow), pixel p = 4 s + k
  float* Ww = Ew + kGrp * kRow;
  float* Pw = Ww + kGrp * kRow;        // [16][8]: rank bits, U, V, a, b, c
  const int x = X0 + (lane & 7), y = Y0 + (lane >> 3);
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
  // B operands (constant per wave): lane holds B[k = lane / 16][j = lane % 16]
  // of step s, i.e. column j for pixel 4 s + k.
  const int pk = lane >> 4, pj = lane & 15;
  float Bm[16], Bu[16];
  Ew[lane * 4 + 0] = G0;
  Ew[lane * 4 + 1] = G1;
  Ew[lane * 4 + 2] = G2;
  Ew[lane * 4 + 3] = GD;
  wave_sync();
#pragma unroll
  for (int st = 0; st < 16; st++) {
    const int p = 4 * st + pk;
    const float px = (float)(p & 7) - 3.5f, py = (float)(p >> 3) - 3.5f;
    float m = 0.f;
    m = pj == 0 ? 1.f : m;
    m = pj == 1 ? px : m;
    m = pj == 2 ? py : m;
    m = pj == 3 ? px * px : m;
    m = pj == 4 ? px * py : m;
    m = pj == 5 ? py * py : m;
    Bm[st] = m;
    Bu[st] = pj < 4 ? Ew[p * 4 + (pj & 3)] : 0.f;
  }
  wave_sync();
  const uint32_t Lmax = __builtin_amdgcn_readfirstlane(wave_max_u32(L));
  const uint32_t start = trange[2 * bin_id];
  const float xa = (float)x, ya = (float)y;
  const float GST = GS * Tf;
  float T = Tf;
  float R = 0.f;
  uint32_t reduced = 0u;
  int ng = 0;
  const int eaddr = (lane & 3) * 16 + (lane >> 2);
  auto flush = [&](int count) {
    wave_sync();
    float a1[16], a2[16];
    const float4* e4 = reinterpret_cast<const float4*>(Ew + pj * kRow + pk * 16);
    const float4* w4 = reinterpret_cast<const float4*>(Ww + pj * kRow + pk * 16);
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const float4 ev = e4[q], wv = w4[q];
      a1[4 * q] = ev.x; a1[4 * q + 1] = ev.y; a1[4 * q + 2] = ev.z; a1[4 * q + 3] = ev.w;
      a2[4 * q] = wv.x; a2[4 * q + 1] = wv.y; a2[4 * q + 2] = wv.z; a2[4 * q + 3] = wv.w;
    }
    f32x4 d1 = {0.f, 0.f, 0.f, 0.f}, d2 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int st = 0; st < 16; st++) {
      d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[st], Bm[st], d1, 0, 0, 0);
      d2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[st], Bu[st], d2, 0, 0, 0);
    }
    wave_sync();
#pragma unroll
    for (int r = 0; r < 4; r++) {
      Ew[(4 * pk + r) * 16 + pj] = d1[r];
      Ww[(4 * pk + r) * 16 + pj] = d2[r];
    }
    wave_sync();
    // one lane per Gaussian forms the ten sums; they go back to LDS so that
    // each atomic instruction covers whole Gaussians (10 consecutive floats)
    float* F = Ww + kGrp * 16;         // [16][10], after the 16x16 D2 block
    if (lane < count) {
      const float* m = Ew + lane * 16;
      const float* u = Ww + lane * 16;
      const float* pr = Pw + lane * 8;
      const float S1 = m[0], Sx = m[1], Sy = m[2], Sxx = m[3], Sxy = m[4], Syy = m[5];
      const float U = pr[1], V = pr[2], a = pr[3], b = pr[4], c = pr[5];
      const float Edx = Sx - U * S1, Edy = Sy - V * S1;
      const float Edxx = Sxx - 2.f * U * Sx + U * U * S1;
      const float Edxy = Sxy - V * Sx - U * Sy + U * V * S1;
      const float Edyy = Syy - 2.f * V * Sy + V * V * S1;
      float* f = F + lane * kGradFields;
      f[0] = S1;
      f[1] = a * Edx + b * Edy;
      f[2] = c * Edy;
      f[3] = a * Edxx + b * Edxy;
      f[4] = a * Edxy + b * Edyy;
      f[5] = c * Edyy;
      f[6] = u[0];
      f[7] = u[1];
      f[8] = u[2];
      f[9] = u[3];
    }
    wave_sync();
    for (int idx = lane; idx < count * kGradFields; idx += 64) {
      const int g = idx / kGradFields, fi = idx - g * kGradFields;
      unsafeAtomicAdd(g2d + (int64_t)__float_as_uint(Pw[g * 8]) * kGradFields + fi, F[idx]);
    }
    wave_sync();
  };
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
      float e = 0.f, w = 0.f;
      if (acc) {
        const float at = __builtin_amdgcn_exp2f(s.lo2 - q);
        const float alpha = fminf(kAlphaMax, at);
        const float inv = __builtin_amdgcn_rcpf(1.f - alpha);
        const float Tk = T * inv;
        w = alpha * Tk;
        const float gcz = __builtin_fmaf(G0, s.cr, __builtin_fmaf(G1, s.cg, __builtin_fmaf(G2, s.cb, GD * s.z)));
        const float dalpha = __builtin_fmaf(Tk, gcz, -(R - GST) * inv);
        e = at > kAlphaMax ? 0.f : dalpha * at;
        R = __builtin_fmaf(gcz, w, R);
        T = Tk;
      }
      Ew[ng * kRow + eaddr] = e;
      Ww[ng * kRow + eaddr] = w;
      if (lane == 0) {
        float* pr = Pw + ng * 8;
        pr[0] = __uint_as_float(rk[i]);
        pr[1] = ((s.ui - (float)X0) - 3.5f) + s.uf;
        pr[2] = ((s.vi - (float)Y0) - 3.5f) + s.vf;
        pr[3] = s.a;
        pr[4] = s.b;
        pr[5] = s.c;
      }
      if (++ng == kGrp) {
        flush(kGrp);
        ng = 0;
      }
    }
    hi = lo;
  }
  if (ng > 0) flush(ng);
  if (lane == 0) atomicAdd((unsigned long long*)&counters_rw[C_REDUCED], (unsigned long long)reduced);
}

template <int TILE>
hipError_t bwd_mfma(const Camera& cam, const Plan& p, char* ws, const ms_images& g, hipStream_t st) {
  constexpr int threads = 64 * (TILE / 8) * (TILE / 8);
  hipLaunchKernelGGL((k_composite_bwd_m<TILE>), dim3(p.tiles), dim3(threads), 0, st, at<uint4>(ws, p.rec),
                     at<uint32_t>(ws, p.pval), rank_mask(p), at<uint32_t>(ws, p.trange), at<uint64_t>(ws, p.counters),
                     cam.W, cam.H, p.tx, p.bx, p.bshift, g.rgb, g.depth, g.silhouette, at<float>(ws, p.tfinal),
                     at<uint32_t>(ws, p.last), at<float>(ws, p.g2d));
  return hipGetLastError();
}

template <int TILE>
hipError_t bwd_scalar(const Camera& cam, const Plan& p, char* ws, const ms_images& g, hipStream_t st) {
  constexpr int threads = 64 * (TILE / 8) * (TILE / 8);
  hipLaunchKernelGGL((k_composite_bwd_s<TILE>), dim3(p.tiles), dim3(threads), 0, st, at<uint4>(ws, p.rec),
                     at<uint32_t>(ws, p.pval), rank_mask(p), at<uint32_t>(ws, p.trange), at<uint64_t>(ws, p.counters),
                     cam.W, cam.H, p.tx, p.bx, p.bshift, g.rgb, g.depth, g.silhouette, at<float>(ws, p.tfinal),
                     at<uint32_t>(ws, p.last), at<float>(ws, p.g2d));
  return hipGetLastError();
}

template <int TILE, int WB>
hipError_t fwd_one(const Camera& cam, const Plan& p, char* ws, const ms_images& out, hipStream_t st) {
  constexpr int threads = 64 * (TILE / 8) * (TILE / 8);
  hipLaunchKernelGGL((k_composite_fwd<TILE, WB>), dim3(p.tiles), dim3(threads), 0, st, at<uint4>(ws, p.rec),
                     at<uint32_t>(ws, p.pval), rank_mask(p), at<uint32_t>(ws, p.trange), at<uint64_t>(ws, p.counters), cam.W,
                     cam.H, p.tx, p.bx, p.bshift, out.rgb, out.depth, out.silhouette, at<float>(ws, p.tfinal),
                     at<uint32_t>(ws, p.last));
  return hipGetLastError();
}

template <int TILE, int WB>
hipError_t bwd_one(const Camera& cam, const Plan& p, char* ws, const ms_images& g, hipStream_t st) {
  constexpr int threads = 64 * (TILE / 8) * (TILE / 8);
  hipLaunchKernelGGL((k_composite_bwd<TILE, WB>), dim3(p.tiles), dim3(threads), 0, st, at<uint4>(ws, p.rec),
                     at<uint32_t>(ws, p.pval), rank_mask(p), at<uint32_t>(ws, p.trange), at<uint64_t>(ws, p.counters), cam.W,
                     cam.H, p.tx, p.bx, p.bshift, g.rgb, g.depth, g.silhouette, at<float>(ws, p.tfinal), at<uint32_t>(ws, p.last),
                     at<float>(ws, p.g2d));
  return hipGetLastError();
}

template <int TILE>
hipError_t fwd_scalar(const Camera& cam, const Plan& p, char* ws, const ms_images& out, hipStream_t st) {
  constexpr int threads = 64 * (TILE / 8) * (TILE / 8);
  hipLaunchKernelGGL((k_composite_fwd_s<TILE>), dim3(p.tiles), dim3(threads), 0, st, at<uint4>(ws, p.rec),
                     at<uint32_t>(ws, p.pval), rank_mask(p), at<uint32_t>(ws, p.trange), at<uint64_t>(ws, p.counters),
                     cam.W, cam.H, p.tx, p.bx, p.bshift, out.rgb, out.depth, out.silhouette, at<float>(ws, p.tfinal),
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

hipError_t launch_composite_fwd(const Camera& cam, const Plan& p, int wave_batch, uint32_t flags, char* ws,
                                const ms_images& out, hipStream_t st) {
  if (flags & MS_FLAG_SCALAR_FWD) {
    switch (p.tile) {
      case 8: return fwd_scalar<8>(cam, p, ws, out, st);
      case 16: return fwd_scalar<16>(cam, p, ws, out, st);
      case 32: return fwd_scalar<32>(cam, p, ws, out, st);
      default: return hipErrorInvalidValue;
    }
  }
  MS_DISPATCH(fwd_one, cam, p, ws, out, st)
}

hipError_t launch_composite_bwd(const Camera& cam, const Plan& p, int wave_batch, uint32_t flags, char* ws,
                                const ms_images& gout, hipStream_t st) {
  if (flags & MS_FLAG_MFMA_BWD) {
    switch (p.tile) {
      case 8: return bwd_mfma<8>(cam, p, ws, gout, st);
      case 16: return bwd_mfma<16>(cam, p, ws, gout, st);
      default: return hipErrorInvalidValue;
    }
  }
  if (flags & MS_FLAG_SCALAR_BWD) {
    switch (p.tile) {
      case 8: return bwd_scalar<8>(cam, p, ws, gout, st);
      case 16: return bwd_scalar<16>(cam, p, ws, gout, st);
      case 32: return bwd_scalar<32>(cam, p, ws, gout, st);
      default: return hipErrorInvalidValue;
    }
  }
  MS_DISPATCH(bwd_one, cam, p, ws, gout, st)
}

}  // namespace ms

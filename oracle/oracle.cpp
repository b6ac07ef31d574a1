// CPU oracle for the differentiable RGB-D Gaussian rasterizer.
//
// TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
// benchmark's CPU-baseline leg may load this library. It shares no code with
// the GPU path; it is written from the paper and from the plain mathematics of
// EWA splatting and "over" compositing, in double precision, with scalar loops.
//
// What it computes (MAC-Ego3D, Sec. 3.3, Eq. 2): each pixel's colour is the sum
// over the Gaussians covering it, in front-to-back order, of colour times that
// Gaussian's projected opacity times the product of (1 - opacity) of the
// Gaussians in front of it. Depth (Sec. 3.5, Eq. 7 renders depths the same way)
// replaces colour by the camera-frame depth; the silhouette is 1 minus the
// final transmittance. The backward pass differentiates these sums (Sec. 3.4
// "Optimization", Sec. 3.5 "Optimization": gradients through differentiable
// rendering to the map and the poses).
//
// The paper leaves the projection f_i^proj undefined. The readings used here:
//   * EWA local-affine projection: Sigma' = J R Sigma R^T J^T + 0.3 I (px^2),
//     Sigma = Rq(q/|q|) diag(s)^2 Rq^T, J the perspective Jacobian with the
//     normalised image coordinate clamped to 1.3x the half field of view;
//   * alpha = min(0.99, o * exp(-d^2/2)), d^2 the Mahalanobis distance under
//     Sigma'; a Gaussian counts at a pixel only if d^2 <= 9 and the unclamped
//     alpha >= 1/255;
//   * compositing stops before the Gaussian whose inclusion would drop the
//     transmittance below 1e-4 (that Gaussian is not composited);
//   * depth D = sum z alpha T (not normalised), silhouette S = 1 - T_final,
//     background 0, pixel (x, y) sampled at integer coordinates.
//
// Discrete structure. Which Gaussians are visible, their screen boxes, their
// depth order and which (pixel, Gaussian) pairs pass the two cut-offs are
// integer outcomes of floating-point tests. They are *defined* by a pinned
// evaluation order (the "pinned recipe" below: binary64 without fused
// multiply-add for the projection, binary32 with the stated fused
// multiply-adds for the per-pixel test) so that any implementation that
// follows the same order obtains bit-identical decisions. All continuous
// values (alpha, transmittance, colour, depth, silhouette, gradients) are
// computed here in double precision from the plain definition.
//
// The only acceleration is bucketing candidate Gaussians by 16x16 pixel
// blocks before the per-pixel walk; a Gaussian whose pixel box does not
// contain a pixel is never a candidate for it, so the bucketing cannot change
// any result. OpenMP parallelises over pixel rows.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

// ----------------------------------------------------------------- constants
// sqrt(0.5 * log2(e)): scales the Mahalanobis factors so that q = d^2/2*log2(e).
const double KAPPA = 0x1.b2da4e9808a53p-1;
// 4.5 * log2(e): q at d^2 = 9 (the 3-sigma footprint).
const double Q9 = 0x1.9f7f051d0f35ep+2;
const double LOG2E = 0x1.71547652b82fep+0;
// Pixel-box half-extent factor: 3 sigma enlarged by 2^-8 so that the binary32
// per-pixel test can never accept a pixel outside the box.
const double BOX_SIGMAS = 3.01171875;
const double DILATION = 0.3;
const double GUARD = 0.65;          // 1.3 x half field of view
const double ALPHA_MAX = 0.99;
const double T_MIN = 1e-4;
const double CENTRE_LIMIT = 4194304.0;   // 2^22 px
const double SIGMA2_LIMIT = 4194304.0;   // 2^22 px^2

// Margins of the ambiguity flags (relative).
const double MARGIN_STOP = 1e-4;
const double MARGIN_CLAMP = 1e-4;

struct Cam {
  int W, H;
  double fx, fy, cx, cy, near_z;
  double R[3][3], t[3];
};

Cam make_cam(const double* V, int W, int H, double fx, double fy, double cx, double cy, double near_z) {
  Cam c;
  c.W = W; c.H = H; c.fx = fx; c.fy = fy; c.cx = cx; c.cy = cy; c.near_z = near_z;
  for (int i = 0; i < 3; i++) {
    for (int j = 0; j < 3; j++) c.R[i][j] = V[4 * i + j];
    c.t[i] = V[4 * i + 3];
  }
  return c;
}

// Pinned log2 for x > 0: frexp, fold the mantissa into [sqrt(2)/2, sqrt(2)],
// then ln m = 2 atanh((m-1)/(m+1)) by its Taylor series (terms to y^23),
// Horner order, binary64, no fused multiply-add.
double pinned_log2(double x) {
  int e;
  double m = std::frexp(x, &e);   // x = m 2^e, m in [0.5, 1)
  m = m * 2.0;
  e = e - 1;
  if (m > 1.4142135623730951) {
    m = m * 0.5;
    e = e + 1;
  }
  double y = (m - 1.0) / (m + 1.0);
  double y2 = y * y;
  double p = 1.0 / 23.0;
  for (int k = 10; k >= 0; k--) p = p * y2 + 1.0 / (double)(2 * k + 1);
  double ln_m = 2.0 * y * p;
  return (double)e + ln_m * LOG2E;
}

// Output of the pinned projection recipe for one Gaussian.
struct Pinned {
  bool visible;
  uint32_t zkey;
  float z32;
  int32_t xlo, xhi, ylo, yhi;   // pixel box, clamped to the image
  int32_t ui, vi;               // floor of the centre
  float uf, vf;                 // centre minus its floor
  float a, b, c;                // scaled Cholesky factors of the conic
  float qcut;                   // per-pixel acceptance bound on q
};

// The pinned recipe. Binary64, round to nearest, no fused multiply-add,
// each sum evaluated left to right as written.
Pinned pinned_project(const double mu[3], const double s[3], const double q[4], double o, const double col[3],
                      const Cam& cam) {
  Pinned P;
  std::memset(&P, 0, sizeof(P));
  P.visible = false;
  const double (*R)[3] = cam.R;
  double p[3];
  for (int i = 0; i < 3; i++) p[i] = ((R[i][0] * mu[0] + R[i][1] * mu[1]) + R[i][2] * mu[2]) + cam.t[i];
  if (!(p[2] > cam.near_z)) return P;
  if (!std::isfinite(p[0]) || !std::isfinite(p[1]) || !std::isfinite(p[2])) return P;
  if (!std::isfinite(o) || !std::isfinite(s[0]) || !std::isfinite(s[1]) || !std::isfinite(s[2])) return P;
  // a Gaussian with a non-finite attribute is culled, colour included
  if (!std::isfinite(col[0]) || !std::isfinite(col[1]) || !std::isfinite(col[2])) return P;
  double n2 = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
  if (!(n2 > 0.0) || !std::isfinite(n2)) return P;
  double rn = 1.0 / std::sqrt(n2);
  double w = q[0] * rn, x = q[1] * rn, y = q[2] * rn, z = q[3] * rn;
  double xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
  double wx = w * x, wy = w * y, wz = w * z;
  double Rq[3][3] = {
      {1.0 - 2.0 * (yy + zz), 2.0 * (xy - wz), 2.0 * (xz + wy)},
      {2.0 * (xy + wz), 1.0 - 2.0 * (xx + zz), 2.0 * (yz - wx)},
      {2.0 * (xz - wy), 2.0 * (yz + wx), 1.0 - 2.0 * (xx + yy)}};
  double M[3][3], Wm[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) M[i][j] = Rq[i][j] * s[j];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) Wm[i][j] = (R[i][0] * M[0][j] + R[i][1] * M[1][j]) + R[i][2] * M[2][j];
  double rz = 1.0 / p[2];
  double xn = p[0] * rz, yn = p[1] * rz;
  double limx = (GUARD * (double)cam.W) / cam.fx;
  double limy = (GUARD * (double)cam.H) / cam.fy;
  double xc = std::min(std::max(xn, -limx), limx);
  double yc = std::min(std::max(yn, -limy), limy);
  double j00 = cam.fx * rz, j02 = -((cam.fx * xc) * rz);
  double j11 = cam.fy * rz, j12 = -((cam.fy * yc) * rz);
  double V0[3], V1[3];
  for (int k = 0; k < 3; k++) {
    V0[k] = j00 * Wm[0][k] + j02 * Wm[2][k];
    V1[k] = j11 * Wm[1][k] + j12 * Wm[2][k];
  }
  double S00 = ((V0[0] * V0[0] + V0[1] * V0[1]) + V0[2] * V0[2]) + DILATION;
  double S01 = (V0[0] * V1[0] + V0[1] * V1[1]) + V0[2] * V1[2];
  double S11 = ((V1[0] * V1[0] + V1[1] * V1[1]) + V1[2] * V1[2]) + DILATION;
  if (!(S00 <= SIGMA2_LIMIT) || !(S11 <= SIGMA2_LIMIT) || !std::isfinite(S01)) return P;
  double u = cam.fx * xn + cam.cx;
  double v = cam.fy * yn + cam.cy;
  if (!(std::fabs(u) <= CENTRE_LIMIT) || !(std::fabs(v) <= CENTRE_LIMIT)) return P;
  double rx = std::ceil(BOX_SIGMAS * std::sqrt(S00));
  double ry = std::ceil(BOX_SIGMAS * std::sqrt(S11));
  double xlo = std::ceil(u - rx), xhi = std::floor(u + rx);
  double ylo = std::ceil(v - ry), yhi = std::floor(v + ry);
  if (!(xlo <= (double)(cam.W - 1)) || !(xhi >= 0.0) || !(ylo <= (double)(cam.H - 1)) || !(yhi >= 0.0)) return P;
  double det = S00 * S11 - S01 * S01;
  if (!(det > 0.0)) return P;
  float z32 = (float)p[2];
  if (!std::isfinite(z32)) return P;
  double sd = std::sqrt(det), s11 = std::sqrt(S11);
  double l11 = s11 / sd;
  double l12 = -S01 / (sd * s11);
  double l22 = 1.0 / s11;
  double ufl = std::floor(u), vfl = std::floor(v);
  double lo255 = 255.0 * o;
  double qc = (lo255 > 0.0) ? std::min(Q9, pinned_log2(lo255)) : -INFINITY;

  P.visible = true;
  P.z32 = z32;
  std::memcpy(&P.zkey, &z32, 4);
  P.xlo = (int32_t)std::max(xlo, 0.0);
  P.xhi = (int32_t)std::min(xhi, (double)(cam.W - 1));
  P.ylo = (int32_t)std::max(ylo, 0.0);
  P.yhi = (int32_t)std::min(yhi, (double)(cam.H - 1));
  P.ui = (int32_t)ufl;
  P.vi = (int32_t)vfl;
  P.uf = (float)(u - ufl);
  P.vf = (float)(v - vfl);
  P.a = (float)(KAPPA * l11);
  P.b = (float)(KAPPA * l12);
  P.c = (float)(KAPPA * l22);
  P.qcut = (float)qc;
  return P;
}

// Pinned per-pixel test value: binary32, fused multiply-add where written.
inline float pinned_q(const Pinned& P, int x, int y) {
  float dx = (float)(x - P.ui) - P.uf;
  float dy = (float)(y - P.vi) - P.vf;
  float t1 = std::fmaf(P.a, dx, P.b * dy);
  float t2 = P.c * dy;
  return std::fmaf(t1, t1, t2 * t2);
}

// ---------------------------------------------------------- plain definition
// Continuous projection of one Gaussian, straight from the definition
// (matrices written out, double precision). `clamp_state` receives or (when
// frozen) imposes the branch of the field-of-view clamp: -1, 0, +1 per axis.
struct Cont {
  double p[3];
  double Rq[3][3];
  double Sigma[3][3];
  double Sc[3][3];
  double J[2][3];
  double S[2][2];          // Sigma'
  double Q[2][2];          // conic = inverse of Sigma'
  double u, v;
  double qn[4], qnorm;
  int clampx, clampy;
  double limx, limy;
};

void mat3_mul(const double A[3][3], const double B[3][3], double C[3][3]) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double acc = 0.0;
      for (int k = 0; k < 3; k++) acc += A[i][k] * B[k][j];
      C[i][j] = acc;
    }
}

void cont_project(const double mu[3], const double s[3], const double q[4], const Cam& cam,
                  bool frozen, int fcx, int fcy, Cont& c) {
  for (int i = 0; i < 3; i++) {
    double acc = cam.t[i];
    for (int j = 0; j < 3; j++) acc += cam.R[i][j] * mu[j];
    c.p[i] = acc;
  }
  c.qnorm = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; k++) c.qn[k] = q[k] / c.qnorm;
  double w = c.qn[0], x = c.qn[1], y = c.qn[2], z = c.qn[3];
  // Rotation matrix of the unit quaternion (w, x, y, z).
  double Rq[3][3] = {
      {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
      {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
      {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
  std::memcpy(c.Rq, Rq, sizeof(Rq));
  // Sigma = Rq diag(s^2) Rq^T
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double acc = 0.0;
      for (int k = 0; k < 3; k++) acc += Rq[i][k] * s[k] * s[k] * Rq[j][k];
      c.Sigma[i][j] = acc;
    }
  // Sigma_c = R Sigma R^T
  double RS[3][3], Rt[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) Rt[i][j] = cam.R[j][i];
  mat3_mul(cam.R, c.Sigma, RS);
  mat3_mul(RS, Rt, c.Sc);
  double X = c.p[0], Y = c.p[1], Z = c.p[2];
  c.limx = GUARD * cam.W / cam.fx;
  c.limy = GUARD * cam.H / cam.fy;
  if (!frozen) {
    double xn = X / Z, yn = Y / Z;
    c.clampx = xn < -c.limx ? -1 : (xn > c.limx ? 1 : 0);
    c.clampy = yn < -c.limy ? -1 : (yn > c.limy ? 1 : 0);
  } else {
    c.clampx = fcx;
    c.clampy = fcy;
  }
  double xt = c.clampx == 0 ? X : Z * c.clampx * c.limx;
  double yt = c.clampy == 0 ? Y : Z * c.clampy * c.limy;
  c.J[0][0] = cam.fx / Z; c.J[0][1] = 0; c.J[0][2] = -cam.fx * xt / (Z * Z);
  c.J[1][0] = 0; c.J[1][1] = cam.fy / Z; c.J[1][2] = -cam.fy * yt / (Z * Z);
  for (int a = 0; a < 2; a++)
    for (int b = 0; b < 2; b++) {
      double acc = 0.0;
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) acc += c.J[a][i] * c.Sc[i][j] * c.J[b][j];
      c.S[a][b] = acc + (a == b ? DILATION : 0.0);
    }
  double det = c.S[0][0] * c.S[1][1] - c.S[0][1] * c.S[1][0];
  c.Q[0][0] = c.S[1][1] / det;
  c.Q[1][1] = c.S[0][0] / det;
  c.Q[0][1] = -c.S[0][1] / det;
  c.Q[1][0] = -c.S[1][0] / det;
  c.u = cam.fx * X / Z + cam.cx;
  c.v = cam.fy * Y / Z + cam.cy;
}

// Exponent of the Gaussian at pixel (x, y): -d^2/2.
inline double power_at(const Cont& c, int x, int y, double& dx, double& dy) {
  dx = (double)x - c.u;
  dy = (double)y - c.v;
  return -0.5 * (c.Q[0][0] * dx * dx + 2.0 * c.Q[0][1] * dx * dy + c.Q[1][1] * dy * dy);
}

struct Inputs {
  int64_t n;
  const double *means, *scales, *quats, *opac, *colors;   // SoA, double
};

inline void gather(const Inputs& in, int64_t i, double mu[3], double s[3], double q[4], double& o, double col[3]) {
  const int64_t n = in.n;
  for (int k = 0; k < 3; k++) {
    mu[k] = in.means[k * n + i];
    s[k] = in.scales[k * n + i];
    col[k] = in.colors[k * n + i];
  }
  for (int k = 0; k < 4; k++) q[k] = in.quats[k * n + i];
  o = in.opac[i];
}

// Per-scene precomputation: pinned records, continuous projections and the
// 16x16-pixel candidate buckets (each bucket sorted by (zkey, index)).
struct Prepared {
  std::vector<Pinned> pin;
  std::vector<Cont> cont;
  std::vector<double> col;       // [n][3]
  std::vector<double> opac;
  int bx, by;                    // bucket grid
  std::vector<std::vector<int32_t>> buckets;
};

const int BUCKET = 16;

void prepare(const Inputs& in, const Cam& cam, Prepared& pr, const int8_t* frozen_clamp, int nthreads) {
  const int64_t n = in.n;
  pr.pin.assign(n, Pinned());
  pr.cont.assign(n, Cont());
  pr.col.assign(3 * n, 0.0);
  pr.opac.assign(n, 0.0);
#pragma omp parallel for num_threads(nthreads) schedule(static)
  for (int64_t i = 0; i < n; i++) {
    double mu[3], s[3], q[4], o, col[3];
    gather(in, i, mu, s, q, o, col);
    pr.pin[i] = pinned_project(mu, s, q, o, col, cam);
    for (int k = 0; k < 3; k++) pr.col[3 * i + k] = col[k];
    pr.opac[i] = o;
    if (pr.pin[i].visible) {
      if (frozen_clamp)
        cont_project(mu, s, q, cam, true, frozen_clamp[2 * i], frozen_clamp[2 * i + 1], pr.cont[i]);
      else
        cont_project(mu, s, q, cam, false, 0, 0, pr.cont[i]);
    }
  }
  pr.bx = (cam.W + BUCKET - 1) / BUCKET;
  pr.by = (cam.H + BUCKET - 1) / BUCKET;
  pr.buckets.assign((size_t)pr.bx * pr.by, std::vector<int32_t>());
  for (int64_t i = 0; i < n; i++) {
    const Pinned& P = pr.pin[i];
    if (!P.visible) continue;
    for (int ty = P.ylo / BUCKET; ty <= P.yhi / BUCKET; ty++)
      for (int tx = P.xlo / BUCKET; tx <= P.xhi / BUCKET; tx++) pr.buckets[(size_t)ty * pr.bx + tx].push_back((int32_t)i);
  }
  const std::vector<Pinned>& pin = pr.pin;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 4)
  for (int64_t b = 0; b < (int64_t)pr.buckets.size(); b++) {
    std::stable_sort(pr.buckets[b].begin(), pr.buckets[b].end(),
                     [&](int32_t i, int32_t j) { return pin[i].zkey < pin[j].zkey; });
  }
}

// Per-pixel walk: the composited list of one pixel.
struct Hit {
  int32_t id;
  double alpha, atil, T, power, dx, dy;
  bool clamped;
};

struct PixelResult {
  double C[3], D, T;
  int64_t evaluated, accepted;
  uint8_t flags;
  int32_t stop_id, clamp_id;
};

enum { FLAG_STOP = 1, FLAG_CLAMP = 2 };

void walk_pixel(const Prepared& pr, const Cam& cam, int x, int y, std::vector<Hit>& hits, PixelResult& r) {
  hits.clear();
  r.C[0] = r.C[1] = r.C[2] = 0.0;
  r.D = 0.0;
  r.T = 1.0;
  r.evaluated = r.accepted = 0;
  r.flags = 0;
  r.stop_id = r.clamp_id = -1;
  const std::vector<int32_t>& cand = pr.buckets[(size_t)(y / BUCKET) * pr.bx + (x / BUCKET)];
  double T = 1.0;
  for (int32_t id : cand) {
    const Pinned& P = pr.pin[id];
    if (x < P.xlo || x > P.xhi || y < P.ylo || y > P.yhi) continue;
    r.evaluated++;
    if (!(pinned_q(P, x, y) <= P.qcut)) continue;
    r.accepted++;
    const Cont& c = pr.cont[id];
    double dx, dy;
    double pw = power_at(c, x, y, dx, dy);
    double atil = pr.opac[id] * std::exp(pw);
    double alpha = std::min(ALPHA_MAX, atil);
    double Tn = T * (1.0 - alpha);
    if (Tn < T_MIN) {
      if (Tn >= T_MIN * (1.0 - MARGIN_STOP)) { r.flags |= FLAG_STOP; r.stop_id = id; }
      break;
    }
    if (std::fabs(atil - ALPHA_MAX) <= ALPHA_MAX * MARGIN_CLAMP) { r.flags |= FLAG_CLAMP; r.clamp_id = id; }
    Hit h;
    h.id = id; h.alpha = alpha; h.atil = atil; h.T = T; h.power = pw; h.dx = dx; h.dy = dy;
    h.clamped = atil > ALPHA_MAX;
    hits.push_back(h);
    for (int k = 0; k < 3; k++) r.C[k] += pr.col[3 * id + k] * alpha * T;
    r.D += c.p[2] * alpha * T;
    T = Tn;
  }
  if (T <= T_MIN * (1.0 + MARGIN_STOP)) {
    r.flags |= FLAG_STOP;
    if (!hits.empty()) r.stop_id = hits.back().id;
  }
  r.T = T;
}

// Per-Gaussian accumulators of the pixel-level adjoint.
struct Acc {
  double gu, gv, gA, gB, gC, go, gc[3], gz;
};

void accumulate_pixel(const Prepared& pr, const std::vector<Hit>& hits, double T_final,
                      const double G_C[3], double G_D, double G_S, std::vector<Acc>& acc) {
  const int n = (int)hits.size();
  double suffix = 0.0;   // sum over later hits of (G_C . c + G_D z) alpha T
  for (int k = n - 1; k >= 0; k--) {
    const Hit& h = hits[k];
    const Cont& c = pr.cont[h.id];
    const double* col = &pr.col[3 * h.id];
    double gcz = G_C[0] * col[0] + G_C[1] * col[1] + G_C[2] * col[2] + G_D * c.p[2];
    double w = h.alpha * h.T;
    Acc& a = acc[h.id];
    for (int j = 0; j < 3; j++) a.gc[j] += G_C[j] * w;
    a.gz += G_D * w;
    double dalpha = h.T * gcz - suffix / (1.0 - h.alpha) + G_S * T_final / (1.0 - h.alpha);
    if (!h.clamped) {
      double e = std::exp(h.power);
      a.go += dalpha * e;
      double gpow = dalpha * h.atil;
      const double A = c.Q[0][0], B = c.Q[0][1], C = c.Q[1][1];
      a.gu += gpow * (A * h.dx + B * h.dy);
      a.gv += gpow * (B * h.dx + C * h.dy);
      a.gA += gpow * (-0.5 * h.dx * h.dx);
      a.gB += gpow * (-h.dx * h.dy);
      a.gC += gpow * (-0.5 * h.dy * h.dy);
    }
    suffix += gcz * w;
  }
}

// Chain rule from the per-Gaussian pixel-level adjoint to the parameters and
// the pose (world-to-camera [R|t]).
void chain_gaussian(const Cont& c, const Acc& a, const Cam& cam, const double mu[3], const double s[3],
                    double gmu[3], double gs[3], double gq[4], double GR[3][3], double Gt[3]) {
  // conic -> Sigma': dL/dSigma' = -Q Ghat Q with Ghat = [[gA, gB/2], [gB/2, gC]]
  double Gh[2][2] = {{a.gA, 0.5 * a.gB}, {0.5 * a.gB, a.gC}};
  double QG[2][2], GS[2][2];
  for (int i = 0; i < 2; i++)
    for (int j = 0; j < 2; j++) QG[i][j] = c.Q[i][0] * Gh[0][j] + c.Q[i][1] * Gh[1][j];
  for (int i = 0; i < 2; i++)
    for (int j = 0; j < 2; j++) GS[i][j] = -(QG[i][0] * c.Q[0][j] + QG[i][1] * c.Q[1][j]);
  // Sigma' = J Sc J^T + 0.3 I -> dL/dJ = 2 GS J Sc, dL/dSc = J^T GS J
  double GJ[2][3], GSc[3][3];
  for (int a2 = 0; a2 < 2; a2++)
    for (int j = 0; j < 3; j++) {
      double acc = 0.0;
      for (int b = 0; b < 2; b++)
        for (int k = 0; k < 3; k++) acc += GS[a2][b] * c.J[b][k] * c.Sc[k][j];
      GJ[a2][j] = 2.0 * acc;
    }
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double acc = 0.0;
      for (int a2 = 0; a2 < 2; a2++)
        for (int b = 0; b < 2; b++) acc += c.J[a2][i] * GS[a2][b] * c.J[b][j];
      GSc[i][j] = acc;
    }
  const double X = c.p[0], Y = c.p[1], Z = c.p[2];
  double gp[3] = {0, 0, 0};
  // u = fx X/Z + cx, v = fy Y/Z + cy
  gp[0] += a.gu * cam.fx / Z;
  gp[2] += -a.gu * cam.fx * X / (Z * Z);
  gp[1] += a.gv * cam.fy / Z;
  gp[2] += -a.gv * cam.fy * Y / (Z * Z);
  // J entries
  gp[2] += GJ[0][0] * (-cam.fx / (Z * Z));
  gp[2] += GJ[1][1] * (-cam.fy / (Z * Z));
  if (c.clampx == 0) {
    gp[0] += GJ[0][2] * (-cam.fx / (Z * Z));
    gp[2] += GJ[0][2] * (2.0 * cam.fx * X / (Z * Z * Z));
  } else {
    gp[2] += GJ[0][2] * (cam.fx * c.clampx * c.limx / (Z * Z));
  }
  if (c.clampy == 0) {
    gp[1] += GJ[1][2] * (-cam.fy / (Z * Z));
    gp[2] += GJ[1][2] * (2.0 * cam.fy * Y / (Z * Z * Z));
  } else {
    gp[2] += GJ[1][2] * (cam.fy * c.clampy * c.limy / (Z * Z));
  }
  // depth used by the depth image
  gp[2] += a.gz;
  // Sc = R Sigma R^T -> dL/dSigma = R^T GSc R, dL/dR += 2 GSc R Sigma
  double GSig[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double acc = 0.0;
      for (int k = 0; k < 3; k++)
        for (int l = 0; l < 3; l++) acc += cam.R[k][i] * GSc[k][l] * cam.R[l][j];
      GSig[i][j] = acc;
    }
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double acc = 0.0;
      for (int k = 0; k < 3; k++)
        for (int l = 0; l < 3; l++) acc += GSc[i][k] * cam.R[k][l] * c.Sigma[l][j];
      GR[i][j] += 2.0 * acc;
    }
  // p = R mu + t
  for (int j = 0; j < 3; j++) {
    double acc = 0.0;
    for (int i = 0; i < 3; i++) acc += cam.R[i][j] * gp[i];
    gmu[j] = acc;
  }
  for (int i = 0; i < 3; i++) {
    for (int j = 0; j < 3; j++) GR[i][j] += gp[i] * mu[j];
    Gt[i] += gp[i];
  }
  // Sigma = M M^T with M = Rq diag(s): dL/dM = 2 GSig M
  double M[3][3], GM[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) M[i][j] = c.Rq[i][j] * s[j];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double acc = 0.0;
      for (int k = 0; k < 3; k++) acc += GSig[i][k] * M[k][j];
      GM[i][j] = 2.0 * acc;
    }
  double GRq[3][3];
  for (int j = 0; j < 3; j++) {
    double acc = 0.0;
    for (int i = 0; i < 3; i++) acc += GM[i][j] * c.Rq[i][j];
    gs[j] = acc;
    for (int i = 0; i < 3; i++) GRq[i][j] = GM[i][j] * s[j];
  }
  // Rq(w, x, y, z): partial derivatives of each entry.
  const double w = c.qn[0], x = c.qn[1], y = c.qn[2], z = c.qn[3];
  double gqn[4] = {0, 0, 0, 0};
  // row 0
  gqn[2] += GRq[0][0] * (-4 * y); gqn[3] += GRq[0][0] * (-4 * z);
  gqn[0] += GRq[0][1] * (-2 * z); gqn[1] += GRq[0][1] * (2 * y); gqn[2] += GRq[0][1] * (2 * x); gqn[3] += GRq[0][1] * (-2 * w);
  gqn[0] += GRq[0][2] * (2 * y); gqn[1] += GRq[0][2] * (2 * z); gqn[2] += GRq[0][2] * (2 * w); gqn[3] += GRq[0][2] * (2 * x);
  // row 1
  gqn[0] += GRq[1][0] * (2 * z); gqn[1] += GRq[1][0] * (2 * y); gqn[2] += GRq[1][0] * (2 * x); gqn[3] += GRq[1][0] * (2 * w);
  gqn[1] += GRq[1][1] * (-4 * x); gqn[3] += GRq[1][1] * (-4 * z);
  gqn[0] += GRq[1][2] * (-2 * x); gqn[1] += GRq[1][2] * (-2 * w); gqn[2] += GRq[1][2] * (2 * z); gqn[3] += GRq[1][2] * (2 * y);
  // row 2
  gqn[0] += GRq[2][0] * (-2 * y); gqn[1] += GRq[2][0] * (2 * z); gqn[2] += GRq[2][0] * (-2 * w); gqn[3] += GRq[2][0] * (2 * x);
  gqn[0] += GRq[2][1] * (2 * x); gqn[1] += GRq[2][1] * (2 * w); gqn[2] += GRq[2][1] * (2 * z); gqn[3] += GRq[2][1] * (2 * y);
  gqn[1] += GRq[2][2] * (-4 * x); gqn[2] += GRq[2][2] * (-4 * y);
  // normalisation q_hat = q / |q|
  double dot = gqn[0] * c.qn[0] + gqn[1] * c.qn[1] + gqn[2] * c.qn[2] + gqn[3] * c.qn[3];
  for (int k = 0; k < 4; k++) gq[k] = (gqn[k] - c.qn[k] * dot) / c.qnorm;
}

void to_double(const float* src, int64_t count, std::vector<double>& dst) {
  dst.resize(count);
  for (int64_t i = 0; i < count; i++) dst[i] = src[i];
}

struct DoubleScene {
  std::vector<double> means, scales, quats, opac, colors;
  Inputs in;
};

void widen(int64_t n, const float* means, const float* scales, const float* quats, const float* opac,
           const float* colors, DoubleScene& d) {
  to_double(means, 3 * n, d.means);
  to_double(scales, 3 * n, d.scales);
  to_double(quats, 4 * n, d.quats);
  to_double(opac, n, d.opac);
  to_double(colors, 3 * n, d.colors);
  d.in.n = n;
  d.in.means = d.means.data();
  d.in.scales = d.scales.data();
  d.in.quats = d.quats.data();
  d.in.opac = d.opac.data();
  d.in.colors = d.colors.data();
}

Cam cam_from_float(const float* viewmat, int W, int H, float fx, float fy, float cx, float cy, float near_z) {
  double V[12];
  for (int i = 0; i < 12; i++) V[i] = viewmat[i];
  return make_cam(V, W, H, fx, fy, cx, cy, near_z);
}

int threads_or_default(int nthreads) { return nthreads > 0 ? nthreads : omp_get_max_threads(); }

}  // namespace

extern "C" {

int or_version(void) { return 1; }

// Pinned projection of every Gaussian (the discrete structure).
// Inputs as in the C ABI (colours only decide culling here).
// Outputs, length n each: visible (0/1), zkey (bits of binary32 depth),
// bbox [4][n] (xlo, xhi, ylo, yhi; clamped pixel box), ctr [2][n] (ui, vi),
// rec [6][n] (uf, vf, a, b, c, qcut), z32 [n]. Culled entries are zero.
int or_project(int64_t n, const float* means, const float* scales, const float* quats, const float* opac,
               const float* colors, const float* viewmat, int W, int H, float fx, float fy, float cx, float cy, float near_z,
               uint8_t* visible, uint32_t* zkey, int32_t* bbox, int32_t* ctr, float* rec, float* z32, int nthreads) {
  Cam cam = cam_from_float(viewmat, W, H, fx, fy, cx, cy, near_z);
  nthreads = threads_or_default(nthreads);
#pragma omp parallel for num_threads(nthreads) schedule(static)
  for (int64_t i = 0; i < n; i++) {
    double mu[3], s[3], q[4], col[3];
    for (int k = 0; k < 3; k++) { mu[k] = means[k * n + i]; s[k] = scales[k * n + i]; col[k] = colors[k * n + i]; }
    for (int k = 0; k < 4; k++) q[k] = quats[k * n + i];
    Pinned P = pinned_project(mu, s, q, (double)opac[i], col, cam);
    visible[i] = P.visible ? 1 : 0;
    zkey[i] = P.zkey;
    bbox[0 * n + i] = P.xlo; bbox[1 * n + i] = P.xhi; bbox[2 * n + i] = P.ylo; bbox[3 * n + i] = P.yhi;
    ctr[0 * n + i] = P.ui; ctr[1 * n + i] = P.vi;
    rec[0 * n + i] = P.uf; rec[1 * n + i] = P.vf; rec[2 * n + i] = P.a;
    rec[3 * n + i] = P.b; rec[4 * n + i] = P.c; rec[5 * n + i] = P.qcut;
    z32[i] = P.z32;
  }
  return 0;
}

// Pinned log2 exposed for its own tests.
double or_pinned_log2(double x) { return pinned_log2(x); }

// Per-tile lists for tile size B: every visible Gaussian whose tile rectangle
// (pixel box divided by B) contains the tile, ordered by (zkey, index).
// Call with ids == NULL to get the total count K (returned).
int64_t or_tile_lists(int64_t n, const uint8_t* visible, const uint32_t* zkey, const int32_t* bbox, int W, int H,
                      int B, int64_t* offsets, uint32_t* ids) {
  const int TX = (W + B - 1) / B, TY = (H + B - 1) / B;
  std::vector<std::vector<uint32_t>> lists((size_t)TX * TY);
  for (int64_t i = 0; i < n; i++) {
    if (!visible[i]) continue;
    int tx0 = bbox[0 * n + i] / B, tx1 = bbox[1 * n + i] / B;
    int ty0 = bbox[2 * n + i] / B, ty1 = bbox[3 * n + i] / B;
    for (int ty = ty0; ty <= ty1; ty++)
      for (int tx = tx0; tx <= tx1; tx++) lists[(size_t)ty * TX + tx].push_back((uint32_t)i);
  }
  int64_t K = 0;
  for (auto& l : lists) K += (int64_t)l.size();
  if (!ids) return K;
  int64_t pos = 0;
  for (size_t t = 0; t < lists.size(); t++) {
    auto& l = lists[t];
    std::stable_sort(l.begin(), l.end(), [&](uint32_t a, uint32_t b) { return zkey[a] < zkey[b]; });
    offsets[t] = pos;
    for (uint32_t id : l) ids[pos++] = id;
  }
  offsets[lists.size()] = pos;
  return K;
}

// Forward render. Outputs: rgb [3][H][W], depth [H][W], sil [H][W], tfinal
// [H][W] (double); ncomp [H][W] (composited count), flags [H][W] (bit 0: the
// stop decision is within its margin; bit 1: an unclamped/clamped decision is
// within its margin); counters [4] = visible, evaluated, accepted, composited.
int or_forward(int64_t n, const float* means, const float* scales, const float* quats, const float* opac,
               const float* colors, const float* viewmat, int W, int H, float fx, float fy, float cx, float cy,
               float near_z, double* rgb, double* depth, double* sil, double* tfinal, int32_t* ncomp,
               uint8_t* flags, int64_t* counters, int nthreads) {
  nthreads = threads_or_default(nthreads);
  DoubleScene ds;
  widen(n, means, scales, quats, opac, colors, ds);
  Cam cam = cam_from_float(viewmat, W, H, fx, fy, cx, cy, near_z);
  Prepared pr;
  prepare(ds.in, cam, pr, nullptr, nthreads);
  int64_t vis = 0, ev = 0, acc = 0, comp = 0;
  for (int64_t i = 0; i < n; i++) vis += pr.pin[i].visible;
  const int64_t P = (int64_t)W * H;
#pragma omp parallel num_threads(nthreads) reduction(+ : ev, acc, comp)
  {
    std::vector<Hit> hits;
    PixelResult r;
#pragma omp for schedule(dynamic, 1)
    for (int y = 0; y < H; y++)
      for (int x = 0; x < W; x++) {
        walk_pixel(pr, cam, x, y, hits, r);
        const int64_t p = (int64_t)y * W + x;
        for (int k = 0; k < 3; k++) rgb[k * P + p] = r.C[k];
        depth[p] = r.D;
        sil[p] = 1.0 - r.T;
        tfinal[p] = r.T;
        ncomp[p] = (int32_t)hits.size();
        flags[p] = r.flags;
        ev += r.evaluated;
        acc += r.accepted;
        comp += (int64_t)hits.size();
      }
  }
  counters[0] = vis; counters[1] = ev; counters[2] = acc; counters[3] = comp;
  return 0;
}

// Backward. Upstream gradients g_rgb [3][H][W], g_depth, g_sil [H][W].
// Outputs (double): d_means [3][n], d_scales [3][n], d_quats [4][n],
// d_opac [n], d_colors [3][n], d_viewmat [12] (dL/d[R|t], row-major),
// d_twist [6] (rho, phi) for the left perturbation exp(xi^) [R|t];
// gflags [n]: 1 where a Gaussian is composited at a pixel with a
// margin-flagged decision, or sits at that decision.
int or_backward(int64_t n, const float* means, const float* scales, const float* quats, const float* opac,
                const float* colors, const float* viewmat, int W, int H, float fx, float fy, float cx, float cy,
                float near_z, const float* g_rgb, const float* g_depth, const float* g_sil, double* d_means,
                double* d_scales, double* d_quats, double* d_opac, double* d_colors, double* d_viewmat,
                double* d_twist, uint8_t* gflags, int nthreads) {
  nthreads = threads_or_default(nthreads);
  DoubleScene ds;
  widen(n, means, scales, quats, opac, colors, ds);
  Cam cam = cam_from_float(viewmat, W, H, fx, fy, cx, cy, near_z);
  Prepared pr;
  prepare(ds.in, cam, pr, nullptr, nthreads);
  const int64_t P = (int64_t)W * H;
  std::vector<std::vector<Acc>> accs(nthreads);
  std::vector<std::vector<int32_t>> flagged(nthreads);
#pragma omp parallel num_threads(nthreads)
  {
    int tid = omp_get_thread_num();
    accs[tid].assign(n, Acc());
    std::memset(accs[tid].data(), 0, sizeof(Acc) * n);
    std::vector<Hit> hits;
    PixelResult r;
#pragma omp for schedule(static)
    for (int y = 0; y < H; y++)
      for (int x = 0; x < W; x++) {
        walk_pixel(pr, cam, x, y, hits, r);
        const int64_t p = (int64_t)y * W + x;
        double GC[3] = {g_rgb[p], g_rgb[P + p], g_rgb[2 * P + p]};
        accumulate_pixel(pr, hits, r.T, GC, g_depth[p], g_sil[p], accs[tid]);
        // A decision inside its margin may go the other way in binary32. A
        // different stop point changes T_final, and a different clamp state
        // changes (1 - alpha) by up to 1%, for the whole pixel: so every
        // Gaussian composited at the pixel is flagged, plus the one at the
        // decision.
        if (r.flags) {
          for (const Hit& h : hits) flagged[tid].push_back(h.id);
          if (r.stop_id >= 0) flagged[tid].push_back(r.stop_id);
          if (r.clamp_id >= 0) flagged[tid].push_back(r.clamp_id);
        }
      }
  }
  std::vector<Acc> acc(n);
  std::memset(acc.data(), 0, sizeof(Acc) * n);
  for (int t = 0; t < nthreads; t++)
    for (int64_t i = 0; i < n; i++) {
      const Acc& s = accs[t][i];
      Acc& d = acc[i];
      d.gu += s.gu; d.gv += s.gv; d.gA += s.gA; d.gB += s.gB; d.gC += s.gC; d.go += s.go; d.gz += s.gz;
      for (int k = 0; k < 3; k++) d.gc[k] += s.gc[k];
    }
  std::memset(gflags, 0, n);
  for (auto& v : flagged)
    for (int32_t id : v) gflags[id] = 1;
  double GR[3][3] = {{0}}, Gt[3] = {0, 0, 0};
  for (int64_t i = 0; i < n; i++) {
    double gmu[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0};
    if (pr.pin[i].visible) {
      double mu[3], s[3], q[4], o, col[3];
      gather(ds.in, i, mu, s, q, o, col);
      chain_gaussian(pr.cont[i], acc[i], cam, mu, s, gmu, gs, gq, GR, Gt);
    }
    for (int k = 0; k < 3; k++) {
      d_means[k * n + i] = gmu[k];
      d_scales[k * n + i] = gs[k];
      d_colors[k * n + i] = pr.pin[i].visible ? acc[i].gc[k] : 0.0;
    }
    for (int k = 0; k < 4; k++) d_quats[k * n + i] = gq[k];
    d_opac[i] = pr.pin[i].visible ? acc[i].go : 0.0;
  }
  for (int i = 0; i < 3; i++) {
    for (int j = 0; j < 3; j++) d_viewmat[4 * i + j] = GR[i][j];
    d_viewmat[4 * i + 3] = Gt[i];
  }
  // left twist: rho = dL/dt, phi = sum_k r_k x g_k + t x dL/dt (r_k, g_k columns)
  double phi[3] = {0, 0, 0};
  for (int k = 0; k < 3; k++) {
    double r[3] = {cam.R[0][k], cam.R[1][k], cam.R[2][k]};
    double g[3] = {GR[0][k], GR[1][k], GR[2][k]};
    phi[0] += r[1] * g[2] - r[2] * g[1];
    phi[1] += r[2] * g[0] - r[0] * g[2];
    phi[2] += r[0] * g[1] - r[1] * g[0];
  }
  phi[0] += cam.t[1] * Gt[2] - cam.t[2] * Gt[1];
  phi[1] += cam.t[2] * Gt[0] - cam.t[0] * Gt[2];
  phi[2] += cam.t[0] * Gt[1] - cam.t[1] * Gt[0];
  for (int k = 0; k < 3; k++) { d_twist[k] = Gt[k]; d_twist[3 + k] = phi[k]; }
  return 0;
}

// ------------------------------------------------------------- frozen mode
// Record, at the given parameters, every pixel's composited list (Gaussian
// ids and clamp states, in order) and every Gaussian's field-of-view clamp
// branch. Two-call protocol: with ids == NULL returns the total length.
int64_t or_record(int64_t n, const float* means, const float* scales, const float* quats, const float* opac,
                  const float* colors, const float* viewmat, int W, int H, float fx, float fy, float cx, float cy,
                  float near_z, int64_t* offsets, int32_t* ids, uint8_t* clamped, int8_t* fov_clamp, int nthreads) {
  nthreads = threads_or_default(nthreads);
  DoubleScene ds;
  widen(n, means, scales, quats, opac, colors, ds);
  Cam cam = cam_from_float(viewmat, W, H, fx, fy, cx, cy, near_z);
  Prepared pr;
  prepare(ds.in, cam, pr, nullptr, nthreads);
  const int64_t P = (int64_t)W * H;
  std::vector<std::vector<Hit>> per(P);
#pragma omp parallel num_threads(nthreads)
  {
    PixelResult r;
#pragma omp for schedule(dynamic, 1)
    for (int y = 0; y < H; y++)
      for (int x = 0; x < W; x++) walk_pixel(pr, cam, x, y, per[(int64_t)y * W + x], r);
  }
  int64_t total = 0;
  for (auto& v : per) total += (int64_t)v.size();
  if (!ids) return total;
  int64_t pos = 0;
  for (int64_t p = 0; p < P; p++) {
    offsets[p] = pos;
    for (const Hit& h : per[p]) {
      ids[pos] = h.id;
      clamped[pos] = h.clamped ? 1 : 0;
      pos++;
    }
  }
  offsets[P] = pos;
  for (int64_t i = 0; i < n; i++) {
    fov_clamp[2 * i] = (int8_t)pr.cont[i].clampx;
    fov_clamp[2 * i + 1] = (int8_t)pr.cont[i].clampy;
  }
  return total;
}

// Loss L = sum_p G_C . C + G_D D + G_S S with every decision frozen to a
// record: the composited lists, clamp states and field-of-view clamp
// branches. Parameters and pose are double so that finite differences can use
// small steps. Decisions are not re-evaluated.
double or_frozen_loss(int64_t n, const double* means, const double* scales, const double* quats,
                      const double* opac, const double* colors, const double* viewmat, int W, int H, double fx,
                      double fy, double cx, double cy, const int64_t* offsets, const int32_t* ids,
                      const uint8_t* clamped, const int8_t* fov_clamp, const float* g_rgb, const float* g_depth,
                      const float* g_sil, int nthreads) {
  nthreads = threads_or_default(nthreads);
  Cam cam = make_cam(viewmat, W, H, fx, fy, cx, cy, 0.0);
  Inputs in{n, means, scales, quats, opac, colors};
  // only Gaussians that appear in some list need a projection
  std::vector<uint8_t> used(n, 0);
  const int64_t P = (int64_t)W * H;
  for (int64_t k = 0; k < offsets[P]; k++) used[ids[k]] = 1;
  std::vector<Cont> cont(n);
#pragma omp parallel for num_threads(nthreads) schedule(static)
  for (int64_t i = 0; i < n; i++) {
    if (!used[i]) continue;
    double mu[3], s[3], q[4], o, col[3];
    gather(in, i, mu, s, q, o, col);
    cont_project(mu, s, q, cam, true, fov_clamp[2 * i], fov_clamp[2 * i + 1], cont[i]);
  }
  double L = 0.0;
#pragma omp parallel for num_threads(nthreads) reduction(+ : L) schedule(static)
  for (int64_t p = 0; p < P; p++) {
    const int x = (int)(p % W), y = (int)(p / W);
    double T = 1.0, C[3] = {0, 0, 0}, D = 0.0;
    for (int64_t k = offsets[p]; k < offsets[p + 1]; k++) {
      const int32_t id = ids[k];
      double dx, dy;
      double pw = power_at(cont[id], x, y, dx, dy);
      double alpha = clamped[k] ? ALPHA_MAX : opac[id] * std::exp(pw);
      for (int j = 0; j < 3; j++) C[j] += colors[j * n + id] * alpha * T;
      D += cont[id].p[2] * alpha * T;
      T *= (1.0 - alpha);
    }
    L += g_rgb[p] * C[0] + g_rgb[P + p] * C[1] + g_rgb[2 * P + p] * C[2] + g_depth[p] * D + g_sil[p] * (1.0 - T);
  }
  return L;
}

}  // extern "C"

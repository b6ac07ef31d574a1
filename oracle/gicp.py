"""Generalized-ICP alignment of the consensus (Sec. 3.4 "3) Alignment", Eqs.
3-4; Sec. 3.5 "3) Alignment", Eq. 6), in numpy.

TEST INFRASTRUCTURE ONLY: imported by the test suite, never by the product
path. Shares no code with the GPU implementation.

What is computed. Source Gaussians (observed points, or another map's
Gaussians) x_k with covariances S_k are aligned to target (map) Gaussians
y_l with covariances S_l by a rigid transform T = [R|t] minimising
    E(T) = sum_(k,l) r^T (R S_k R^T + S_l + eps I)^-1 r,   r = T x_k - y_l,
over the correspondences (k, l): Eq. 6 with the source covariance rotated
by T (Generalized-ICP's plane-to-plane form; Eq. 6 as printed omits the
rotation), and Eq. 4's Mahalanobis distance when the sources are points
(S_k = 0). Readings where the paper is silent:
  - eps I (eps >= 0, a parameter, 1e-6 m^2 by default) keeps the matrix
    invertible for flat Gaussians;
  - correspondences: each source takes the nearest target mean within the
    Generalized-ICP point-selection distance d_max (0.02 m, Sec. 4.1),
    inclusive, ties to the smaller target index; the decision is an integer
    taken in binary32 in a pinned order, no fused operations:
      y_k = ((R_k0 x_0 + R_k1 x_1) + R_k2 x_2) + t_k,
      d = y - mu_l (per component), d2 = (d_0 d_0 + d_1 d_1) + d_2 d_2,
      accepted iff d2 <= fl32(d_max * d_max);
  - a source whose transformed point, or a target whose mean, has a
    non-finite coordinate takes no part;
  - covariances of Gaussians given by scales and unit quaternions:
    S = R_q diag(s^2) R_q^T;
  - one iteration: correspondences at the current T, then the Gauss-Newton
    step on the left twist xi = (rho, phi) of T <- exp(xi^) T, with the
    matrices (R S_k R^T + S_l + eps I)^-1 held at the current T:
      J = [I | -[T x]_x],  H = sum J^T M J,  g = sum J^T M r,
      xi = -(H + lam I)^-1 g,  lam = 1e-12 trace(H) / 6;
    T is stored in binary32 between iterations (as the device stores it).
"""
import math

import numpy as np
from scipy.spatial import cKDTree


def quat_cov(scales, quats):
    """[n][3][3] covariances R_q diag(s^2) R_q^T from scales [3][n] and
    quaternions [4][n] (w, x, y, z; normalised here)."""
    s = np.asarray(scales, np.float64)
    q = np.asarray(quats, np.float64)
    q = q / np.linalg.norm(q, axis=0)
    w, x, y, z = q
    R = np.empty((q.shape[1], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    M = R * s.T[:, None, :]
    return M @ M.transpose(0, 2, 1)


def transform32(T, x):
    """Binary32 y = R x + t in the pinned order. T: [12] (fp32 values), x: [3][n]."""
    T = np.asarray(T, np.float32)
    x = np.asarray(x, np.float32)
    return np.stack([(((T[4 * k] * x[0]).astype(np.float32) + (T[4 * k + 1] * x[1]).astype(np.float32))
                      .astype(np.float32) + (T[4 * k + 2] * x[2]).astype(np.float32)).astype(np.float32)
                     + T[4 * k + 3] for k in range(3)]).astype(np.float32)


def correspond(T, src, tgt, d_max=0.02):
    """Target index per source ([n] int64, -1 when none within d_max)."""
    with np.errstate(invalid="ignore", over="ignore"):
        y = transform32(T, src)
    mu = np.asarray(tgt, np.float32)
    dmax2 = np.float32(np.float32(d_max) * np.float32(d_max))
    out = np.full(y.shape[1], -1, np.int64)
    # a non-finite target mean is never a neighbour, a non-finite transformed
    # source has none
    live = np.flatnonzero(np.all(np.isfinite(mu), axis=0))
    qk = np.flatnonzero(np.all(np.isfinite(y), axis=0))
    if live.size == 0 or qk.size == 0:
        return out
    tree = cKDTree(mu[:, live].T.astype(np.float64))
    # binary64 superset of the binary32 test; the pinned distance decides
    cand = tree.query_ball_point(y[:, qk].T.astype(np.float64), r=float(d_max) * (1 + 1e-4) + 1e-6)
    for k, c in zip(qk, cand):
        if not c:
            continue
        c = live[np.asarray(sorted(c), np.int64)]
        d = (y[:, k:k + 1] - mu[:, c]).astype(np.float32)
        d2 = ((d[0] * d[0]).astype(np.float32) + (d[1] * d[1]).astype(np.float32)).astype(np.float32)
        d2 = (d2 + (d[2] * d[2]).astype(np.float32)).astype(np.float32)
        ok = d2 <= dmax2
        if ok.any():
            best = np.min(d2[ok])
            out[k] = int(c[ok & (d2 == best)].min())
    return out


def hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def normal_equations(T, src, src_cov, tgt, tgt_cov, corr, eps=1e-6):
    """(H [6][6], g [6], cost, count) at T for the given correspondences, in
    binary64. src_cov: [n][3][3] or None (points); tgt_cov: [m][3][3]."""
    V = np.asarray(T, np.float64).reshape(3, 4)      # a binary32 pose widens exactly
    R, t = V[:, :3], V[:, 3]
    k = np.flatnonzero(corr >= 0)
    l = corr[k]
    x = np.asarray(src, np.float32).astype(np.float64)[:, k]
    y = np.asarray(tgt, np.float32).astype(np.float64)[:, l]
    p = R @ x + t[:, None]
    r = (p - y).T                                             # [c][3]
    C = tgt_cov[l] + eps * np.eye(3)
    if src_cov is not None:
        C = C + R @ src_cov[k] @ R.T
    M = np.linalg.inv(C)
    H = np.zeros((6, 6))
    g = np.zeros(6)
    cost = 0.0
    for i in range(len(k)):
        J = np.concatenate([np.eye(3), -hat(p[:, i])], axis=1)
        MJ = M[i] @ J
        H += J.T @ MJ
        g += J.T @ (M[i] @ r[i])
        cost += float(r[i] @ M[i] @ r[i])
    return H, g, cost, len(k)


def exp_se3(xi):
    """4x4 exp of the twist (rho, phi) (closed form)."""
    rho, phi = np.asarray(xi[:3], np.float64), np.asarray(xi[3:], np.float64)
    th = float(np.linalg.norm(phi))
    K = hat(phi)
    if th < 1e-12:
        Rx, Vm = np.eye(3) + K, np.eye(3) + 0.5 * K
    else:
        Rx = np.eye(3) + math.sin(th) / th * K + (1 - math.cos(th)) / th ** 2 * (K @ K)
        Vm = np.eye(3) + (1 - math.cos(th)) / th ** 2 * K + (th - math.sin(th)) / th ** 3 * (K @ K)
    E = np.eye(4)
    E[:3, :3] = Rx
    E[:3, 3] = Vm @ rho
    return E


def gn_update(T, H, g):
    """T <- exp(xi^) T with xi = -(H + lam I)^-1 g; returns binary32 [12]."""
    lam = 1e-12 * np.trace(H) / 6.0
    xi = -np.linalg.solve(H + lam * np.eye(6), g)
    P = np.eye(4)
    P[:3] = np.asarray(T, np.float32).astype(np.float64).reshape(3, 4)
    return (exp_se3(xi) @ P)[:3].reshape(12).astype(np.float32), xi


def align(T0, src, src_cov, tgt, tgt_cov, iters=10, d_max=0.02, eps=1e-6):
    """Generalized-ICP iterations from T0: returns (T [12] binary32, per-iteration
    (cost, count) list, last correspondences)."""
    T = np.asarray(T0, np.float32)
    hist = []
    corr = None
    for _ in range(iters):
        corr = correspond(T, src, tgt, d_max)
        H, g, cost, cnt = normal_equations(T, src, src_cov, tgt, tgt_cov, corr, eps)
        hist.append((cost, cnt))
        if cnt < 6:
            break
        T, _ = gn_update(T, H, g)
    return T, hist, corr

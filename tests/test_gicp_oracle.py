"""Pins of the Generalized-ICP oracle (oracle/gicp.py) with nothing of its
own arithmetic: exact recovery of a known rigid transform from noiseless
sources; the normal equations against central differences of the cost
(2 g = dE/dxi with the matrices held) and of g itself (H = dg/dxi where the
residuals vanish); R S_k R^T + S_l against a closed form; the
correspondence step against a brute force over every target, with the
inclusive threshold and the tie-break to the smaller index."""
import math

import numpy as np
from scipy.spatial.transform import Rotation

from oracle import gicp as G


def _lattice(rng, n, spacing=0.1, jitter=0.02):
    """Target means on a jittered lattice (neighbours >= 0.06 m apart, so a
    source within d_max of its own target has no other candidate)."""
    side = int(math.ceil(n ** (1 / 3)))
    idx = np.stack(np.meshgrid(*[np.arange(side)] * 3, indexing="ij"), 0).reshape(3, -1)[:, :n]
    return (idx * spacing + rng.uniform(-jitter, jitter, idx.shape)).astype(np.float32) + np.float32(1.0)


def _pose(rng, deg, metres):
    R = Rotation.from_rotvec(np.deg2rad(deg) * rng.standard_normal(3) / math.sqrt(3)).as_matrix()
    t = rng.normal(0, metres, 3)
    return np.concatenate([R, t[:, None]], axis=1).reshape(12).astype(np.float32)


def _compose(A, B):
    P = np.eye(4)
    Q = np.eye(4)
    P[:3] = np.asarray(A, np.float64).reshape(3, 4)
    Q[:3] = np.asarray(B, np.float64).reshape(3, 4)
    return (P @ Q)[:3].reshape(12)


def _inverse(T):
    V = np.asarray(T, np.float64).reshape(3, 4)
    R, t = V[:, :3], V[:, 3]
    return np.concatenate([R.T, (-R.T @ t)[:, None]], axis=1).reshape(12)


def test_recovers_a_known_transform():
    rng = np.random.default_rng(1)
    tgt = _lattice(rng, 600)
    tcov = G.quat_cov(np.exp(rng.uniform(np.log(0.002), np.log(0.03), (3, 600))), rng.standard_normal((4, 600)))
    T_true = _pose(rng, 8.0, 0.3)
    inv = _inverse(T_true).reshape(3, 4)
    src = (inv[:, :3] @ tgt.astype(np.float64) + inv[:, 3:]).astype(np.float32)   # noiseless sources
    T0 = _compose(_pose(rng, 0.2, 0.004), T_true).astype(np.float32)              # within d_max of the truth
    T, hist, corr = G.align(T0, src, None, tgt, tcov, iters=8)
    assert np.array_equal(corr, np.arange(600))
    assert np.abs(T - T_true).max() <= 2e-6, np.abs(T - T_true).max()
    assert hist[-1][0] <= 1e-6 * hist[0][0]
    # the same with Gaussian sources (their covariance rotated by T)
    scov = G.quat_cov(np.exp(rng.uniform(np.log(0.002), np.log(0.03), (3, 600))), rng.standard_normal((4, 600)))
    T, hist, corr = G.align(T0, src, scov, tgt, tcov, iters=8)
    assert np.abs(T - T_true).max() <= 2e-6


def test_normal_equations_against_central_differences():
    rng = np.random.default_rng(2)
    tgt = _lattice(rng, 300)
    tcov = G.quat_cov(np.exp(rng.uniform(np.log(0.002), np.log(0.03), (3, 300))), rng.standard_normal((4, 300)))
    scov = G.quat_cov(np.exp(rng.uniform(np.log(0.002), np.log(0.02), (3, 300))), rng.standard_normal((4, 300)))
    T = _pose(rng, 5.0, 0.2)
    inv = _inverse(T).reshape(3, 4)
    src = (inv[:, :3] @ (tgt.astype(np.float64) + rng.normal(0, 0.004, tgt.shape)) + inv[:, 3:]).astype(np.float32)
    corr = np.arange(300)
    H, g, cost, cnt = G.normal_equations(T, src, scov, tgt, tcov, corr)
    V = np.asarray(T, np.float64).reshape(3, 4)
    R = V[:, :3]
    M = np.linalg.inv(tcov + 1e-6 * np.eye(3) + R @ scov @ R.T)        # held at T
    x, y = src.astype(np.float64), tgt.astype(np.float64)

    def E(xi):
        P = np.eye(4)
        P[:3] = V
        Tn = (G.exp_se3(xi) @ P)[:3]
        r = (Tn[:, :3] @ x + Tn[:, 3:] - y).T
        return float(np.einsum("ni,nij,nj->", r, M, r))
    h = 1e-6
    fd = np.array([(E(h * e) - E(-h * e)) / (2 * h) for e in np.eye(6)])
    assert np.allclose(fd, 2 * g, rtol=1e-6, atol=1e-9 * np.abs(g).max())
    assert abs(E(np.zeros(6)) - cost) <= 1e-12 * cost

    # where every residual vanishes, H is the derivative of g
    y0 = (V[:, :3] @ x + V[:, 3:]).astype(np.float32)
    def gvec(xi):
        P = np.eye(4)
        P[:3] = V
        Tn = (G.exp_se3(xi) @ P)[:3].reshape(12)
        return G.normal_equations(Tn, src, None, y0, tcov, corr)[1]
    H0 = G.normal_equations(T, src, None, y0, tcov, corr)[0]
    Jg = np.stack([(gvec(h * e) - gvec(-h * e)) / (2 * h) for e in np.eye(6)], axis=1)
    assert np.allclose(Jg, H0, rtol=2e-4, atol=2e-4 * np.abs(H0).max())


def test_rotated_source_covariance_closed_form():
    # source covariance diag(a, b, c) rotated 90 degrees about z becomes diag(b, a, c)
    a, b, c, sl = 4e-4, 1e-4, 9e-4, 2.5e-4
    T = np.array([0, -1, 0, 0, 1, 0, 0, 0, 0, 0, 1, 0], np.float32)
    src = np.array([[0.0], [0.0], [1.0]], np.float32)
    tgt = np.array([[0.015625], [0.0], [1.0]], np.float32)         # residual (-2^-6, 0, 0), exact
    scov = np.diag([a, b, c])[None]
    tcov = (sl * np.eye(3))[None]
    H, g, cost, cnt = G.normal_equations(T, src, scov, tgt, tcov, np.array([0]), eps=0.0)
    assert cnt == 1 and abs(cost - 0.015625 ** 2 / (b + sl)) <= 1e-15


def test_correspondences_against_brute_force():
    rng = np.random.default_rng(3)
    tgt = rng.uniform(0, 0.5, (3, 3000)).astype(np.float32)
    src = rng.uniform(0, 0.5, (3, 800)).astype(np.float32)
    T = _pose(rng, 3.0, 0.01)
    got = G.correspond(T, src, tgt, 0.02)
    y = G.transform32(T, src)
    dmax2 = np.float32(np.float32(0.02) * np.float32(0.02))
    for k in range(src.shape[1]):
        best, bi = None, -1
        for l in range(tgt.shape[1]):
            d = (y[:, k] - tgt[:, l]).astype(np.float32)
            d2 = np.float32(np.float32(np.float32(d[0] * d[0]) + np.float32(d[1] * d[1])) + np.float32(d[2] * d[2]))
            if d2 <= dmax2 and (best is None or d2 < best):
                best, bi = d2, l
        assert got[k] == bi, (k, got[k], bi)
    assert (got >= 0).sum() > 100
    # inclusive threshold and the tie-break: d_max = 0.5 (exact squares)
    I = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], np.float32)
    tg = np.array([[0.0, 1.0], [0.0, 0.0], [0.0, 0.0]], np.float32)
    after = float(np.nextafter(np.float32(0.5), np.float32(1)))
    sr = np.array([[-0.5, -after, 0.5], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]], np.float32)
    # exactly d_max from target 0: in; just beyond: none; 0.5 from both: the smaller index
    assert G.correspond(I, sr, tg, 0.5).tolist() == [0, -1, 0]


def test_non_finite_inputs_take_no_part():
    rng = np.random.default_rng(4)
    tgt = rng.uniform(0, 0.2, (3, 500)).astype(np.float32)
    src = rng.uniform(0, 0.2, (3, 300)).astype(np.float32)
    I = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], np.float32)
    t2, s2 = tgt.copy(), src.copy()
    t2[:, 11] = np.nan
    s2[:, 3] = np.inf
    got = G.correspond(I, s2, t2, 0.02)
    assert got[3] == -1 and 11 not in got
    # the rest as if target 11 were absent
    t3 = tgt.copy()
    t3[:, 11] = 1e6
    want = G.correspond(I, src, t3, 0.02)
    want[3] = -1
    assert np.array_equal(got, want)

"""The compositing kernels skip a staged record for an 8x8 sub-block when
interval bounds on t1 = a dx + b dy and t2 = c dy over the sub-block's
rounded pixel offsets show that no pixel can pass the binary32 acceptance
test q <= qcut. This file restates that bound in numpy float32 (written here
from its derivation, not taken from the kernel) and checks it against brute
force: every pixel of the sub-block evaluated with the pinned binary32
recipe (t1 = fma(a, dx, b * dy), t2 = c * dy, q = fma(t1, t1, t2 * t2)), on
Gaussians chosen to stress it: needle-like ones at every orientation, centres
far off-screen, offsets near 2^22 px, sub-blocks placed around the edge of
the acceptance ellipse. A record that some pixel accepts must never be
skipped."""
import numpy as np

F32 = np.float32
EPS = F32(2.0 ** -20)
KAPPA = float.fromhex("0x1.b2da4e9808a53p-1")
Q9 = float.fromhex("0x1.9f7f051d0f35ep+2")


def _fma(a, b, c):
    # binary32 fused multiply-add: the product and sum in extended precision,
    # one rounding to binary32
    return (np.longdouble(a) * np.longdouble(b) + np.longdouble(c)).astype(F32)


def _gaussians(rng, n):
    lam1 = 10 ** rng.uniform(np.log10(0.3), np.log10(4e6), n)
    lam2 = np.maximum(0.3, lam1 * 10 ** rng.uniform(-7, 0, n))
    th = rng.uniform(0, np.pi, n)
    s00 = lam1 * np.cos(th) ** 2 + lam2 * np.sin(th) ** 2
    s11 = lam1 * np.sin(th) ** 2 + lam2 * np.cos(th) ** 2
    s01 = (lam1 - lam2) * np.sin(th) * np.cos(th)
    det = s00 * s11 - s01 ** 2
    sd, s1 = np.sqrt(det), np.sqrt(s11)
    a = (KAPPA * s1 / sd).astype(F32)
    b = (KAPPA * (-s01 / (sd * s1))).astype(F32)
    c = (KAPPA / s1).astype(F32)
    qc = np.minimum(Q9, np.log2(255 * rng.uniform(1 / 255, 1, n))).astype(F32)
    u = rng.uniform(-3000, 4000, n)
    v = rng.uniform(-3000, 4000, n)
    far = rng.random(n) < 0.05
    u[far] += 2.0 ** 21          # offsets near the top of the exact integer range
    # a sub-block near the ellipse edge
    r = np.sqrt(np.maximum(qc, 0) / KAPPA ** 2) * rng.uniform(0.7, 1.3, n)
    phi = rng.uniform(0, 2 * np.pi, n)
    px = u + r * (np.sqrt(lam1) * np.cos(phi) * np.cos(th) - np.sqrt(lam2) * np.sin(phi) * np.sin(th))
    py = v + r * (np.sqrt(lam1) * np.cos(phi) * np.sin(th) + np.sqrt(lam2) * np.sin(phi) * np.cos(th))
    px += rng.uniform(-8, 8, n)
    py += rng.uniform(-8, 8, n)
    x0 = (np.floor(px / 8) * 8).astype(np.int64)
    y0 = (np.floor(py / 8) * 8).astype(np.int64)
    ui, vi = np.floor(u).astype(F32), np.floor(v).astype(F32)
    uf, vf = (u - np.floor(u)).astype(F32), (v - np.floor(v)).astype(F32)
    return a, b, c, qc, ui, vi, uf, vf, x0, y0


def _reaches(a, b, c, qc, ui, vi, uf, vf, x0, y0):
    """The bound, in binary32 step by step."""
    gx = (x0.astype(F32) - ui).astype(F32)                    # exact integers
    gy = (y0.astype(F32) - vi).astype(F32)
    dx0 = (gx - uf).astype(F32)
    dx1 = ((F32(7) + gx).astype(F32) - uf).astype(F32)
    dy0 = (gy - vf).astype(F32)
    dy1 = ((F32(7) + gy).astype(F32) - vf).astype(F32)
    ax0, ax1 = (a * dx0).astype(F32), (a * dx1).astype(F32)
    by0, by1 = (b * dy0).astype(F32), (b * dy1).astype(F32)
    lo1 = (np.minimum(ax0, ax1) + np.minimum(by0, by1)).astype(F32)
    hi1 = (np.maximum(ax0, ax1) + np.maximum(by0, by1)).astype(F32)
    ym = np.maximum(np.abs(dy0), np.abs(dy1))
    m1 = np.maximum(np.maximum(lo1, -hi1), F32(0))
    m2 = (np.abs(c) * np.maximum(np.maximum(dy0, -dy1), F32(0))).astype(F32)
    span = ((np.abs(a) * np.maximum(np.abs(dx0), np.abs(dx1))).astype(F32) + (np.abs(b) * ym).astype(F32)).astype(F32)
    e1 = (EPS * (span + F32(3)).astype(F32)).astype(F32)
    e2 = (EPS * (np.abs(c) * ym).astype(F32)).astype(F32)
    r1 = np.maximum((m1 - e1).astype(F32), F32(0))
    r2 = np.maximum((m2 - e2).astype(F32), F32(0))
    return _fma(r1, r1, (r2 * r2).astype(F32)) <= (qc * (F32(1) + EPS)).astype(F32), gx, gy


def _accepted_anywhere(a, b, c, qc, gx, gy, uf, vf):
    hit = np.zeros(a.shape, bool)
    for yl in range(8):
        dy = ((F32(yl) + gy).astype(F32) - vf).astype(F32)
        p = (b * dy).astype(F32)
        t2 = (c * dy).astype(F32)
        t2s = (t2 * t2).astype(F32)
        for xl in range(8):
            dx = ((F32(xl) + gx).astype(F32) - uf).astype(F32)
            t1 = _fma(a, dx, p)
            hit |= _fma(t1, t1, t2s) <= qc
    return hit


def test_skipped_records_composite_nowhere():
    rng = np.random.default_rng(20241212)
    a, b, c, qc, ui, vi, uf, vf, x0, y0 = _gaussians(rng, 60000)
    reach, gx, gy = _reaches(a, b, c, qc, ui, vi, uf, vf, x0, y0)
    hit = _accepted_anywhere(a, b, c, qc, gx, gy, uf, vf)
    assert hit.sum() > 10000 and (~reach).sum() > 10000      # both outcomes well represented
    assert not np.any(hit & ~reach), np.flatnonzero(hit & ~reach)[:10]


def test_bound_is_tight_enough_to_matter():
    # among sub-blocks that no pixel reaches, the bound drops most
    rng = np.random.default_rng(7)
    a, b, c, qc, ui, vi, uf, vf, x0, y0 = _gaussians(rng, 20000)
    reach, gx, gy = _reaches(a, b, c, qc, ui, vi, uf, vf, x0, y0)
    hit = _accepted_anywhere(a, b, c, qc, gx, gy, uf, vf)
    assert (~reach & ~hit).sum() > 0.8 * (~hit).sum()


def test_faint_and_never_accepting_records():
    # qcut = 0 accepts only q = 0; qcut = -inf (opacity 0) accepts nothing
    a = np.full(3, 0.5, F32)
    b = np.zeros(3, F32)
    c = np.full(3, 0.5, F32)
    qc = np.array([0.0, -np.inf, 0.0], F32)
    ui = np.array([10, 10, 10], F32)
    vi = np.array([10, 10, 10], F32)
    uf = np.zeros(3, F32)
    vf = np.zeros(3, F32)
    x0 = np.array([8, 8, 24], np.int64)        # centre pixel (10, 10) inside the first two blocks
    y0 = np.array([8, 8, 24], np.int64)
    reach, gx, gy = _reaches(a, b, c, qc, ui, vi, uf, vf, x0, y0)
    hit = _accepted_anywhere(a, b, c, qc, gx, gy, uf, vf)
    assert hit.tolist() == [True, False, False]
    assert reach.tolist() == [True, False, False]

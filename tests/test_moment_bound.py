"""The backward's per-Gaussian sums in moment form, restated step by step in
numpy binary32, against binary64 per-pixel sums: the error bound stated with
the binary32 matrix-core backward holds for Gaussians placed where it is
tightest -- elongated Gaussians whose centre lies far from the 8x8 sub-block
(large U, V), whose composited pixels sit in a corner of it (|k1| near its
maximum), and faint ones (opacity within a few per cent of the 1/255 floor,
qcut near 0).

Per sub-block and Gaussian, with e the per-pixel values, the moments S of e
over (1, xi, eta, xi^2, xi eta, eta^2) are summed in binary32, then
  k1 = a U + b V,  P1 = a Sx + b Sy - k1 S1,  P2 = c (Sy - V S1),
  P1x = (a Sxx + b Sxy - k1 Sx) - U P1,  P1y = (a Sxy + b Syy - k1 Sy) - V P1,
  P2y = c ((Syy - 2 V Sy) + V^2 S1),
and each must lie within
  |dP1| <= g L S,  |dP1x| <= g (3.5 + |U|) L S,  |dP1y| <= g (3.5 + |V|) L S,
  |dP2| <= g M S,  |dP2y| <= g (3.5 + |V|) M S,
with S = sum |e|, L = 3.5 (|a| + |b|) + |k1|, M = 7 |c| + sqrt(qcut),
g = gamma_64 + 4u + (rounding of the binary64 reference, negligible).
Relative to the sums' natural size (sqrt(qcut) S times the same offset
factors) the bound does not grow with the Gaussian's elongation or the
distance of its centre, which the sampled cases push to the extremes.
"""
import math

import numpy as np

from oracle import brute
from paper_2412_09723_amd import scenes

U32 = 2.0 ** -24
GAMMA64 = 64 * U32 / (1 - 64 * U32)
G = GAMMA64 + 4 * U32
KMAX = float.fromhex("0x1.b2da4e9808a53p-1") / math.sqrt(0.3)


def _fma(a, b, c):
    return brute.fmaf(np.float32(a), np.float32(b), np.float32(c))


def _f(x):
    return np.float32(x)


def _cases(rng, count=6000):
    """(record, X0, Y0) triples: needles, anisotropic and faint Gaussians from
    projected scenes, each paired with an 8x8 sub-block that its acceptance
    region only clips (a corner or an edge), often far from its centre."""
    intr = scenes.Intrinsics(640, 480, 500.0, 500.0, 320.0, 240.0)
    out = []
    for kind in ("needle", "anisotropic", "faint"):
        sc = scenes.frustum_scene(400, intr, rng, zmin=0.8, zmax=3.0)
        n = sc.n
        if kind == "needle":
            la = rng.integers(0, 3, n)
            sc.scales[:] = np.float32(0.0008)
            sc.scales[la, np.arange(n)] = rng.uniform(0.1, 0.8, n).astype(np.float32)
        elif kind == "anisotropic":
            sc.scales[:] = np.exp(rng.uniform(np.log(0.002), np.log(0.3), (3, n))).astype(np.float32)
        if kind == "faint":
            sc.opacity[:] = ((1.0 / 255.0) * np.exp(rng.uniform(1e-3, 0.04, n))).astype(np.float32)
        else:
            sc.opacity[:] = np.exp(rng.uniform(np.log(0.02), 0.0, n)).astype(np.float32)
        for r in brute.pinned(sc):
            if not r["visible"]:
                continue
            # sub-blocks holding an accepted pixel at a random place (often a
            # corner or an edge of the region the Gaussian reaches)
            px = rng.integers(r["xlo_raw"], r["xhi_raw"] + 1, 400)
            py = rng.integers(r["ylo_raw"], r["yhi_raw"] + 1, 400)
            ok = brute.pinned_q(r, px, py) <= r["qcut"]
            for x, y in list(zip(px[ok], py[ok]))[:12]:
                out.append((r, int(x) - int(rng.integers(0, 8)), int(y) - int(rng.integers(0, 8))))
    rng.shuffle(out)
    return out[:count] if len(out) > count else out


def _sums(r, X0, Y0, rng):
    ys, xs = np.mgrid[0:8, 0:8]
    X, Y = X0 + xs, Y0 + ys
    q = brute.pinned_q(r, X, Y)
    acc = q <= r["qcut"]
    if not acc.any():
        return None
    # per-pixel values of mixed sign where the Gaussian composites, 0 elsewhere
    e = np.where(acc, rng.standard_normal((8, 8)) * np.exp(rng.uniform(-3, 3, (8, 8))), 0.0).astype(np.float32)
    a, b, c = (float(r[k]) for k in "abc")
    ui, vi, uf, vf = r["ui"], r["vi"], float(r["uf"]), float(r["vf"])
    # binary64 reference from the pixels' own offsets (the binary32 ones of the recipe, exactly widened)
    dx = ((X - ui).astype(np.float32) - np.float32(uf)).astype(np.float64)
    dy = ((Y - vi).astype(np.float32) - np.float32(vf)).astype(np.float64)
    t1, t2 = a * dx + b * dy, c * dy
    e64 = e.astype(np.float64)
    ref = np.array([np.sum(e64 * t1), np.sum(e64 * t2), np.sum(e64 * t1 * dx), np.sum(e64 * t1 * dy),
                    np.sum(e64 * t2 * dy)])
    # binary32 moments about the sub-block centre, summed in binary32 in pixel order
    xi = (xs - 3.5).astype(np.float32)
    eta = (ys - 3.5).astype(np.float32)

    def s32(v):
        acc32 = np.float32(0.0)
        for t in v.reshape(-1):
            acc32 = np.float32(acc32 + np.float32(t))
        return acc32
    S1 = s32(e)
    Sx, Sy = s32(e * xi), s32(e * eta)
    Sxx, Sxy, Syy = s32(e * (xi * xi)), s32(e * (xi * eta)), s32(e * (eta * eta))
    U = _f(_f(_f(-(X0 - ui)) - _f(3.5)) + _f(uf))
    V = _f(_f(_f(-(Y0 - vi)) - _f(3.5)) + _f(vf))
    k1 = _fma(a, U, _f(_f(b) * V))
    P1 = _fma(a, Sx, _fma(b, Sy, -_f(k1 * S1)))
    P2 = _f(_f(c) * _fma(-V, S1, Sy))
    P1x = _f(_fma(a, Sxx, _fma(b, Sxy, -_f(k1 * Sx))) - _f(U * P1))
    P1y = _f(_fma(a, Sxy, _fma(b, Syy, -_f(k1 * Sy))) - _f(V * P1))
    P2y = _f(_f(c) * _fma(_f(V * V), S1, _fma(_f(-2.0 * V), Sy, Syy)))
    got = np.array([P1, P2, P1x, P1y, P2y], np.float64)
    S = float(np.sum(np.abs(e64)))
    L = 3.5 * (abs(a) + abs(b)) + abs(float(k1))
    M = 7.0 * abs(c) + math.sqrt(max(float(r["qcut"]), 0.0))
    bound = G * S * np.array([L, M, (3.5 + abs(float(U))) * L, (3.5 + abs(float(V))) * L,
                              (3.5 + abs(float(V))) * M]) + 1e-12 * np.abs(ref)
    return dict(ref=ref, got=got, bound=bound, a=a, b=b, c=c, U=float(U),
                V=float(V), k1=float(k1), qcut=float(r["qcut"]), S=S)


def test_factor_bounds_from_the_dilation():
    """|a|, |b|, |c| <= K / sqrt(0.3) for every projected Gaussian (the
    0.3 px^2 dilation bounds the inverse screen covariance)."""
    rng = np.random.default_rng(3)
    worst = 0.0
    for r, _, _ in _cases(rng, count=3000):
        worst = max(worst, abs(float(r["a"])), abs(float(r["b"])), abs(float(r["c"])))
    assert worst <= KMAX * (1 + 1e-6), (worst, KMAX)


def test_moment_form_meets_its_bound_where_it_is_tightest():
    rng = np.random.default_rng(17)
    checked = faint = far = corner = 0
    ratio = 0.0
    for r, X0, Y0 in _cases(rng):
        res = _sums(r, X0, Y0, rng)
        if res is None:
            continue
        err = np.abs(res["got"] - res["ref"])
        assert np.all(err <= res["bound"]), (err, res["bound"], res)
        ratio = max(ratio, float(np.max(err / res["bound"])))
        # |k1| stays within its stated maximum for every composited Gaussian
        assert abs(res["k1"]) <= 3.5 * (abs(res["a"]) + abs(res["b"])) + math.sqrt(max(res["qcut"], 0)) + 1e-3
        checked += 1
        faint += res["qcut"] < 0.1
        far += max(abs(res["U"]), abs(res["V"])) > 30
        corner += abs(res["k1"]) > 0.7 * (3.5 * (abs(res["a"]) + abs(res["b"])))
    # the cases reach the corners of the bound
    assert checked > 2000 and faint > 100 and far > 200 and corner > 100, (checked, faint, far, corner)
    print(f"{checked} (sub-block, Gaussian) cases ({faint} faint, {far} far-centred, {corner} corner); "
          f"worst error / bound {ratio:.3f}")

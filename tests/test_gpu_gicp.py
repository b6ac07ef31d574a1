"""GPU parity of the Generalized-ICP alignment (ms_gicp_*) against the
oracle: correspondences bit for bit (an integer decision in the same pinned
binary32 order on both sides), the normal equations (binary64 on both
sides) within 1e-9, and whole alignments -- exact recovery of a known
transform, and the room workload's iterations -- on point and Gaussian
sources, the full map or the candidates of the selection as targets, and
empty, non-finite and degenerate inputs."""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import gicp as G
from oracle import select as SEL
from paper_2412_09723_amd import scenes
from paper_2412_09723_amd.align import GeneralizedICP

pytestmark = pytest.mark.gpu
dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _sums(H, g, cost, cnt):
    iu = np.triu_indices(6)
    return np.concatenate([H[iu], g, [cost, cnt]])


def _check_sums(got, want):
    got = got.cpu().numpy()
    assert got[28] == want[28]
    Hs = np.abs(want[:21]).max()
    assert np.abs(got[:21] - want[:21]).max() <= 1e-9 * Hs
    gs = max(np.abs(want[21:27]).max(), 1e-300)
    assert np.abs(got[21:27] - want[21:27]).max() <= 1e-9 * max(gs, 1e-6 * Hs)
    assert abs(got[27] - want[27]) <= 1e-9 * abs(want[27])


def _room(n_src, seed=0):
    sc, src, Tt, T0 = scenes.gicp_scene(n_src, seed=seed)
    tgt = {"means": dev(sc.means), "scales": dev(sc.scales), "quats": dev(sc.quats)}
    return sc, src, Tt, T0, tgt


def test_room_correspondences_and_normal_equations():
    print("gicp room 20k sources, 1M targets", flush=True)
    sc, src, Tt, T0, tgt = _room(20000)
    g = GeneralizedICP(20000, sc.n)
    g.build(tgt)
    s = {"means": dev(src)}
    T = dev(T0)
    corr = g.correspond(s, T).cpu().numpy()
    want = G.correspond(T0, src, sc.means, 0.02)
    assert np.array_equal(corr, want) and (want >= 0).sum() > 15000
    tcov = G.quat_cov(sc.scales, sc.quats)
    out = g.normal_equations(s, tgt, T, dev(corr))
    _check_sums(out, _sums(*G.normal_equations(T0, src, None, sc.means, tcov, want)))
    # Gaussian sources: their covariance rotated by T
    rng = np.random.default_rng(1)
    ssc = np.exp(rng.uniform(np.log(0.002), np.log(0.02), (3, 20000))).astype(np.float32)
    sq = rng.standard_normal((4, 20000)).astype(np.float32)
    sg = {"means": dev(src), "scales": dev(ssc), "quats": dev(sq)}
    out = g.normal_equations(sg, tgt, T, dev(corr))
    _check_sums(out, _sums(*G.normal_equations(T0, src, G.quat_cov(ssc, sq), sc.means, tcov, want)))


def test_room_alignment_matches_the_oracle():
    print("gicp room alignment", flush=True)
    sc, src, Tt, T0, tgt = _room(20000, seed=1)
    g = GeneralizedICP(20000, sc.n)
    g.build(tgt)
    T = dev(T0)
    corr, hist = g.align({"means": dev(src)}, tgt, T, iters=6, history=True)
    torch.cuda.synchronize()
    Tw, whist, wcorr = G.align(T0, src, None, sc.means, G.quat_cov(sc.scales, sc.quats), iters=6)
    Tg = T.cpu().numpy()
    assert np.abs(Tg - Tw).max() <= 1e-6, np.abs(Tg - Tw).max()
    h = hist.cpu().numpy()
    for i, (cost, cnt) in enumerate(whist):
        assert abs(h[i, 28] - cnt) <= 2 and abs(h[i, 27] - cost) <= 1e-5 * cost, (i, h[i, 27:], cost, cnt)
    # the pose moves toward the truth and the cost falls (exact recovery is
    # the lattice test's; the noisy room map has its own optimum)
    assert np.abs(Tg - Tt).max() < np.abs(T0 - Tt).max() and h[-1, 27] < h[0, 27]


@pytest.mark.parametrize("targets", ["map", "candidates"])
def test_alignment_sums_equal_the_direct_normal_equations(targets):
    """ms_gicp_align reads each target from a per-entry record computed once
    per call; its sums equal, bit for bit, ms_gicp_normal_equations over the
    same correspondences, which reads the target map itself. Gaussian
    sources, the whole map or a candidate list as targets, the first and a
    later iteration."""
    print(f"gicp record path against the direct path, {targets}", flush=True)
    sc, src, Tt, T0, tgt = _room(20000, seed=3)
    rng = np.random.default_rng(4)
    ssc = np.exp(rng.uniform(np.log(0.002), np.log(0.02), (3, 20000))).astype(np.float32)
    sq = rng.standard_normal((4, 20000)).astype(np.float32)
    s = {"means": dev(src), "scales": dev(ssc), "quats": dev(sq)}
    g = GeneralizedICP(20000, sc.n)
    if targets == "map":
        g.build(tgt)
    else:
        cand = SEL.select(sc.means, sc.viewmat.reshape(-1)[:12].astype(np.float32), sc.intr, max_dist=3.0)
        assert 10000 < cand.size < sc.n
        g.build(tgt, dev(cand))
    T = dev(T0)
    for step in range(2):
        Tk = T.clone()
        corr, hist = g.align(s, tgt, T, iters=1, history=True)
        direct = g.normal_equations(s, tgt, Tk, corr)
        torch.cuda.synchronize()
        assert (corr >= 0).sum().item() > 5000, step
        assert torch.equal(hist[0], direct), (step, (hist[0] - direct).abs().max().item())


def test_known_transform_and_selected_targets():
    print("gicp lattice recovery", flush=True)
    rng = np.random.default_rng(2)
    side = 12
    idx = np.stack(np.meshgrid(*[np.arange(side)] * 3, indexing="ij"), 0).reshape(3, -1)
    tgt_np = (idx * 0.1 + rng.uniform(-0.02, 0.02, idx.shape) + 1.0).astype(np.float32)
    n = tgt_np.shape[1]
    ts = np.exp(rng.uniform(np.log(0.002), np.log(0.03), (3, n))).astype(np.float32)
    tq = rng.standard_normal((4, n)).astype(np.float32)
    R = Rotation.from_rotvec(np.deg2rad(8.0) * rng.standard_normal(3) / math.sqrt(3)).as_matrix()
    Tt = np.concatenate([R, rng.normal(0, 0.3, (3, 1))], axis=1)
    src = (R.T @ (tgt_np.astype(np.float64) - Tt[:, 3:])).astype(np.float32)
    Rp = Rotation.from_rotvec(np.deg2rad(0.2) * rng.standard_normal(3) / math.sqrt(3)).as_matrix()
    T0 = np.concatenate([Rp @ R, (Rp @ Tt[:, 3] + rng.normal(0, 0.004, 3))[:, None]], axis=1)
    T0 = T0.reshape(12).astype(np.float32)
    tgt = {"means": dev(tgt_np), "scales": dev(ts), "quats": dev(tq)}
    g = GeneralizedICP(n, n)
    g.build(tgt)
    T = dev(T0)
    corr, _ = g.align({"means": dev(src)}, tgt, T, iters=8)
    assert np.array_equal(corr.cpu().numpy(), np.arange(n))
    assert np.abs(T.cpu().numpy() - Tt.reshape(12)).max() <= 2e-6
    # targets given as an index list (a candidate set): the same alignment on a subset
    vm = np.array([1, 0, 0, -1.55, 0, 1, 0, -1.55, 0, 0, 1, 0.5], np.float32)   # the lattice in view
    intr = scenes.Intrinsics(200, 200, 150.0, 150.0, 100.0, 100.0)
    cand = SEL.select(tgt_np, vm, intr, max_dist=2.2)
    assert 100 < cand.size < n
    g.build(tgt, dev(cand))
    T = dev(T0)
    corr = g.correspond({"means": dev(src)}, T).cpu().numpy()
    sub = np.full(n, -1)
    sub[cand] = cand
    want = G.correspond(T0, src, tgt_np[:, cand], 0.02)
    want = np.where(want >= 0, cand[np.maximum(want, 0)], -1)
    assert np.array_equal(corr, want)


def test_empty_degenerate_and_dense():
    g = GeneralizedICP(4096, 4096)
    I = dev(np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], np.float32))
    empty = {"means": torch.zeros((3, 0), device="cuda")}
    rng = np.random.default_rng(3)
    pts = rng.uniform(0, 0.3, (3, 4096)).astype(np.float32)      # dense: many candidates per cell
    g.build(empty)
    assert (g.correspond({"means": dev(pts)}, I) == -1).all()
    T = I.clone()
    _, hist = g.align({"means": dev(pts)}, empty, T, iters=2, history=True)
    assert torch.equal(T, I) and hist[:, 28].sum().item() == 0      # no correspondences: T stays
    tg = rng.uniform(0, 0.3, (3, 3000)).astype(np.float32)
    tg[:, 5] = np.nan
    src = pts.copy()
    src[:, 7] = np.inf
    g.build({"means": dev(tg)})
    Tn = np.array([1, 0, 0, 0.001, 0, 1, 0, -0.002, 0, 0, 1, 0.0005], np.float32)
    got = g.correspond({"means": dev(src)}, dev(Tn)).cpu().numpy()
    assert np.array_equal(got, G.correspond(Tn, src, tg, 0.02))
    assert got[7] == -1
    assert g.correspond(empty, I).numel() == 0

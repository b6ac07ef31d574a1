"""Helpers for the GPU parity tests: move scenes to the device and compare the
HIP path with the oracle."""
import numpy as np
import torch

import oracle
from paper_2412_09723_amd import raster


def to_dev(sc, device="cuda"):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    m = dict(means=t(sc.means), scales=t(sc.scales), quats=t(sc.quats), opacity=t(sc.opacity), colors=t(sc.colors))
    return m, t(sc.viewmat)


def run_job(sc, tile=16, wave_batch=64, cap=None, check=True, scalar=False, bin_tile=0, bwd=None):
    m, vm = to_dev(sc)
    mode = "scalar" if scalar else "lds"
    opts = raster.RenderOptions(tile=tile, wave_batch=wave_batch, pair_capacity=cap, check=check,
                                fwd_records=mode, bwd_records=bwd or mode, bin_tile=bin_tile)
    job = raster.Job(m, vm, sc.intr, opts)
    rgb, depth, sil = job.forward()
    return job, (rgb, depth, sil)


def expected_order(pr):
    vis = np.flatnonzero(pr["visible"])
    return vis[np.lexsort((vis, pr["zkey"][vis]))]


def check_structure(job, sc, tile):
    """Keys, records and bin lists: bit-exact with the oracle. Lists hold
    depth ranks into rank-order records (list kind 0) or Gaussian indices into
    index-order records (kind 1); both must give the oracle's (depth, index)
    order in every bin."""
    pr = oracle.project(sc)
    st = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in job.state().items()}
    nv, K = int(st["counters"][0]), int(st["counters"][1])
    assert not st["counters"][2], "pair capacity overflow"
    assert nv == int(pr["visible"].sum())
    zk = np.where(pr["visible"] == 1, pr["zkey"], np.uint32(0xFFFFFFFF))
    assert np.array_equal(st["depth_key"].view(np.uint32)[:sc.n], zk)
    order = expected_order(pr)
    if st["list_kind"] == 0:
        assert np.array_equal(st["sorted_index"].view(np.uint32)[:nv], order.astype(np.uint32))
        rec = st["records"][:nv].view(np.uint32)
        idx = rec[:, 15].astype(np.int64)
        assert np.array_equal(idx, order)
        rank_of = st["rank_of"][:sc.n]
        assert np.array_equal(rank_of[order], np.arange(nv))
    else:
        idx = np.flatnonzero(pr["visible"])
        rec = st["records"][idx].view(np.uint32)
        assert np.array_equal(rec[:, 15].astype(np.int64), idx)
    assert np.array_equal(rec[:, 0].view(np.float32), pr["ctr"][0][idx].astype(np.float32))
    assert np.array_equal(rec[:, 1].view(np.float32), pr["ctr"][1][idx].astype(np.float32))
    for w, k in ((2, 0), (3, 1), (4, 2), (5, 3), (6, 4), (7, 5)):
        assert np.array_equal(rec[:, w], pr["rec"][k][idx].view(np.uint32)), f"record word {w}"
    assert np.array_equal(rec[:, 9], pr["zkey"][idx])
    bb = pr["bbox"][:, idx].astype(np.uint32)
    assert np.array_equal(rec[:, 13], bb[0] | (bb[1] << 16))
    assert np.array_equal(rec[:, 14], bb[2] | (bb[3] << 16))
    # bin lists
    W, H = sc.intr.width, sc.intr.height
    off, ids = oracle.tile_lists(pr, W, H, tile)
    assert K == len(ids)
    tr = st["tile_range"].view(np.uint32).astype(np.int64)
    lens = tr[:, 1] - tr[:, 0]
    assert np.array_equal(lens, np.diff(off))
    nonempty = lens > 0
    assert np.array_equal(tr[nonempty, 0], off[:-1][nonempty])
    entries = st["pair_rank"][:K].view(np.uint32).astype(np.int64)
    if st["list_kind"] == 0:
        assert np.array_equal(order[entries], ids.astype(np.int64))
        tiles_of = st["pair_tile"][:K].view(np.uint32)
        assert np.array_equal(tiles_of, np.repeat(np.arange(len(lens)), lens).astype(np.uint32))
    else:
        assert np.array_equal(entries, ids.astype(np.int64))
    return pr, st


def rel_err(got, ref, floor_frac=1e-3):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    floor = floor_frac * max(float(np.abs(ref).max()), 1e-300)
    return np.abs(got - ref) / np.maximum(np.abs(ref), floor)


def check_images(imgs, ref, tol=1e-4):
    """Max relative error of RGB, depth and silhouette vs the oracle, on pixels
    whose stop decision is outside its margin; returns (max errors, flagged)."""
    rgb, depth, sil = (t.cpu().numpy() for t in imgs)
    ok = (ref["flags"] & 1) == 0
    e_rgb = rel_err(rgb, ref["rgb"])[:, ok].max(initial=0.0)
    e_d = rel_err(depth, ref["depth"])[ok].max(initial=0.0)
    e_s = rel_err(sil, ref["sil"])[ok].max(initial=0.0)
    assert np.isfinite(rgb).all() and np.isfinite(depth).all() and np.isfinite(sil).all()
    assert e_rgb <= tol and e_d <= tol and e_s <= tol, (e_rgb, e_d, e_s, int((~ok).sum()))
    return (e_rgb, e_d, e_s), int((~ok).sum())


def check_grads(g, ref, tol=1e-3, pose=True, map_grads=True):
    """Elementwise |g - o| <= tol * max(|o|, 1e-2 ||o||_inf) on Gaussians not
    flagged by the margin protocol, plus a normwise bound on everything."""
    keep = ref["gflags"] == 0
    worst = {}
    if map_grads:
        for k, rows in (("means", 3), ("scales", 3), ("quats", 4), ("opacity", 1), ("colors", 3)):
            got = g[k].detach().cpu().numpy().astype(np.float64).reshape(rows, -1)
            o = np.asarray(ref[k], np.float64).reshape(rows, -1)
            scale = max(float(np.abs(o).max()), 1e-30)
            err = np.abs(got - o) / np.maximum(np.abs(o), 1e-2 * scale)
            e = float(err[:, keep].max(initial=0.0))
            nrm = float(np.linalg.norm(got - o) / max(np.linalg.norm(o), 1e-30))
            worst[k] = (e, nrm)
            assert np.isfinite(got).all(), k
            assert e <= tol, (k, e, int(np.argmax(err.max(axis=0))))
            assert nrm <= tol, (k, nrm)
    if pose:
        for k in ("viewmat", "twist"):
            got = g[k].detach().cpu().numpy().astype(np.float64)
            o = np.asarray(ref[k], np.float64)
            e = float(np.abs(got - o).max() / max(np.abs(o).max(), 1e-30))
            worst[k] = e
            assert e <= tol, (k, e, got, o)
    return worst


def check_reordered_grads(gb, ga, keys):
    """The same gradient terms summed by atomics in another order: compared at
    the gradient tolerance, 1e-3 elementwise with a floor of 1e-2 of the
    tensor maximum, and 1e-3 normwise."""
    for k in keys:
        a, b = ga[k].cpu().numpy().astype(np.float64), gb[k].cpu().numpy().astype(np.float64)
        scale = max(np.abs(a).max(initial=0.0), 1e-30)
        err = np.abs(b - a) / np.maximum(np.abs(a), 1e-2 * scale)
        assert err.max(initial=0.0) <= 1e-3, (k, float(err.max()))
        assert np.linalg.norm(b - a) <= 1e-3 * max(np.linalg.norm(a), 1e-30), k

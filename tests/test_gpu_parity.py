"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Discrete structure (depth keys, projected records, depth order, per-tile
lists) bit-exact; RGB, depth and silhouette within 1e-4 max relative error
(floor 1e-3 of the image maximum) on pixels whose stop decision lies outside
its 1e-4 margin; gradients within 1e-3 (floor 1e-2 of the tensor maximum)
elementwise on Gaussians outside the margin protocol, and normwise on all.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2412_09723_amd import raster, scenes
from tests.gpu_util import check_grads, check_images, check_reordered_grads, check_structure, run_job, to_dev
from tests.helpers import make_scene

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def _up(sc, w_depth=1.0, w_sil=0.5, salt=2):
    return scenes.upstream_grads(sc.intr, scenes.rng_for(0, 0, salt=salt), w_depth, w_sil)


def _dev_grads(g):
    return [torch.from_numpy(a).cuda() for a in g]


@pytest.mark.parametrize("tile,wb,scalar,bin_tile,bwd", [
    (16, 64, False, 0, None), (8, 32, False, 0, None), (32, 128, False, 0, None), (16, 128, False, 0, None),
    (8, 64, False, 0, None), (32, 32, False, 0, None), (8, 64, True, 0, None), (16, 64, True, 0, None),
    (32, 64, True, 0, None), (16, 64, False, 64, None), (16, 64, True, 128, None), (32, 64, False, 128, None),
    (8, 32, True, 32, None), (16, 64, False, 128, "mfma"), (8, 64, False, 0, "mfma"), (16, 64, True, 0, "mfma"),
    (32, 64, False, 128, "mfma"), (32, 128, False, 0, "mfma"), (16, 64, False, 128, "mfma_bf16x3"),
    (8, 64, False, 0, "mfma_bf16x3")])
def test_small_frustum_forward_backward(tile, wb, scalar, bin_tile, bwd):
    _log(f"small_frustum tile={tile} wb={wb} scalar={scalar} bin={bin_tile} bwd={bwd}")
    sc = scenes.small_frustum()
    job, imgs = run_job(sc, tile=tile, wave_batch=wb, scalar=scalar, bin_tile=bin_tile, bwd=bwd)
    check_structure(job, sc, bin_tile or tile)
    ref = oracle.forward(sc)
    errs, flagged = check_images(imgs, ref)
    _log(f"  image max rel err {errs}, flagged {flagged}")
    up = _up(sc)
    g = job.backward(*_dev_grads(up))
    torch.cuda.synchronize()
    rb = oracle.backward(sc, *up)
    worst = check_grads(g, rb)
    _log(f"  grad worst {worst}")


def test_rotated_pose_and_ragged_image():
    _log("ragged 37x23 rotated pose")
    from scipy.spatial.transform import Rotation
    intr = scenes.Intrinsics(37, 23, 30.0, 31.0, 18.3, 11.1)
    R0 = Rotation.from_euler("xyz", [6, -4, 9], degrees=True).as_matrix()
    vm = np.concatenate([R0, np.array([[0.04], [-0.03], [0.1]])], axis=1).reshape(12).astype(np.float32)
    sc = scenes.frustum_scene(700, intr, scenes.rng_for(9, 77), viewmat=vm)
    sc.means[0, :20] *= 2.5           # some centres off-screen
    sc.means[2, 20:25] = 0.1          # behind the near plane
    for tile, scalar, bwd in ((8, False, None), (16, False, None), (32, False, None), (8, True, None),
                              (16, True, None), (32, True, None), (8, False, "mfma"), (16, False, "mfma"),
                              (32, False, "mfma"), (16, False, "mfma_bf16x3")):
        job, imgs = run_job(sc, tile=tile, wave_batch=32, scalar=scalar, bwd=bwd)
        check_structure(job, sc, tile)
        ref = oracle.forward(sc)
        check_images(imgs, ref)
        up = _up(sc, 1.0, 1.0, salt=5)
        g = job.backward(*_dev_grads(up))
        check_grads(g, oracle.backward(sc, *up))


@pytest.mark.parametrize("scalar,tile,bin_tile,bwd", [(False, 16, 0, None), (True, 16, 0, None),
                                                     (False, 32, 128, None), (False, 16, 128, "mfma"),
                                                     (False, 32, 128, "mfma"), (False, 32, 256, "mfma"),
                                                     (False, 16, 128, "mfma_bf16x3")])
def test_room_1m_full_size(scalar, tile, bin_tile, bwd):
    """1200x680, 1M Gaussians (the benchmark workload). Bin 0 (3225 bins)
    takes the global depth-sort path, bins of 128 the per-bin sort, and bins
    of 256 hold up to 30k pairs each, beyond one block's in-LDS sort. The
    upstream gradient carries a silhouette term, so the G_S T_final / (1 -
    alpha) part of every composited Gaussian's gradient is exercised at full
    size."""
    _log(f"room_view full size scalar={scalar} tile={tile} bin={bin_tile} bwd={bwd}")
    sc = scenes.room_view()
    job, imgs = run_job(sc, tile=tile, wave_batch=64, scalar=scalar, bin_tile=bin_tile, bwd=bwd)
    check_structure(job, sc, bin_tile or tile)
    ref = oracle.forward(sc)
    errs, flagged = check_images(imgs, ref)
    _log(f"  image max rel err {errs}, flagged {flagged}")
    up = _up(sc, 0.5, 0.5)
    g = job.backward(*_dev_grads(up))
    torch.cuda.synchronize()
    worst = check_grads(g, oracle.backward(sc, *up))
    _log(f"  grad worst {worst}")


def test_empty_map_and_all_culled():
    _log("empty / culled")
    intr = scenes.Intrinsics(40, 30, 40.0, 40.0, 20.0, 15.0)
    empty = make_scene(np.zeros((3, 0)), np.zeros((3, 0)), np.zeros((4, 0)), np.zeros(0), np.zeros((3, 0)), intr)
    job, (rgb, depth, sil) = run_job(empty)
    assert not rgb.any() and not depth.any() and not sil.any()
    g = job.backward(*_dev_grads(_up(empty)))
    assert not g["twist"].any() and not g["viewmat"].any()
    behind = make_scene([[0, 0, np.nan], [0, 0, 0], [-1.0, 0.1, 2.0]], np.full((3, 3), 0.05),
                        np.tile([[1], [0], [0], [0]], 3), [0.5] * 3, np.ones((3, 3)), intr)
    job, (rgb, depth, sil) = run_job(behind)
    assert not rgb.any() and job.stats()["visible"] == 0
    g = job.backward(*_dev_grads(_up(behind)))
    for k in ("means", "scales", "quats", "opacity", "colors"):
        assert not g[k].any()


def test_capacity_overflow_is_reported_not_truncated():
    _log("overflow")
    sc = scenes.small_frustum()
    m, vm = to_dev(sc)
    from paper_2412_09723_amd import raster, _lib
    job = raster.Job(m, vm, sc.intr, raster.RenderOptions(pair_capacity=1000))
    rgb, depth, sil = job.forward()
    st = job.stats()
    assert st["overflow"] and st["pairs"] > 1000
    assert torch.isnan(rgb).all() and torch.isnan(depth).all()
    g = job.backward(*_dev_grads(_up(sc)))
    assert torch.isnan(g["twist"]).all()
    with pytest.raises(_lib.MacsplatError):
        raster.Job(m, vm, sc.intr, raster.RenderOptions(pair_capacity=1000, check=True, grow=False)).forward()
    grown = raster.Job(m, vm, sc.intr, raster.RenderOptions(pair_capacity=1000, check=True))
    rgb2, _, _ = grown.forward()
    assert grown.cap >= st["pairs"] and not grown.stats()["overflow"] and torch.isfinite(rgb2).all()


def test_repeat_determinism_of_forward():
    """Forward images and discrete state are bitwise identical across runs
    (no atomics in the forward)."""
    _log("determinism")
    sc = scenes.small_frustum()
    job, imgs = run_job(sc, tile=16, wave_batch=64)
    a = [t.clone() for t in imgs]
    s1 = job.state()["pair_rank"].clone()
    imgs2 = job.forward()
    for x, y in zip(a, imgs2):
        assert torch.equal(x, y)
    assert torch.equal(s1, job.state()["pair_rank"])


def test_pose_only_and_map_only_flags():
    _log("flags")
    sc = scenes.small_frustum()
    job, _ = run_job(sc)
    up = _dev_grads(_up(sc))
    full = job.backward(*up)
    pose = job.backward(*up, map_grads=False)
    mapg = job.backward(*up, pose_grads=False)
    assert set(pose) == {"viewmat", "twist"}
    assert "twist" not in mapg
    assert torch.allclose(pose["twist"], full["twist"], rtol=1e-5, atol=1e-9)
    assert torch.allclose(mapg["means"], full["means"], rtol=1e-4, atol=1e-9)


@pytest.mark.parametrize("W,H,tile", [(160, 120, 16), (160, 120, 8), (400, 300, 8)])
def test_exact_depth_ties_keep_index_order(W, H, tile):
    """Many Gaussians at exactly the same depth (identity pose, three depth
    values): every bin list must hold them in index order, on the per-bin
    sort path (the first two cases) and on the global sort path (1900 bins)."""
    _log(f"depth ties {W}x{H} tile {tile}")
    intr = scenes.Intrinsics(W, H, 150.0, 150.0, W / 2.0, H / 2.0)
    sc = scenes.frustum_scene(3000, intr, scenes.rng_for(9, 123))
    z = np.array([2.0, 2.5, 3.0], np.float32)[np.arange(sc.n) % 3]
    sc.means[0] *= z / sc.means[2]
    sc.means[1] *= z / sc.means[2]
    sc.means[2] = z
    job, imgs = run_job(sc, tile=tile, wave_batch=64, bwd="mfma")
    _, st = check_structure(job, sc, tile)
    assert st["list_kind"] == (1 if (W // tile) * (H // tile) <= 1024 else 0)
    check_images(imgs, oracle.forward(sc))
    up = _up(sc)
    g = job.backward(*_dev_grads(up))
    torch.cuda.synchronize()
    check_grads(g, oracle.backward(sc, *up))


@pytest.mark.parametrize("tile,wb,bwd", [(16, 64, "mfma"), (8, 32, "mfma"), (32, 128, "mfma"),
                                         (16, 64, "mfma_bf16x3")])
def test_needle_gaussians_grazing_sub_blocks(tile, wb, bwd):
    """Thin, strongly anisotropic Gaussians at random orientations, with
    opacities down to the 1/255 cut-off: their acceptance ellipses cover a
    small part of their pixel boxes and graze many 8x8 sub-blocks, which is
    where the compositing kernels' record skipping must stay conservative."""
    _log(f"needles tile {tile} wb {wb} bwd {bwd}")
    intr = scenes.Intrinsics(160, 120, 150.0, 150.0, 80.0, 60.0)
    rng = scenes.rng_for(9, 321)
    sc = scenes.frustum_scene(2500, intr, rng, zmin=1.0, zmax=4.0)
    n = sc.n
    long_axis = rng.integers(0, 3, size=n)
    sc.scales[:] = np.float32(0.0015)
    sc.scales[long_axis, np.arange(n)] = rng.uniform(0.05, 0.4, size=n).astype(np.float32)
    sc.opacity[:] = np.exp(rng.uniform(np.log(1.0 / 255.0), 0.0, size=n)).astype(np.float32)
    job, imgs = run_job(sc, tile=tile, wave_batch=wb, bwd=bwd)
    check_structure(job, sc, tile)
    errs, flagged = check_images(imgs, oracle.forward(sc))
    _log(f"  image max rel err {errs}, flagged {flagged}")
    up = _up(sc, 1.0, 1.0, salt=7)
    g = job.backward(*_dev_grads(up))
    torch.cuda.synchronize()
    _log(f"  grad worst {check_grads(g, oracle.backward(sc, *up))}")


@pytest.mark.parametrize("W,H,tile,bin_tile", [(16384, 8, 16, 128), (8, 16384, 8, 0), (1, 1, 16, 0), (1, 700, 8, 0),
                                               (16384, 24, 32, 0)])
def test_extreme_image_shapes(W, H, tile, bin_tile):
    """The largest image edge the ABI accepts, one-pixel images and strips,
    where almost every bin, tile and sub-block is ragged: (16384, 8) has 128
    bins of 128 px in one row; (16384, 24) at tile 32 has 512 bins of one
    tile each; (8, 16384) at tile 8 has 2048 bins (the global sort path)."""
    _log(f"shape {W}x{H} tile {tile} bin {bin_tile}")
    f = 200.0
    intr = scenes.Intrinsics(W, H, f, f, W / 2.0, H / 2.0)
    sc = scenes.frustum_scene(1500, intr, scenes.rng_for(9, 400 + W % 97 + H % 89), zmin=1.0, zmax=3.0)
    job, imgs = run_job(sc, tile=tile, wave_batch=32, bin_tile=bin_tile, bwd="mfma")
    check_structure(job, sc, bin_tile or tile)
    check_images(imgs, oracle.forward(sc))
    up = _up(sc, 1.0, 1.0, salt=9)
    g = job.backward(*_dev_grads(up))
    torch.cuda.synchronize()
    check_grads(g, oracle.backward(sc, *up))


def test_degenerate_gaussians_mixed_into_a_scene():
    """A scene with degenerate Gaussians sprinkled in: zero-norm rotation,
    zero, tiny, NaN and huge scales, non-finite colour and opacity, opacity 0
    and 1, a centre far outside the guard band, one on the near plane. The
    structure, images and gradients must match the oracle, which culls the
    same ones; culled Gaussians get exactly zero gradients."""
    _log("degenerate mix")
    intr = scenes.Intrinsics(96, 72, 90.0, 90.0, 48.0, 36.0)
    sc = scenes.frustum_scene(600, intr, scenes.rng_for(9, 555))
    sc.quats[:, 0] = 0.0                       # zero-norm rotation
    sc.scales[:, 1] = 0.0                      # zero scale: dilation only
    sc.scales[:, 2] = 1e-7                     # tiny
    sc.scales[0, 3] = np.nan                   # non-finite scale
    sc.scales[:, 4] = 5e3                      # far beyond the 2D variance limit
    sc.colors[1, 5] = np.inf                   # non-finite colour
    sc.opacity[6] = np.nan                     # non-finite opacity
    sc.opacity[7] = 0.0                        # never accepted
    sc.opacity[8] = 1.0                        # clamped alpha
    sc.means[0, 9] = sc.means[2, 9] * 1e5      # centre far outside the guard band
    sc.means[2, 10] = 0.2                      # on the near plane
    job, imgs = run_job(sc, tile=16, wave_batch=64, bwd="mfma")
    pr, _ = check_structure(job, sc, 16)
    check_images(imgs, oracle.forward(sc))
    up = _up(sc, 1.0, 1.0, salt=11)
    g = job.backward(*_dev_grads(up))
    torch.cuda.synchronize()
    check_grads(g, oracle.backward(sc, *up))
    culled = np.flatnonzero(pr["visible"] == 0)
    assert len(culled) >= 5
    for k in ("means", "scales", "quats", "opacity", "colors"):
        a = g[k].detach().cpu().numpy().reshape(-1, sc.n)
        assert not a[:, culled].any(), k


def test_long_bin_segment_with_depth_ties():
    """One bin holding 20000 pairs (more than a workgroup sorts in LDS), with
    exact depth ties: the chunked global-memory sort must keep (depth, index)
    order too."""
    _log("long segment with ties")
    intr = scenes.Intrinsics(48, 40, 60.0, 60.0, 24.0, 20.0)
    sc = scenes.frustum_scene(20000, intr, scenes.rng_for(9, 777))
    z = np.array([2.0, 2.5, 3.0, 3.5], np.float32)[np.arange(sc.n) % 4]
    sc.means[0] *= z / sc.means[2]
    sc.means[1] *= z / sc.means[2]
    sc.means[2] = z
    job, imgs = run_job(sc, tile=16, wave_batch=64, bin_tile=128, bwd="mfma")
    _, st = check_structure(job, sc, 128)
    assert st["list_kind"] == 1
    lens = st["tile_range"].view(np.uint32).astype(np.int64)
    assert (lens[:, 1] - lens[:, 0]).max() > 16384
    check_images(imgs, oracle.forward(sc))
    up = _up(sc)
    g = job.backward(*_dev_grads(up))
    torch.cuda.synchronize()
    check_grads(g, oracle.backward(sc, *up))


@pytest.mark.parametrize("bwd,schedule", [("mfma", "grid"), ("mfma", "queue"), ("mfma_bf16x3", "grid"),
                                          ("lds", "grid"), ("scalar", "grid")])
def test_stale_gradient_arrays_are_overwritten(bwd, schedule):
    """Gradient arrays filled with stale values beforehand: every Gaussian's
    gradient is written, the culled ones with exact zeros, the rest as in a
    backward into fresh arrays, on every backward variant and schedule."""
    _log(f"stale gradient arrays bwd={bwd} schedule={schedule}")
    sc = scenes.small_frustum()
    sc.means[2, :300] = -1.0                    # behind the camera: culled
    sc.means[0, 300:400] *= 40.0                # far outside the guard band: culled
    m, vm = to_dev(sc)
    opts = raster.RenderOptions(check=True, bwd_records=bwd, fwd_records="scalar" if bwd == "scalar" else "lds",
                                schedule=schedule)
    job = raster.Job(m, vm, sc.intr, opts)
    job.forward()
    up = _dev_grads(_up(sc))
    fresh = {k: v.clone() for k, v in job.backward(*up).items()}
    stale = {k: torch.full_like(m[k], 7.0) for k in ("means", "scales", "quats", "opacity", "colors")}
    stale["viewmat"] = torch.full((12,), 7.0, device="cuda")
    stale["twist"] = torch.full((6,), 7.0, device="cuda")
    got = job.backward(*up, out=stale)
    torch.cuda.synchronize()
    culled = job.state()["depth_key"].cpu().numpy().view(np.uint32)[:sc.n] == 0xFFFFFFFF
    assert culled.sum() >= 350
    for k in ("means", "scales", "quats", "opacity", "colors"):
        a = got[k].cpu().numpy().reshape(-1, sc.n)
        assert not a[:, culled].any(), k
        assert np.isfinite(a).all() and (a != 7.0).any(), k
    check_reordered_grads(got, fresh, ("means", "scales", "quats", "opacity", "colors", "viewmat", "twist"))


@pytest.mark.parametrize("bwd", ["mfma", "mfma_bf16x3"])
def test_stale_gradient_arrays_sparse_visibility(bwd):
    """Four of every five Gaussians culled (behind the camera): the
    projection adjoint packs a block's few visible Gaussians onto its first
    threads and hands their gradients to the slots' owners through LDS, and
    each owner writes its slot (zero when culled) into stale arrays. Every
    gradient against the oracle, the culled ones exactly zero."""
    _log(f"stale gradient arrays, sparse visibility, bwd={bwd}")
    sc = scenes.small_frustum()
    idx = np.arange(sc.n)
    sc.means[2, idx % 5 != 0] = -1.0
    m, vm = to_dev(sc)
    job = raster.Job(m, vm, sc.intr, raster.RenderOptions(check=True, bwd_records=bwd))
    job.forward()
    up = _up(sc)
    stale = {k: torch.full_like(m[k], 7.0) for k in ("means", "scales", "quats", "opacity", "colors")}
    stale["viewmat"] = torch.full((12,), 7.0, device="cuda")
    stale["twist"] = torch.full((6,), 7.0, device="cuda")
    got = job.backward(*_dev_grads(up), out=stale)
    torch.cuda.synchronize()
    culled = job.state()["depth_key"].cpu().numpy().view(np.uint32)[:sc.n] == 0xFFFFFFFF
    assert culled.sum() >= 4 * sc.n // 5
    per_block = np.add.reduceat((~culled).astype(np.int64), np.arange(0, sc.n, 1024))
    assert per_block.max() <= 256, per_block
    for k in ("means", "scales", "quats", "opacity", "colors"):
        a = got[k].cpu().numpy().reshape(-1, sc.n)
        assert not a[:, culled].any(), k
        assert np.isfinite(a).all(), k
    check_grads(got, oracle.backward(sc, *up))

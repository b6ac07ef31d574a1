"""Seeded synthetic inputs: determinism and the distributions they promise."""
import math

import numpy as np

from paper_2412_09723_amd import scenes


def test_config0_deterministic_and_shaped():
    a, b = scenes.small_frustum(), scenes.small_frustum()
    for k in ("means", "scales", "quats", "opacity", "colors", "viewmat"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    assert a.means.shape == (3, 4096) and a.means.dtype == np.float32
    assert a.quats.shape == (4, 4096)
    assert a.intr == scenes.Intrinsics(160, 120, 150.0, 150.0, 80.0, 60.0)


def test_config0_distributions():
    s = scenes.small_frustum()
    z = s.means[2]
    assert z.min() >= 1.0 and z.max() <= 5.0
    u = s.intr.fx * s.means[0] / z + s.intr.cx
    v = s.intr.fy * s.means[1] / z + s.intr.cy
    assert u.min() >= -1e-3 and u.max() <= 160 + 1e-3
    assert v.min() >= -1e-3 and v.max() <= 120 + 1e-3
    ls = np.log(s.scales)
    assert ls.min() >= math.log(0.01) - 1e-6 and ls.max() <= math.log(0.1) + 1e-6
    assert abs(ls.mean() - 0.5 * (math.log(0.01) + math.log(0.1))) < 0.05
    assert np.allclose(np.linalg.norm(s.quats, axis=0), 1.0, atol=1e-6)
    logit = np.log(s.opacity / (1 - s.opacity))
    assert abs(logit.mean()) < 0.08 and abs(logit.std() - 1.0) < 0.05
    assert s.colors.min() >= 0 and s.colors.max() <= 1


def test_room_split_and_bounds():
    rng = scenes.rng_for(1, 0)
    pts = scenes.room_scene(20000, rng)
    on_face = ((np.abs(pts[0]) < 0.1) | (np.abs(pts[0] - 6) < 0.1) | (np.abs(pts[1]) < 0.1)
               | (np.abs(pts[1] - 4) < 0.1) | (np.abs(pts[2]) < 0.1) | (np.abs(pts[2] - 3) < 0.1))
    frac = on_face.mean()
    # 70% planar plus the volumetric points that happen to fall within 10 cm of a face
    assert 0.70 < frac < 0.80
    assert pts.min() > -0.2 and pts[0].max() < 6.2


def test_room_pose_looks_along_x():
    vm = scenes.room_center_pose().reshape(3, 4).astype(np.float64)
    R, t = vm[:, :3], vm[:, 3]
    assert np.allclose(R @ R.T, np.eye(3))
    assert np.isclose(np.linalg.det(R), 1.0)
    centre = -R.T @ t
    assert np.allclose(centre, [3, 2, 1.5])
    assert np.allclose(R[2], [1, 0, 0])


def test_perturb_pose_magnitudes():
    vm = scenes.room_center_pose()
    p = scenes.perturb_pose(vm, scenes.rng_for(1, 0, salt=3))
    A = vm.reshape(3, 4).astype(np.float64)
    B = p.reshape(3, 4).astype(np.float64)
    dR = B[:, :3] @ A[:, :3].T
    ang = math.degrees(math.acos(max(-1.0, min(1.0, (np.trace(dR) - 1) / 2))))
    assert abs(ang - 1.0) < 1e-3
    dt = B[:, 3] - dR @ A[:, 3]
    assert abs(np.linalg.norm(dt) - 0.02) < 1e-6


def test_upstream_grads_shape_and_scale():
    intr = scenes.SMALL_INTR
    gc, gd, gs = scenes.upstream_grads(intr, scenes.rng_for(0, 0, salt=2), 0.5, 0.0)
    assert gc.shape == (3, 120, 160) and gd.shape == (120, 160)
    assert np.allclose(np.abs(gc), 1.0 / (3 * 120 * 160))
    assert np.allclose(np.abs(gd), 0.5 / (120 * 160))
    assert not gs.any()


def test_poisson_trace_reproducible():
    a = scenes.poisson_trace(8, 30.0, 2.0, seed=5)
    b = scenes.poisson_trace(8, 30.0, 2.0, seed=5)
    assert a == b
    assert 8 * 30 * 2 * 0.7 < len(a) < 8 * 30 * 2 * 1.3
    assert all(a[i][0] <= a[i + 1][0] for i in range(len(a) - 1))


def test_autotune_shape_key_buckets_sizes():
    from paper_2412_09723_amd import autotune, scenes
    i1, i2 = scenes.ROOM_INTR, scenes.VGA_INTR
    assert autotune.shape_key([1000, 5000], [i1, i2]) == autotune.shape_key([1023, 4097], [i1, i2])
    assert autotune.shape_key([1000], [i1]) != autotune.shape_key([1000], [i2])
    assert autotune.shape_key([1000, 5000], [i1, i2]).startswith("2|")

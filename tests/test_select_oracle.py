"""Pins of the candidate-selection oracle (oracle/select.py) against the two
criteria of Sec. 3.4 "1) Selection" stated without its recipe: hand-made
means on each side of every inclusive or strict threshold, and, on random
maps under rotated poses, a re-derivation through the camera centre
c = -R^T t and the 3x4 projection matrix K [R|t] (numpy matrix products),
away from the thresholds by a stated relative margin."""
import numpy as np
from scipy.spatial.transform import Rotation

from oracle import select as SEL
from paper_2412_09723_amd import scenes

INTR = scenes.Intrinsics(160, 120, 150.0, 150.0, 80.0, 60.0)
IDENT = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], np.float32)


def test_thresholds():
    # fx = fy = 128, z = 2: every border below is exact in binary32
    intr = scenes.Intrinsics(160, 120, 128.0, 128.0, 80.0, 60.0)
    after = lambda x: float(np.nextafter(np.float32(x), np.float32(np.inf)))
    cols = [
        (0.0, 0.0, 2.0),                 # centre of the image, 2 m: in
        (0.0, 0.0, 3.0),                 # exactly max_dist on the axis: in (inclusive)
        (0.0, 0.0, after(3.0)),          # just beyond: out
        (0.0, 0.0, 0.2),                 # on the near plane: out (strict)
        (0.0, 0.0, -1.0),                # behind: out
        (-1.25, 0.0, 2.0),               # u = 128 (-0.625) + 80 = 0 exactly: in
        (1.234375, 0.0, 2.0),            # u = 159 = W - 1 exactly: in
        (after(1.234375), 0.0, 2.0),     # just right of it: out
        (0.0, 0.921875, 2.0),            # v = 119 = H - 1 exactly: in
        (float("nan"), 0.0, 2.0),        # non-finite: out
    ]
    mu = np.asarray(cols, np.float32).T
    got = SEL.select_mask(mu, IDENT, intr, near_z=0.2, max_dist=3.0).tolist()
    assert got == [True, True, False, False, False, True, True, False, True, False]
    # a margin of 2 px admits the point just right of the border and one 2 px out (u = 161), not 161.5
    mu2 = np.asarray([[after(1.234375), 0.0, 2.0], [1.265625, 0.0, 2.0], [1.2734375, 0.0, 2.0]], np.float32).T
    assert SEL.select_mask(mu2, IDENT, intr, max_dist=3.0, margin=2.0).tolist() == [True, True, False]


def test_matches_camera_centre_and_projection_matrix():
    rng = np.random.default_rng(5)
    checked = excluded = selected = 0
    for trial in range(8):
        R0 = Rotation.from_euler("xyz", rng.uniform(-40, 40, 3), degrees=True).as_matrix()
        t0 = rng.uniform(-1, 1, 3)
        vm = np.concatenate([R0, t0[:, None]], axis=1).reshape(12).astype(np.float32)
        n = 20000
        mu = rng.uniform(-4, 4, (3, n)).astype(np.float32)
        dmax, margin = float(rng.uniform(1.5, 4.0)), float(rng.choice([0.0, 3.0]))
        got = SEL.select_mask(mu, vm, INTR, near_z=0.2, max_dist=dmax, margin=margin)
        V = vm.astype(np.float64).reshape(3, 4)
        R, t = V[:, :3], V[:, 3]
        c = -R.T @ t                                            # camera centre in world coordinates
        dist = np.linalg.norm(mu.astype(np.float64) - c[:, None], axis=0)
        K = np.array([[np.float32(INTR.fx), 0, np.float32(INTR.cx)], [0, np.float32(INTR.fy), np.float32(INTR.cy)],
                      [0, 0, 1]], np.float64)
        h = K @ (R @ mu.astype(np.float64) + t[:, None])        # homogeneous pixel coordinates
        z = (R @ mu.astype(np.float64) + t[:, None])[2]
        with np.errstate(all="ignore"):
            u, v = h[0] / h[2], h[1] / h[2]
        W, H = INTR.width, INTR.height
        dm = np.float64(np.float32(dmax))
        m = np.float64(np.float32(margin))
        want = (z > 0.2) & (dist <= dm) & (u >= -m) & (u <= W - 1 + m) & (v >= -m) & (v <= H - 1 + m)
        rel = 1e-9
        amb = (np.abs(dist - dm) <= rel * dm) | (np.abs(z - 0.2) <= rel)
        for val, lo_, hi_ in ((u, -m, W - 1 + m), (v, -m, H - 1 + m)):
            amb |= (np.abs(val - lo_) <= rel * (W + m)) | (np.abs(val - hi_) <= rel * (W + m))
        ok = ~amb
        assert np.array_equal(got[ok], want[ok])
        checked += int(ok.sum())
        excluded += int(amb.sum())
        selected += int(got.sum())
    assert selected > 1000 and excluded <= 10, (selected, excluded)


def test_indices_keep_map_order():
    rng = np.random.default_rng(2)
    mu = rng.uniform(-3, 3, (3, 5000)).astype(np.float32)
    idx = SEL.select(mu, IDENT, INTR, max_dist=3.5)
    mask = SEL.select_mask(mu, IDENT, INTR, max_dist=3.5)
    assert idx.dtype == np.int32 and np.all(np.diff(idx) > 0)
    assert [i for i in range(5000) if mask[i]] == idx.tolist()

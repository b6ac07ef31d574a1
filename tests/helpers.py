"""Small shared helpers for the tests (scene construction, comparisons)."""
import numpy as np

from paper_2412_09723_amd import scenes


def make_scene(means, scales, quats, opacity, colors, intr, viewmat=None):
    f = lambda a: np.ascontiguousarray(np.asarray(a, np.float32))
    vm = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], np.float32) if viewmat is None else f(viewmat)
    return scenes.Scene(f(means), f(scales), f(quats), f(opacity), f(colors), vm, intr)


def tiny_scene(seed, n=48, W=32, H=24, f=30.0, pose=None):
    intr = scenes.Intrinsics(W, H, f, f, W / 2.0, H / 2.0)
    return scenes.frustum_scene(n, intr, scenes.rng_for(9, seed), viewmat=pose)


def rel_err(got, ref, floor_frac=1e-3):
    """Elementwise |g - o| / max(|o|, floor_frac * max|o|)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    floor = floor_frac * max(float(np.abs(ref).max()), 1e-300)
    return np.abs(got - ref) / np.maximum(np.abs(ref), floor)

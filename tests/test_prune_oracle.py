"""Pins of the pruning oracle (oracle/prune.py) against App. C.1's three
criteria: hand-made cases on each side of every strict threshold, the
scale tests switched off without a scale threshold, and a per-Gaussian
loop over a random map that restates each criterion and the stable
compaction element by element."""
import numpy as np

from oracle import prune as PR

F32 = np.float32


def _map(op, sc):
    sc = np.asarray(sc, F32).T
    n = sc.shape[1]
    return {"means": np.arange(3 * n, dtype=F32).reshape(3, n), "scales": sc,
            "quats": np.ones((4, n), F32), "opacity": np.asarray(op, F32),
            "colors": np.full((3, n), 0.5, F32)}


def test_thresholds_are_strict():
    op = [0.005, np.nextafter(F32(0.005), F32(0)), 0.5, 0.5, 0.5, 0.5, 0.5, 0.5]
    sc = [[0.01, 0.01, 0.01],          # kept
          [0.01, 0.01, 0.01],          # opacity just below: removed
          [0.25, 0.2, 0.2],            # largest scale exactly tau_s: kept
          [np.nextafter(F32(0.25), F32(1)), 0.2, 0.2],   # just above: removed
          [0.15625, 0.0078125, 0.0078125],      # largest exactly 10 x the other two (exact in binary32): kept
          [0.15625, 0.0078125, 0.00390625],     # 10 x 0.01171875 < 0.15625: removed (elongated)
          [0.004, 0.1, 0.005],         # the largest in the middle: removed
          [0.05, 0.05, 0.0]]           # equal largest, other two sum 0.05: kept
    mask = PR.prune_mask(op, np.asarray(sc, F32).T)
    assert mask.tolist() == [False, True, False, True, False, True, True, False]


def test_no_scale_threshold_runs_opacity_only():
    op = [0.001, 0.5, 0.5]
    sc = [[0.01, 0.01, 0.01], [3.0, 0.01, 0.01], [0.3, 0.3, 0.3]]
    assert PR.prune_mask(op, np.asarray(sc, F32).T, tau_s=0.0).tolist() == [True, False, False]
    assert PR.prune_mask(op, np.asarray(sc, F32).T).tolist() == [True, True, True]


def test_against_a_per_gaussian_loop():
    rng = np.random.default_rng(17)
    n = 3000
    op = rng.uniform(0, 0.03, n).astype(F32)
    sc = (10 ** rng.uniform(-3, -0.3, (n, 3))).astype(F32)
    needle = rng.random(n) < 0.2
    sc[needle, 0] *= 30
    m = _map(op, sc)
    out, mask = PR.prune(m, 0.005, 0.25, 10.0)
    want_keep = []
    for i in range(n):
        s = [F32(v) for v in sc[i]]
        j = 0
        for k in (1, 2):
            if s[k] > s[j]:
                j = k
        others = [s[k] for k in range(3) if k != j]
        other = F32(others[0] + others[1])
        removed = bool(op[i] < F32(0.005)) or bool(s[j] > F32(0.25)) or bool(s[j] > F32(F32(10.0) * other))
        assert removed == bool(mask[i]), i
        if not removed:
            want_keep.append(i)
    assert 0.2 * n < len(want_keep) < 0.9 * n
    for k, v in m.items():
        assert np.array_equal(out[k], v[..., want_keep]), k

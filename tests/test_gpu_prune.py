"""Map pruning on the device (ms_prune) against the oracle, bit for bit:
the surviving Gaussians, their order and the count, on a room map with
faint, large and needle-like Gaussians mixed in, on ragged and degenerate
sizes, with everything or nothing removed, and in opacity-only mode."""
import numpy as np
import pytest
import torch

from oracle import prune as PR
from paper_2412_09723_amd import scenes, track

pytestmark = pytest.mark.gpu
KEYS = ("means", "scales", "quats", "opacity", "colors")


def _log(msg):
    print(msg, flush=True)


def _map(n, seed):
    """A room map with about a fifth of its Gaussians faint, large or needle-like."""
    if n == 0:
        return {k: np.zeros((r, 0) if r > 1 else (0,), np.float32)
                for k, r in zip(KEYS, (3, 3, 4, 1, 3))}
    sc = scenes.room_view(n=n)
    m = {k: np.ascontiguousarray(getattr(sc, k)).astype(np.float32) for k in KEYS}
    rng = scenes.rng_for(31, seed)
    pick = rng.random(n)
    m["opacity"][pick < 0.07] = rng.uniform(0.0, 0.01, int((pick < 0.07).sum())).astype(np.float32)
    big = (pick >= 0.07) & (pick < 0.12)
    m["scales"][:, big] *= np.float32(20.0)
    needle = (pick >= 0.12) & (pick < 0.2)
    m["scales"][rng.integers(0, 3, n) [needle], np.flatnonzero(needle)] *= np.float32(25.0)
    return m


def _run(m, *taus):
    d = {k: torch.from_numpy(v).cuda() for k, v in m.items()}
    out = track.prune_map(d, *taus)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _check(m, taus=()):
    got = _run(m, *taus)
    want, mask = PR.prune(m, *taus)
    for k in KEYS:
        assert got[k].shape == want[k].shape, (k, got[k].shape, want[k].shape)
        assert np.array_equal(got[k], want[k]), k
    return int((~mask).sum()), mask.size


@pytest.mark.parametrize("n", [1_000_000, 4097, 1025, 1023, 1])
def test_prune_matches_oracle(n):
    _log(f"prune n={n}")
    kept, total = _check(_map(n, n))
    if n >= 1000:
        assert 0.6 * total < kept < 0.95 * total


def test_prune_empty_all_and_none():
    _check(_map(0, 0))
    m = _map(5000, 3)
    m0 = dict(m, opacity=np.zeros_like(m["opacity"]))
    assert _check(m0)[0] == 0                                   # everything removed
    m1 = dict(m, opacity=np.full_like(m["opacity"], 0.5), scales=np.full_like(m["scales"], 0.01))
    assert _check(m1)[0] == 5000                                # nothing removed


def test_prune_opacity_only():
    m = _map(20000, 5)
    kept, total = _check(m, (0.005, 0.0, 10.0))
    assert kept == int((m["opacity"] >= np.float32(0.005)).sum())

"""Pins of the Eq. 7 pair-loss oracle (oracle/pairloss.py): central finite
differences of the whole loss in binary64 with respect to entries of all
four rendered images (away from the kink of |.|), the exchange symmetry of
the pair, the optimum at identical views, and each term alone against its
closed form."""
import numpy as np
import pytest

from oracle import pairloss as PL
from oracle import ssim as S


def _views(H, W, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, (3, H, W))
    y = np.clip(x + rng.normal(0, 0.1, x.shape), 0, 1)
    di = rng.uniform(1, 5, (H, W))
    dj = di + rng.normal(0, 0.05, di.shape)
    return x, y, di, dj


@pytest.mark.parametrize("H,W", [(23, 37), (12, 12)])
def test_gradient_against_central_differences(H, W):
    x, y, di, dj = _views(H, W, 1)
    L, grads = PL.pair_loss_grad(x, y, di, dj)
    rng = np.random.default_rng(2)
    h = 1e-6
    for which, arr in enumerate((x, y, di, dj)):
        for _ in range(12):
            idx = tuple(int(rng.integers(s)) for s in arr.shape)
            other = (y, x, dj, di)[which]
            if abs(arr[idx] - other[idx]) < 1e-3:
                continue                       # the kink of |.| is not differentiable
            base = arr[idx]
            arr[idx] = base + h
            lp, _ = PL.pair_loss_grad(x, y, di, dj)
            arr[idx] = base - h
            lm, _ = PL.pair_loss_grad(x, y, di, dj)
            arr[idx] = base
            fd = (lp - lm) / (2 * h)
            g = grads[which][idx]
            assert abs(fd - g) <= 1e-6 * max(abs(g), 1e-3 / arr.size), (which, idx, fd, g)


def test_exchange_symmetry_and_optimum():
    x, y, di, dj = _views(16, 20, 3)
    L1, (a, b, c, d) = PL.pair_loss_grad(x, y, di, dj)
    L2, (a2, b2, c2, d2) = PL.pair_loss_grad(y, x, dj, di)
    assert abs(L1 - L2) <= 1e-14
    for u, v in ((a, b2), (b, a2), (c, d2), (d, c2)):
        assert np.abs(u - v).max() <= 1e-15
    L0, g0 = PL.pair_loss_grad(x, x.copy(), di, di.copy())
    assert abs(L0) <= 1e-15 and all(np.abs(g).max() <= 1e-15 for g in g0)


def test_terms_alone():
    x, y, di, dj = _views(10, 14, 4)
    L, g = PL.pair_loss_grad(x, y, di, dj, 1.0, 0.0, 0.0)
    assert abs(L - np.mean(np.abs(x - y))) <= 1e-15
    assert np.array_equal(g[0], np.sign(x - y) / x.size) and not g[2].any()
    L, g = PL.pair_loss_grad(x, y, di, dj, 0.0, 0.0, 1.0)
    assert abs(L - np.mean(np.abs(di - dj))) <= 1e-15
    L, g = PL.pair_loss_grad(x, y, di, dj, 0.0, 1.0, 0.0)
    ls, gx = S.ssim_loss_grad(x, y, 1.0)
    assert abs(L - ls) <= 1e-15 and np.abs(g[0] - gx).max() == 0.0

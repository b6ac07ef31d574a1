"""GPU parity of Eq. 7 for one pair of rendered views (ms_pair_loss_grad)
against the oracle: the loss within 1e-5 relative, the four gradients at
the gradient tolerance (1e-3 elementwise with a floor of 1e-2 of the
maximum, 1e-3 normwise), on ragged frames, strips thinner than the window,
a single pixel and the full 1200x680 frame; accumulation; the optimum."""
import numpy as np
import pytest
import torch

from oracle import pairloss as PL
from paper_2412_09723_amd.track import pair_loss_grad

pytestmark = pytest.mark.gpu


def _views(H, W, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, (3, H, W)).astype(np.float32)
    y = np.clip(x + rng.normal(0, 0.1, x.shape), 0, 1).astype(np.float32)
    y[:, 1::5, 1::7] = x[:, 1::5, 1::7]              # exact ties: sign(0) = 0 on both sides
    di = rng.uniform(1, 5, (H, W)).astype(np.float32)
    dj = (di + rng.normal(0, 0.05, di.shape)).astype(np.float32)
    dj[1::3, 1::4] = di[1::3, 1::4]
    return x, y, di, dj


def _check_grad(got, want):
    """Gradient tolerance, with the floor no lower than 1e-2 of the size one
    entry's gradient naturally has (weight / entries)."""
    got = got.astype(np.float64)
    scale = max(float(np.abs(want).max()), 0.1 / want.size)
    err = np.abs(got - want) / np.maximum(np.abs(want), 1e-2 * scale)
    assert err.max() <= 1e-3, float(err.max())
    assert np.linalg.norm(got - want) <= 1e-3 * max(np.linalg.norm(want), 1e-30)


def _run(views, grads=None, accumulate=False, loss=None, w=(0.8, 0.2, 0.1)):
    dev = [torch.from_numpy(v).cuda() for v in views]
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    g = pair_loss_grad(*dev, *w, grads=grads, accumulate=accumulate, loss=loss)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in g], float(loss.cpu()[0])


@pytest.mark.parametrize("H,W", [(23, 37), (150, 200), (1, 1), (7, 300), (64, 96), (680, 1200)])
def test_pair_loss_matches_oracle(H, W):
    print(f"pair loss {H}x{W}", flush=True)
    views = _views(H, W, H + W)
    got, lv = _run(views)
    want_loss, want = PL.pair_loss_grad(*views)
    assert abs(lv - want_loss) <= 1e-5 * abs(want_loss), (lv, want_loss)
    for g, w_ in zip(got, want):
        _check_grad(g, w_)


def test_pair_loss_accumulates_and_optimum():
    views = _views(40, 52, 9)
    rng = np.random.default_rng(1)
    base = [(rng.standard_normal(v.shape) * 1e-5).astype(np.float32) for v in views]
    grads = tuple(torch.from_numpy(b.copy()).cuda() for b in base)
    loss = torch.full((1,), 0.25, dtype=torch.float32, device="cuda")
    got, lv = _run(views, grads=grads, accumulate=True, loss=loss)
    want_loss, want = PL.pair_loss_grad(*views)
    assert abs(lv - (0.25 + want_loss)) <= 1e-5
    for g, b, w_ in zip(got, base, want):
        _check_grad(g - b, w_)
    x, _, di, _ = views
    got, lv = _run((x, x.copy(), di, di.copy()))
    assert abs(lv) <= 1e-6
    assert max(np.abs(g).max() for g in got) <= 1e-2 * 0.2 / x.size

"""Persistent compositing over a tile queue (MS_FLAG_TILE_QUEUE, and eight
per-XCD queues with MS_FLAG_XCD_QUEUES): the same images bit for bit as the
one-workgroup-per-tile grid (each pixel's arithmetic does not depend on
which workgroup runs its tile, or when), gradients equal up to the order of
floating-point atomics, and every job within the oracle bar. The queue
itself must be a permutation of the tiles sorted by the expected work of
their bins, longest first, with each bin's tiles together in row-major
order, and the per-sub-block list depths the forward leaves for the
backward's queue must equal the maximum of the pixels' last-composited
positions."""
import numpy as np
import pytest
import torch

import oracle
from paper_2412_09723_amd import raster, scenes
from tests.gpu_util import check_grads, check_images, check_reordered_grads, to_dev
from tests.test_gpu_batch import KEYS, _dev, _mixed_scenes, _upstream

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def cost_class(c: int) -> int:
    """0 for no work, else 1 + 4 floor(log2 c) plus the two bits below the
    leading one (quarter-octave classes)."""
    if c == 0:
        return 0
    lg = c.bit_length() - 1
    f = (c >> (lg - 2)) & 3 if lg >= 2 else (c << (2 - lg)) & 3
    return 1 + 4 * lg + f


def _check_sorted_permutation(order, bins, bin_costs):
    """`order` holds every tile once; tiles of one bin are consecutive and in
    ascending (row-major) order; bins appear by non-increasing cost class."""
    order = np.asarray(order, np.int64)
    assert np.array_equal(np.sort(order), np.arange(len(bins))), "queue is not a permutation of the tiles"
    b = bins[order]
    starts = np.flatnonzero(np.r_[True, b[1:] != b[:-1]])
    assert len(starts) == len(np.unique(b)), "a bin's tiles are not consecutive in the queue"
    for s, e in zip(starts, np.r_[starts[1:], len(b)]):
        assert (np.diff(order[s:e]) > 0).all()
    cls = np.array([cost_class(int(bin_costs[x])) for x in b[starts]])
    assert (np.diff(cls) <= 0).all(), "queue not sorted longest first"


def _tile_bins(W, H, tile, bin_tile):
    tx, ty = (W + tile - 1) // tile, (H + tile - 1) // tile
    bx = (W + bin_tile - 1) // bin_tile
    s = bin_tile // tile
    t = np.arange(tx * ty)
    return (t % tx) // s + ((t // tx) // s) * bx


def _sub_block_depths(last, tile):
    """Per compositing tile and 8x8 sub-block (row-major in the tile): the
    maximum of the last-composited positions, 0 where the sub-block lies
    outside the image."""
    H, W = last.shape
    sb = tile // 8
    tx, ty = (W + tile - 1) // tile, (H + tile - 1) // tile
    pad = np.zeros((ty * tile, tx * tile), np.int64)
    pad[:H, :W] = last
    blocks = pad.reshape(ty, sb, 8, tx, sb, 8).max(axis=(2, 5))     # [ty, sb, tx, sb]
    return blocks.transpose(0, 2, 1, 3).reshape(tx * ty, sb * sb)


@pytest.mark.parametrize("schedule,tile,bin_tile", [("queue", 16, 0), ("xcd_queue", 16, 64), ("queue", 8, 32),
                                                    ("xcd_queue", 32, 128)])
def test_queue_order_and_sub_block_depths(schedule, tile, bin_tile):
    _log(f"tile queue order: {schedule} tile={tile} bin={bin_tile}")
    sc = _mixed_scenes()[2]            # 6000 Gaussians at 200x150
    m, vm = to_dev(sc)
    opts = raster.RenderOptions(tile=tile, bin_tile=bin_tile, check=True, schedule=schedule)
    job = raster.Job(m, vm, sc.intr, opts)
    job.forward()
    torch.cuda.synchronize()
    st = job.state()
    last = st["last"].cpu().numpy().astype(np.int64)
    depths = _sub_block_depths(last, tile)
    assert np.array_equal(st["tile_cost"].cpu().numpy().astype(np.int64), depths)
    tr = st["tile_range"].cpu().numpy().astype(np.int64)
    bins = _tile_bins(sc.intr.width, sc.intr.height, tile, bin_tile or tile)
    _check_sorted_permutation(st["tile_order"].cpu().numpy(), bins, tr[:, 1] - tr[:, 0])
    up = _dev(_upstream(sc, 1))
    job.backward(*up)
    torch.cuda.synchronize()
    bwd_costs = np.bincount(bins, weights=depths.sum(axis=1), minlength=len(tr)).astype(np.int64)
    _check_sorted_permutation(job.state()["tile_order"].cpu().numpy(), bins, bwd_costs)


@pytest.mark.parametrize("schedule,tile,bin_tile,bwd", [("queue", 16, 0, "mfma"), ("xcd_queue", 16, 128, "mfma"),
                                                        ("queue", 8, 32, "mfma_bf16x3"), ("xcd_queue", 32, 128, "mfma"),
                                                        ("queue", 16, 64, "lds")])
def test_queue_batch_equals_grid_and_oracle(schedule, tile, bin_tile, bwd):
    """A batch of a 160x120 frustum, a ragged 37x23 view, a 200x150 view and
    an empty map: queued against the grid (images bit-exact, gradients up to
    atomic order) and each job against the oracle. The LDS backward ignores
    the queue flag and runs as a grid."""
    _log(f"queued batch {schedule} tile={tile} bin={bin_tile} bwd={bwd}")
    scs = _mixed_scenes()
    devs = [to_dev(sc) for sc in scs]
    ups = [_dev(_upstream(sc, j)) for j, sc in enumerate(scs)]
    res = {}
    for sched in ("grid", schedule):
        opts = raster.RenderOptions(tile=tile, bin_tile=bin_tile, bwd_records=bwd, check=True, schedule=sched)
        batch = raster.BatchJob([m for m, _ in devs], [vm for _, vm in devs], [sc.intr for sc in scs], opts)
        outs = [tuple(t.clone() for t in o) for o in batch.forward()]
        gbs = batch.backward(ups)
        torch.cuda.synchronize()
        res[sched] = (outs, {j: {k: v.clone() for k, v in g.items()} for j, g in enumerate(gbs)})
        del batch
    for j, sc in enumerate(scs):
        for x, y in zip(res["grid"][0][j], res[schedule][0][j]):
            assert torch.equal(x, y), j
        check_reordered_grads(res[schedule][1][j], res["grid"][1][j], (KEYS if sc.n else ()) + ("viewmat", "twist"))
        if sc.n:
            check_images(res[schedule][0][j], oracle.forward(sc))
            check_grads(res[schedule][1][j], oracle.backward(sc, *_upstream(sc, j)))


@pytest.mark.parametrize("schedule", ["queue", "xcd_queue"])
def test_queue_fewer_tiles_than_queues_and_repeat(schedule):
    """A 37x23 view at tile 16 (six tiles, fewer than the eight XCD queues)
    and a 1x1 image: every tile is composited exactly once, and a second
    forward (the claim counters start again from zero) repeats the first bit
    for bit."""
    sc = _mixed_scenes()[1]
    for intr in (sc.intr, scenes.Intrinsics(1, 1, 30.0, 31.0, 0.3, 0.4)):
        _log(f"small image {intr.width}x{intr.height} {schedule}")
        s2 = scenes.Scene(sc.means, sc.scales, sc.quats, sc.opacity, sc.colors, sc.viewmat, intr)
        m, vm = to_dev(s2)
        q = raster.Job(m, vm, intr, raster.RenderOptions(check=True, schedule=schedule))
        g = raster.Job(m, vm, intr, raster.RenderOptions(check=True))
        a = [t.clone() for t in q.forward()]
        b = [t.clone() for t in q.forward()]
        c = g.forward()
        torch.cuda.synchronize()
        for x, y, z in zip(a, b, c):
            assert torch.equal(x, y) and torch.equal(x, z)
        up = _dev(scenes.upstream_grads(intr, scenes.rng_for(7, 5, salt=2), 1.0, 0.5))
        check_reordered_grads(q.backward(*up), g.backward(*up), KEYS + ("viewmat", "twist"))
        check_images(a, oracle.forward(s2))


def test_queue_room_1m_full_size():
    """1200x680, 1M Gaussians (the benchmark frame): the queued forward and
    backward against the grid and the oracle."""
    _log("room_view full size, tile queue")
    sc = scenes.room_view()
    m, vm = to_dev(sc)
    up_np = scenes.upstream_grads(sc.intr, scenes.rng_for(0, 0, salt=2), 0.5, 0.5)
    up = _dev(up_np)
    q = raster.Job(m, vm, sc.intr, raster.RenderOptions(check=True, schedule="queue"))
    imgs = [t.clone() for t in q.forward()]
    gq = {k: v.clone() for k, v in q.backward(*up).items()}
    torch.cuda.synchronize()
    del q
    g = raster.Job(m, vm, sc.intr, raster.RenderOptions(check=True))
    for x, y in zip(imgs, g.forward()):
        assert torch.equal(x, y)
    check_reordered_grads(gq, g.backward(*up), KEYS + ("viewmat", "twist"))
    torch.cuda.synchronize()
    del g
    check_images(imgs, oracle.forward(sc))
    check_grads(gq, oracle.backward(sc, *up_np))

"""Batched rendering (several agents' maps through one launch sequence):
every job's images equal rendering it alone bit for bit (identical lists and
per-pixel arithmetic), its gradients equal the lone backward up to the order
of floating-point atomics, and every job meets the oracle bar."""
import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import oracle
from paper_2412_09723_amd import raster, scenes
from tests.gpu_util import check_grads, check_images, check_reordered_grads, to_dev
from tests.helpers import make_scene

pytestmark = pytest.mark.gpu
KEYS = ("means", "scales", "quats", "opacity", "colors")


def _log(msg):
    print(msg, flush=True)


def _mixed_scenes():
    out = [scenes.small_frustum()]
    intr = scenes.Intrinsics(37, 23, 30.0, 31.0, 18.3, 11.1)
    R0 = Rotation.from_euler("xyz", [6, -4, 9], degrees=True).as_matrix()
    vm = np.concatenate([R0, np.array([[0.04], [-0.03], [0.1]])], axis=1).reshape(12).astype(np.float32)
    out.append(scenes.frustum_scene(700, intr, scenes.rng_for(9, 77), viewmat=vm))
    intr2 = scenes.Intrinsics(200, 150, 180.0, 175.0, 99.5, 76.0)
    R1 = Rotation.from_euler("xyz", [-3, 8, -2], degrees=True).as_matrix()
    vm2 = np.concatenate([R1, np.array([[-0.1], [0.05], [0.2]])], axis=1).reshape(12).astype(np.float32)
    out.append(scenes.frustum_scene(6000, intr2, scenes.rng_for(9, 78), viewmat=vm2))
    empty_intr = scenes.Intrinsics(24, 16, 20.0, 20.0, 12.0, 8.0)
    out.append(make_scene(np.zeros((3, 0)), np.zeros((3, 0)), np.zeros((4, 0)), np.zeros(0), np.zeros((3, 0)),
                          empty_intr))
    return out


def _upstream(sc, salt):
    return scenes.upstream_grads(sc.intr, scenes.rng_for(7, salt, salt=2), 1.0, 0.5)


def _dev(arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


@pytest.mark.parametrize("tile,bin_tile,bwd", [(16, 0, "mfma"), (8, 32, "lds"), (32, 128, "mfma"),
                                               (16, 64, "scalar")])
def test_batch_equals_alone_and_oracle(tile, bin_tile, bwd):
    _log(f"batch of mixed jobs tile={tile} bin={bin_tile} bwd={bwd}")
    scs = _mixed_scenes()
    opts = raster.RenderOptions(tile=tile, bin_tile=bin_tile, bwd_records=bwd, check=True)
    devs = [to_dev(sc) for sc in scs]
    batch = raster.BatchJob([m for m, _ in devs], [vm for _, vm in devs], [sc.intr for sc in scs], opts)
    outs = batch.forward()
    ups = [_dev(_upstream(sc, j)) for j, sc in enumerate(scs)]
    gbs = batch.backward(ups)
    torch.cuda.synchronize()
    for j, sc in enumerate(scs):
        m, vm = devs[j]
        alone = raster.Job(m, vm, sc.intr, opts)
        ref_imgs = alone.forward()
        for x, y in zip(outs[j], ref_imgs):
            assert torch.equal(x, y), j
        ga = alone.backward(*ups[j])
        torch.cuda.synchronize()
        if sc.n:
            check_reordered_grads(gbs[j], ga, KEYS)
        check_reordered_grads(gbs[j], ga, ("viewmat", "twist"))
        if sc.n:
            check_images(outs[j], oracle.forward(sc))
            check_grads(gbs[j], oracle.backward(sc, *_upstream(sc, j)))
        else:
            assert not any(t.any() for t in outs[j])


def test_batch_empty_maps_first_and_between():
    """Empty maps ahead of and between non-empty ones: an empty job owns no
    Gaussian slots, so its slot range coincides with the next job's start;
    every projection and adjoint block must still find the non-empty job."""
    mixed = _mixed_scenes()
    empty, tiny, small, mid = mixed[3], mixed[1], mixed[0], mixed[2]
    scs = [empty, tiny, empty, small, mid, empty]
    _log(f"batch with empty maps at 0, 2, 5: n = {[sc.n for sc in scs]}")
    opts = raster.RenderOptions(check=True)
    devs = [to_dev(sc) for sc in scs]
    batch = raster.BatchJob([m for m, _ in devs], [vm for _, vm in devs], [sc.intr for sc in scs], opts)
    outs = batch.forward()
    ups = [_dev(_upstream(sc, j)) for j, sc in enumerate(scs)]
    gbs = batch.backward(ups)
    torch.cuda.synchronize()
    for j, sc in enumerate(scs):
        m, vm = devs[j]
        alone = raster.Job(m, vm, sc.intr, opts)
        for x, y in zip(outs[j], alone.forward()):
            assert torch.equal(x, y), j
        ga = alone.backward(*ups[j])
        torch.cuda.synchronize()
        check_reordered_grads(gbs[j], ga, (KEYS if sc.n else ()) + ("viewmat", "twist"))
        if not sc.n:
            assert not any(t.any() for t in outs[j])
            assert not gbs[j]["twist"].any() and not gbs[j]["viewmat"].any()
    check_grads(gbs[1], oracle.backward(tiny, *_upstream(tiny, 1)))


def test_batch_per_job_gradient_flags():
    """Tracking (pose-only) and mapping (all gradients) jobs in one batch."""
    scs = _mixed_scenes()[:3]
    devs = [to_dev(sc) for sc in scs]
    opts = raster.RenderOptions(check=True)
    batch = raster.BatchJob([m for m, _ in devs], [vm for _, vm in devs], [sc.intr for sc in scs], opts)
    batch.forward()
    ups = [_dev(_upstream(sc, j)) for j, sc in enumerate(scs)]
    gbs = batch.backward(ups, map_grads=[False, True, True], pose_grads=[True, False, True])
    torch.cuda.synchronize()
    assert set(gbs[0]) == {"viewmat", "twist"} and "twist" not in gbs[1] and set(gbs[2]) >= set(KEYS) | {"twist"}
    for j, (m, vm) in enumerate(devs):
        alone = raster.Job(m, vm, scs[j].intr, opts)
        alone.forward()
        ga = alone.backward(*ups[j])
        check_reordered_grads(gbs[j], ga, [k for k in gbs[j]])


def test_batch_config3_full_size():
    """Four agents' room maps of 200k, 600k, 1.2M and 2M Gaussians at
    1200x680 in one batch, against each rendered alone, and the smallest's
    images and gradients against the oracle."""
    _log("four_agent_rooms batch: 200k/600k/1.2M/2M at 1200x680")
    scs = scenes.four_agent_rooms()
    devs = [to_dev(sc) for sc in scs]
    opts = raster.RenderOptions(check=True)
    batch = raster.BatchJob([m for m, _ in devs], [vm for _, vm in devs], [sc.intr for sc in scs], opts)
    outs = batch.forward()
    ups_np = [scenes.upstream_grads(sc.intr, scenes.rng_for(3, j, salt=2), 0.5, 0.0) for j, sc in enumerate(scs)]
    ups = [_dev(u) for u in ups_np]
    gbs = batch.backward(ups)
    torch.cuda.synchronize()
    _log(f"  batch stats {batch.stats()}")
    for j, sc in enumerate(scs):
        m, vm = devs[j]
        alone = raster.Job(m, vm, sc.intr, opts)
        for x, y in zip(outs[j], alone.forward()):
            assert torch.equal(x, y), j
        ga = alone.backward(*ups[j])
        torch.cuda.synchronize()
        check_reordered_grads(gbs[j], ga, KEYS + ("viewmat", "twist"))
        del alone, ga
    # the 200k map's images and gradients from the batch against the oracle
    check_images(outs[0], oracle.forward(scs[0]))
    check_grads(gbs[0], oracle.backward(scs[0], *ups_np[0]))


def test_autotuner_picks_a_measured_candidate():
    from paper_2412_09723_amd import autotune
    scs = _mixed_scenes()[:3]
    devs = [to_dev(sc) for sc in scs]
    ups = [_dev(_upstream(sc, j)) for j, sc in enumerate(scs)]
    tuner = autotune.Autotuner(reps=1)
    res = tuner.tune_batch([m for m, _ in devs], [vm for _, vm in devs], [sc.intr for sc in scs], ups)
    assert len(res.table) == 9 + len(autotune.SCHEDULES) - 1
    assert abs(res.ms - min(res.table.values())) < 1e-3
    assert res.options.tile in autotune.TILES and res.options.wave_batch in autotune.WAVE_BATCHES
    assert res.options.schedule in autotune.SCHEDULES
    assert res.options.bin_tile >= res.options.tile
    again = tuner.tune_batch([m for m, _ in devs], [vm for _, vm in devs], [sc.intr for sc in scs], ups)
    assert again.options == res.options         # cached


def test_views_of_one_map_accumulate_into_one_gradient():
    """Eight keyframes of one 500k-Gaussian map at 640x480 in one batch, the
    map gradients summed into one set of arrays (MS_FLAG_ACCUMULATE_MAP_GRADS):
    against the sum of the views rendered alone and against the oracle's sum
    over the views; pose gradients per view against the lone ones."""
    _log("keyframe_ring batch with shared map gradients: 8 views 640x480, 500k Gaussians")
    sc, vms = scenes.keyframe_ring()
    dev = torch.device("cuda")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    m = {k: t(getattr(sc, k)) for k in KEYS}
    vmt = [t(vm) for vm in vms]
    opts = raster.RenderOptions(check=True)
    batch = raster.BatchJob([m] * len(vms), vmt, [sc.intr] * len(vms), opts)
    batch.forward()
    ups = [scenes.upstream_grads(sc.intr, scenes.rng_for(2, v, salt=2), 1.0, 0.5) for v in range(len(vms))]
    shared = {k: torch.full_like(m[k], 7.0) for k in KEYS}        # stale values: the call zeroes them
    gbs = batch.backward([_dev(u) for u in ups], shared_map_grads=shared)
    torch.cuda.synchronize()
    alone_sum = {k: torch.zeros_like(m[k]) for k in KEYS}
    for v, vm in enumerate(vmt):
        job = raster.Job(m, vm, sc.intr, opts)
        job.forward()
        ga = job.backward(*_dev(ups[v]))
        torch.cuda.synchronize()
        for k in KEYS:
            alone_sum[k] += ga[k]
        check_reordered_grads(gbs[v], ga, ("viewmat", "twist"))
        assert all(gbs[v][k] is shared[k] for k in KEYS)
        del job, ga
    check_reordered_grads(shared, alone_sum, KEYS)
    ref = {k: 0.0 for k in KEYS}
    gflags = np.zeros(sc.n, np.uint8)
    for vm, up in zip(vms, ups):
        rb = oracle.backward(scenes.Scene(sc.means, sc.scales, sc.quats, sc.opacity, sc.colors, vm, sc.intr), *up)
        for k in KEYS:
            ref[k] = ref[k] + rb[k]
        gflags |= rb["gflags"]
    ref["gflags"] = gflags
    _log(f"  shared map gradients vs oracle: {check_grads(shared, ref, pose=False)}")

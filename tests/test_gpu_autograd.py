"""Differentiation through the torch.autograd.Function: a mapping step over
8 keyframes (640x480, poses on a 1 m circle facing outward, 500k Gaussians).

The loss is sum_v <G_v, render_v> for seeded upstream images G_v, so the map
gradient is the sum of the per-view backward passes. Checked against
(1) the oracle's analytic gradient summed over views, elementwise and
normwise, map and pose; (2) frozen-decision central finite differences of
the oracle in binary64 (h = 1e-4) on 64 sampled parameters, which pins the
oracle's gradient at this configuration.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2412_09723_amd import raster, scenes
from tests.gpu_util import check_grads

pytestmark = pytest.mark.gpu

KINDS = (("means", 3), ("scales", 3), ("quats", 4), ("opacity", 1), ("colors", 3))


def _log(msg):
    print(msg, flush=True)


def _view(sc, vm):
    return scenes.Scene(sc.means, sc.scales, sc.quats, sc.opacity, sc.colors, vm, sc.intr)


def test_mapping_step_through_autograd_matches_oracle_and_fd():
    _log("keyframe_ring autograd: 8 views 640x480, 500k Gaussians")
    sc, vms = scenes.keyframe_ring()
    dev = torch.device("cuda")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    m = {k: t(getattr(sc, k)).requires_grad_(True) for k, _ in KINDS}
    vmt = [t(vm).requires_grad_(True) for vm in vms]
    ups = [scenes.upstream_grads(sc.intr, scenes.rng_for(2, v, salt=2), 1.0, 0.5) for v in range(len(vms))]
    outs, grads = [], []
    for v, vm in enumerate(vmt):
        rgb, depth, sil = raster.render(m, vm, sc.intr, raster.RenderOptions(check=True))
        outs += [rgb, depth, sil]
        grads += [t(u) for u in ups[v]]
    torch.autograd.backward(outs, grads)
    torch.cuda.synchronize()
    got = {k: m[k].grad for k, _ in KINDS}

    # oracle: analytic gradient summed over views
    ref = {k: 0.0 for k, _ in KINDS}
    gflags = np.zeros(sc.n, np.uint8)
    pose_ref = []
    for v, vm in enumerate(vms):
        rb = oracle.backward(_view(sc, vm), *ups[v])
        for k, _ in KINDS:
            ref[k] = ref[k] + rb[k]
        gflags |= rb["gflags"]
        pose_ref.append(rb["viewmat"])
    ref["gflags"] = gflags
    worst = check_grads(got, ref, pose=False)
    _log(f"  map gradients vs oracle: {worst}")
    for v in range(len(vms)):
        gv = vmt[v].grad.detach().cpu().numpy().astype(np.float64)
        e = np.abs(gv - pose_ref[v]).max() / max(np.abs(pose_ref[v]).max(), 1e-30)
        assert e <= 1e-3, (v, e)

    # frozen-decision central differences of the oracle on 64 parameters
    rng = np.random.default_rng(2024)
    vis = np.stack([oracle.project(_view(sc, vm))["visible"] for vm in vms])   # [views][n]
    recs = {}
    params = {k: getattr(sc, k).astype(np.float64).reshape(rows, -1).copy() for k, rows in KINDS}
    h = 1e-4
    checked = 0
    for _ in range(64):
        kind, rows = KINDS[int(rng.integers(len(KINDS)))]
        r = int(rng.integers(rows))
        col = np.asarray(ref[kind]).reshape(rows, -1)[r]
        pool = np.flatnonzero((col != 0.0) & (gflags == 0))
        i = int(rng.choice(pool))
        a = float(col[i])
        fd = 0.0
        for v in np.flatnonzero(vis[:, i]):
            if v not in recs:
                recs[v] = oracle.record(_view(sc, vms[v]))
            base = params[kind][r, i]
            params[kind][r, i] = base + h
            lp = oracle.frozen_loss(params, vms[v], sc.intr, recs[v], *ups[v])
            params[kind][r, i] = base - h
            lm = oracle.frozen_loss(params, vms[v], sc.intr, recs[v], *ups[v])
            params[kind][r, i] = base
            fd += (lp - lm) / (2 * h)
        g = float(got[kind].detach().cpu().numpy().reshape(rows, -1)[r, i])
        scale = max(float(np.abs(np.asarray(ref[kind])).max()), 1e-30)
        assert abs(fd - a) <= 1e-6 * scale + 1e-5 * abs(a), (kind, r, i, fd, a)
        assert abs(g - fd) <= 1e-3 * max(abs(fd), 1e-2 * scale), (kind, r, i, g, fd)
        checked += 1
    assert checked == 64, checked
    _log("  64 sampled parameters: oracle = frozen FD, GPU within 1e-3")


def test_autograd_requested_inputs_only():
    """Only the inputs that require grad get gradients; the pose-only and
    map-only paths agree with the full backward."""
    sc = scenes.small_frustum()
    dev = torch.device("cuda")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    up = [t(u) for u in scenes.upstream_grads(sc.intr, scenes.rng_for(0, 0, salt=2), 1.0, 0.5)]

    def run(map_grad, pose_grad):
        m = {k: t(getattr(sc, k)).requires_grad_(map_grad) for k, _ in KINDS}
        vm = t(sc.viewmat).requires_grad_(pose_grad)
        outs = raster.render(m, vm, sc.intr, raster.RenderOptions(check=True))
        torch.autograd.backward(list(outs), up)
        return m, vm

    m_all, vm_all = run(True, True)
    m_map, vm_map = run(True, False)
    m_pose, vm_pose = run(False, True)
    assert vm_map.grad is None and all(m_pose[k].grad is None for k, _ in KINDS)
    for k, _ in KINDS:
        assert torch.allclose(m_map[k].grad, m_all[k].grad, rtol=1e-4, atol=1e-9)
    assert torch.allclose(vm_pose.grad, vm_all.grad, rtol=1e-5, atol=1e-9)


def test_holder_keeps_a_workspace_per_pending_backward():
    """Two renders through one holder before their backward (the multi-view
    mapping pattern): each keeps its own workspace, so both gradients equal
    those of renders without a holder. A Job whose workspace another forward
    has reused refuses its backward, and autograd refuses a backward after
    an in-place update of the map."""
    sc = scenes.small_frustum()
    dev = torch.device("cuda")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    vms = [sc.viewmat, scenes.perturb_pose(sc.viewmat, scenes.rng_for(0, 0, salt=3))]
    ups = [[t(u) for u in scenes.upstream_grads(sc.intr, scenes.rng_for(0, v, salt=2), 1.0, 0.5)]
           for v in range(2)]

    def grads(holder):
        m = {k: t(getattr(sc, k)).requires_grad_(True) for k, _ in KINDS}
        outs = []
        for vm in vms:
            outs.append(raster.render(m, t(vm), sc.intr, raster.RenderOptions(check=True), holder))
        for o, u in zip(outs, ups):           # both forwards ran before either backward
            torch.autograd.backward(list(o), u)
        return {k: m[k].grad.clone() for k, _ in KINDS}

    holder = {}
    shared = grads(holder)
    assert len(holder["pool"]) == 2 and not any(e["busy"] for e in holder["pool"])
    alone = grads(None)
    for k, _ in KINDS:
        assert torch.allclose(shared[k], alone[k], rtol=1e-5, atol=1e-9), k
    again = grads(holder)                     # the pool is reused, not grown
    assert len(holder["pool"]) == 2
    for k, _ in KINDS:
        assert torch.allclose(again[k], alone[k], rtol=1e-5, atol=1e-9), k

    # two Jobs on one workspace: the first one's state is gone
    m = {k: t(getattr(sc, k)) for k, _ in KINDS}
    a = raster.Job(m, t(vms[0]), sc.intr, raster.RenderOptions())
    b = raster.Job(m, t(vms[1]), sc.intr, raster.RenderOptions(), workspace=a.ws)
    a.forward()
    b.forward()
    with pytest.raises(RuntimeError, match="another forward"):
        a.backward(*ups[0])
    b.backward(*ups[1])

    # in-place update of a map tensor between forward and backward
    m = {k: t(getattr(sc, k)).requires_grad_(True) for k, _ in KINDS}
    leaf = {k: v for k, v in m.items()}
    mc = {k: v * 1.0 for k, v in leaf.items()}
    outs = raster.render(mc, t(vms[0]), sc.intr)
    with torch.no_grad():
        mc["opacity"].mul_(0.5)
    with pytest.raises(RuntimeError):
        torch.autograd.backward(list(outs), ups[0])

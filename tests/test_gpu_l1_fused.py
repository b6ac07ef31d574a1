"""The tracking loss's gradient formed inside the compositing backward
(ms_backward_l1) against (1) ms_l1_loss_grad followed by ms_backward, on
every backward variant, and (2) the oracle's backward of the L1 loss between
its own render and the target. The targets sit at least 0.05 away from the
oracle's render on every plane, so every sign is the same on both sides."""
import numpy as np
import pytest
import torch

import oracle
from paper_2412_09723_amd import raster, scenes
from tests.gpu_util import check_grads, to_dev

pytestmark = pytest.mark.gpu
KEYS = ("means", "scales", "quats", "opacity", "colors", "viewmat", "twist")


def _target(ref, rng):
    off = lambda shp: (rng.uniform(0.05, 0.5, shp) * rng.choice([-1.0, 1.0], shp))
    return (ref["rgb"] + off(ref["rgb"].shape), ref["depth"] + off(ref["depth"].shape),
            ref["sil"] + off(ref["sil"].shape))


@pytest.mark.parametrize("name,bwd", [("small", "mfma"), ("small", "mfma_bf16x3"), ("small", "lds"),
                                      ("small", "scalar"), ("room", "mfma")])
def test_fused_equals_planes_and_oracle(name, bwd):
    print(f"fused L1 {name} {bwd}", flush=True)
    sc = scenes.small_frustum() if name == "small" else scenes.room_view()
    w = (1.0, 0.5, 0.25)
    ref = oracle.forward(sc)
    tgt_np = [a.astype(np.float32) for a in _target(ref, np.random.default_rng(3))]
    tgt = [torch.from_numpy(a).cuda() for a in tgt_np]
    m, vm = to_dev(sc)
    opts = raster.RenderOptions(check=True, bwd_records=bwd, fwd_records="scalar" if bwd == "scalar" else "lds")
    job = raster.Job(m, vm, sc.intr, opts)
    pred = job.forward()
    fused = {k: v.clone() for k, v in job.backward_l1(pred, tgt, *w).items()}
    # the same upstream through gradient planes
    from paper_2412_09723_amd import _lib
    from paper_2412_09723_amd._lib import MsImages, MsIntrinsics, check, ref as cref
    import ctypes
    H, W = sc.intr.height, sc.intr.width
    gr = (torch.empty(3, H, W, device="cuda"), torch.empty(H, W, device="cuda"), torch.empty(H, W, device="cuda"))
    im = lambda t3: MsImages(*[t.data_ptr() for t in t3])
    lib = _lib.load()
    check(lib.ms_l1_loss_grad(cref(im(pred)), cref(im(tgt)), cref(job.c_intr), *w, cref(im(gr)), None,
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    planes = job.backward(*gr)
    torch.cuda.synchronize()
    for k in KEYS:
        a, b = fused[k].cpu().numpy(), planes[k].cpu().numpy()
        assert np.abs(a - b).max() <= 1e-5 * max(np.abs(b).max(), 1e-30), k
    # the oracle's backward of the L1 loss of its own render against the target
    P = H * W
    up = (w[0] / (3 * P) * np.sign(ref["rgb"] - tgt_np[0]), w[1] / P * np.sign(ref["depth"] - tgt_np[1]),
          w[2] / P * np.sign(ref["sil"] - tgt_np[2]))
    up = [u.astype(np.float32) for u in up]
    worst = check_grads(fused, oracle.backward(sc, *up))
    print(f"  grad worst {worst}", flush=True)

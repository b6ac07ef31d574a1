"""The allocation-free pruning entry point (ms_prune_noalloc, scratch in a
static device array) against ms_prune (scratch in a caller's workspace),
through the C ABI: every output array and the survivor count bit for bit,
on two calls in a row, the second on a smaller map (the static array keeps
the first call's counts, which must not leak into the second)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2412_09723_amd import _lib, scenes
from paper_2412_09723_amd._lib import MsMap, check, ref

pytestmark = pytest.mark.gpu

KEYS = ("means", "scales", "quats", "opacity", "colors")
ROWS = {"means": 3, "scales": 3, "quats": 4, "opacity": 1, "colors": 3}


def _map(n, seed):
    rng = scenes.rng_for(17, seed)
    sc = scenes.room_view(n=n)
    m = {k: torch.from_numpy(np.ascontiguousarray(getattr(sc, k))).cuda() for k in KEYS}
    # faint, oversized and needle-like Gaussians mixed in, so that about a fifth go
    k = n // 5
    idx = torch.from_numpy(rng.choice(n, size=k, replace=False)).cuda()
    m["opacity"][idx[: k // 3]] = 0.001
    m["scales"][0, idx[k // 3: 2 * k // 3]] = 0.6
    m["scales"][1, idx[2 * k // 3:]] = 0.5
    m["scales"][0, idx[2 * k // 3:]] = 0.01
    m["scales"][2, idx[2 * k // 3:]] = 0.01
    return m


def _run(lib, m, noalloc):
    n = m["means"].shape[1]
    dev = m["means"].device
    out = {k: torch.full((ROWS[k] * max(n, 1),), float("nan"), dtype=torch.float32, device=dev) for k in KEYS}
    kept = torch.full((1,), -1, dtype=torch.int64, device=dev)
    src = MsMap(n, *[m[k].data_ptr() for k in KEYS])
    dst = MsMap(n, *[out[k].data_ptr() for k in KEYS])
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    if noalloc:
        check(lib.ms_prune_noalloc(ref(src), 0.005, 0.25, 10.0, ref(dst), ctypes.c_void_p(kept.data_ptr()), st))
    else:
        ws = torch.empty(int(lib.ms_prune_workspace_bytes(n)) + 256, dtype=torch.uint8, device=dev)
        check(lib.ms_prune(ref(src), 0.005, 0.25, 10.0, ref(dst), ctypes.c_void_p(kept.data_ptr()),
                           ctypes.c_void_p(ws.data_ptr()), ws.numel(), st))
    torch.cuda.synchronize()
    k = int(kept.item())
    return k, {key: out[key][:ROWS[key] * k].cpu().numpy() for key in KEYS}


def test_prune_noalloc_equals_prune_on_two_calls():
    lib = _lib.load()
    for n, seed in ((1_000_000, 1), (300_001, 2)):   # the second smaller than the first
        print(f"prune noalloc n={n}", flush=True)
        m = _map(n, seed)
        k_ref, ref_out = _run(lib, m, noalloc=False)
        k_got, got = _run(lib, m, noalloc=True)
        assert k_got == k_ref and 0 < k_ref < n
        for key in KEYS:
            assert np.array_equal(got[key].view(np.uint32), ref_out[key].view(np.uint32)), key

"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments on the host before any launch."""
import ctypes
import os
import re

import pytest

from paper_2412_09723_amd import _lib
from paper_2412_09723_amd._lib import MsImages, MsIntrinsics, MsMap, MsOptions, ref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "macsplat.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        import paper_2412_09723_amd.build as b
        b.build()
    return _lib.load()


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ms_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert len(syms) >= 8
    for s in syms:
        assert hasattr(lib, s), s
    assert set(_lib.EXPORTED) <= set(syms)


def test_version_and_status_strings(lib):
    assert lib.ms_abi_version() == 5
    for code in range(6):
        assert lib.ms_status_string(code)
    assert lib.ms_status_string(99) == b"unknown status"


INTR = MsIntrinsics(160, 120, 150.0, 150.0, 80.0, 60.0)
OPTS = MsOptions(16, 64, 0.2, 0)


def test_workspace_bytes(lib):
    a = lib.ms_workspace_bytes(4096, ref(INTR), ref(OPTS), 1 << 20)
    b = lib.ms_workspace_bytes(8192, ref(INTR), ref(OPTS), 1 << 20)
    c = lib.ms_workspace_bytes(0, ref(INTR), ref(OPTS), 0)
    assert a > 0 and b > a and c > 0
    assert lib.ms_workspace_bytes(4096, ref(INTR), ref(MsOptions(12, 64, 0.2, 0)), 1 << 20) == 0
    assert lib.ms_workspace_bytes(4096, ref(INTR), ref(MsOptions(16, 48, 0.2, 0)), 1 << 20) == 0
    assert lib.ms_workspace_bytes(4096, ref(INTR), ref(MsOptions(16, 64, 0.0, 0)), 1 << 20) == 0
    assert lib.ms_workspace_bytes(4096, ref(INTR), ref(MsOptions(16, 64, 0.2, 0, 8)), 1 << 20) == 0
    assert lib.ms_workspace_bytes(4096, ref(INTR), ref(MsOptions(16, 64, 0.2, 0, 48)), 1 << 20) == 0
    assert lib.ms_workspace_bytes(4096, ref(INTR), ref(MsOptions(16, 64, 0.2, 0, 512)), 1 << 20) == 0
    assert lib.ms_workspace_bytes(4096, ref(INTR), ref(MsOptions(16, 64, 0.2, 0, 128)), 1 << 20) > 0
    assert lib.ms_workspace_bytes(-1, ref(INTR), ref(OPTS), 1 << 20) == 0
    assert lib.ms_workspace_bytes(4096, ref(MsIntrinsics(0, 120, 150, 150, 80, 60)), ref(OPTS), 1 << 20) == 0
    assert lib.ms_workspace_bytes(4096, ref(MsIntrinsics(160, 120, -1, 150, 80, 60)), ref(OPTS), 1 << 20) == 0
    assert lib.ms_workspace_bytes(4096, None, ref(OPTS), 1 << 20) == 0


FAKE = 0x100000   # never dereferenced: every case below fails validation first


def _fwd(lib, m, vm=FAKE, intr=INTR, opts=OPTS, ws=FAKE, ws_bytes=1 << 40, cap=1 << 20, out=True):
    imgs = MsImages(FAKE, FAKE, FAKE) if out else MsImages(0, 0, 0)
    return lib.ms_forward(ref(m) if m is not None else None, ctypes.c_void_p(vm), ref(intr), ref(opts),
                          ctypes.c_void_p(ws), ws_bytes, cap, ref(imgs), None)


def test_forward_rejects_bad_arguments(lib):
    m = MsMap(4096, FAKE, FAKE, FAKE, FAKE, FAKE)
    assert _fwd(lib, None) == _lib.MS_ERR_INVALID_ARG
    assert _fwd(lib, MsMap(4096, FAKE, 0, FAKE, FAKE, FAKE)) == _lib.MS_ERR_INVALID_ARG
    assert b"null map array" in lib.ms_last_error()
    assert _fwd(lib, MsMap(-3, FAKE, FAKE, FAKE, FAKE, FAKE)) == _lib.MS_ERR_INVALID_ARG
    assert _fwd(lib, m, vm=0) == _lib.MS_ERR_INVALID_ARG
    assert _fwd(lib, m, out=False) == _lib.MS_ERR_INVALID_ARG
    assert _fwd(lib, m, opts=MsOptions(24, 64, 0.2, 0)) == _lib.MS_ERR_UNSUPPORTED
    assert _fwd(lib, m, opts=MsOptions(16, 100, 0.2, 0)) == _lib.MS_ERR_UNSUPPORTED
    assert _fwd(lib, m, opts=MsOptions(16, 64, float("nan"), 0)) == _lib.MS_ERR_INVALID_ARG
    assert _fwd(lib, m, intr=MsIntrinsics(20000, 10, 1, 1, 0, 0)) == _lib.MS_ERR_INVALID_ARG
    assert _fwd(lib, m, cap=-1) == _lib.MS_ERR_INVALID_ARG
    assert _fwd(lib, m, ws=FAKE + 8) == _lib.MS_ERR_WORKSPACE
    assert _fwd(lib, m, ws=0) == _lib.MS_ERR_WORKSPACE
    assert _fwd(lib, m, ws_bytes=1024) == _lib.MS_ERR_WORKSPACE
    assert b"needed" in lib.ms_last_error()


def test_backward_rejects_bad_arguments(lib):
    m = MsMap(4096, FAKE, FAKE, FAKE, FAKE, FAKE)
    gi = MsImages(FAKE, FAKE, FAKE)
    g_all = _lib.MsGrads(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE)
    g_nopose = _lib.MsGrads(FAKE, FAKE, FAKE, FAKE, FAKE, 0, 0)

    def bwd(grads, opts=OPTS, gout=gi, ws_bytes=1024):
        return lib.ms_backward(ref(m), ctypes.c_void_p(FAKE), ref(INTR), ref(opts), ctypes.c_void_p(FAKE), ws_bytes,
                               1 << 20, ref(gout) if gout is not None else None,
                               ref(grads) if grads is not None else None, None)

    assert bwd(None) == _lib.MS_ERR_INVALID_ARG
    assert bwd(g_all, gout=None) == _lib.MS_ERR_INVALID_ARG
    assert bwd(g_nopose) == _lib.MS_ERR_INVALID_ARG                     # pose gradient requested
    assert bwd(g_nopose, opts=MsOptions(16, 64, 0.2, _lib.MS_FLAG_NO_POSE_GRAD)) == _lib.MS_ERR_WORKSPACE
    g_pose_only = _lib.MsGrads(0, 0, 0, 0, 0, FAKE, FAKE)
    assert bwd(g_pose_only) == _lib.MS_ERR_INVALID_ARG
    assert bwd(g_pose_only, opts=MsOptions(16, 64, 0.2, _lib.MS_FLAG_POSE_GRAD_ONLY)) == _lib.MS_ERR_WORKSPACE


def test_read_stats_and_view_reject_bad_workspace(lib):
    out = (ctypes.c_int64 * 7)()
    assert lib.ms_read_stats(ctypes.c_void_p(FAKE + 4), 1 << 40, 10, ref(INTR), ref(OPTS), 100, out, None) \
        == _lib.MS_ERR_WORKSPACE
    v = _lib.MsStateView()
    assert lib.ms_state_view_get(ctypes.c_void_p(FAKE), 16, 10, ref(INTR), ref(OPTS), 100, ref(v)) \
        == _lib.MS_ERR_WORKSPACE
    assert lib.ms_state_view_get(ctypes.c_void_p(FAKE), 1 << 40, 10, ref(INTR), ref(OPTS), 100, None) \
        == _lib.MS_ERR_INVALID_ARG


def test_shared_map_gradients_need_the_accumulate_flag(lib):
    """Two views of one map writing one set of map gradient arrays race
    unless both accumulate; the batch is rejected before any launch."""
    from paper_2412_09723_amd._lib import MsGrads, MsJob
    m = MsMap(4096, FAKE, FAKE, FAKE, FAKE, FAKE)
    shared = MsGrads(FAKE + 0x10000, FAKE + 0x20000, FAKE + 0x30000, FAKE + 0x40000, FAKE + 0x50000, 0, 0)
    other = MsGrads(FAKE + 0x60000, FAKE + 0x70000, FAKE + 0x80000, FAKE + 0x90000, FAKE + 0xA0000, 0, 0)
    img = MsImages(FAKE, FAKE, FAKE)

    def job(grads, flags):
        return MsJob(m, FAKE, INTR, img, img, grads, flags | _lib.MS_FLAG_NO_POSE_GRAD)

    def batch(*js):
        arr = (MsJob * len(js))(*js)
        # the workspace size is far too small: a batch that passes validation fails there
        return lib.ms_backward_batch(len(js), arr, ref(OPTS), ctypes.c_void_p(FAKE), 256, 1 << 20, None)

    acc = _lib.MS_FLAG_ACCUMULATE_MAP_GRADS
    assert batch(job(shared, 0), job(shared, 0)) == _lib.MS_ERR_INVALID_ARG
    assert batch(job(shared, acc), job(shared, 0)) == _lib.MS_ERR_INVALID_ARG
    assert batch(job(shared, acc), job(shared, acc)) == _lib.MS_ERR_WORKSPACE
    assert batch(job(shared, 0), job(other, 0)) == _lib.MS_ERR_WORKSPACE


def test_prune_rejects_bad_arguments(lib):
    m = MsMap(4096, FAKE, FAKE + 0x100000, FAKE + 0x200000, FAKE + 0x300000, FAKE + 0x400000)
    out = MsMap(4096, FAKE + 0x500000, FAKE + 0x600000, FAKE + 0x700000, FAKE + 0x800000, FAKE + 0x900000)
    kept = ctypes.c_void_p(FAKE + 0xA00000)

    def call(src=m, dst=out, to=0.005, ts=0.25, te=10.0, ws=FAKE + 0xB00000, wsb=1 << 20, k=kept):
        return lib.ms_prune(ref(src) if src is not None else None, to, ts, te, ref(dst) if dst is not None else None,
                            k, ctypes.c_void_p(ws), wsb, None)
    assert call(src=None) == _lib.MS_ERR_INVALID_ARG
    assert call(dst=None) == _lib.MS_ERR_INVALID_ARG
    assert call(k=None) == _lib.MS_ERR_INVALID_ARG
    assert call(dst=MsMap(4095, *[getattr(out, f) for f in ("means", "scales", "quats", "opacity", "colors")])) \
        == _lib.MS_ERR_INVALID_ARG                                          # capacity below n
    assert call(dst=MsMap(4096, out.means, out.scales, m.quats, out.opacity, out.colors)) == _lib.MS_ERR_INVALID_ARG
    assert call(te=-1.0) == _lib.MS_ERR_INVALID_ARG
    assert call(to=float("nan")) == _lib.MS_ERR_INVALID_ARG
    assert call(ws=0) == _lib.MS_ERR_WORKSPACE
    assert call(wsb=lib.ms_prune_workspace_bytes(4096) - 1) == _lib.MS_ERR_WORKSPACE


def test_ssim_loss_rejects_bad_arguments(lib):
    n_bytes = 3 * 64 * 48 * 4

    def call(pred=FAKE, target=FAKE + (1 << 24), C=3, W=64, H=48, weight=0.2, grad=FAKE + (2 << 24), acc=0):
        return lib.ms_ssim_loss_grad(ctypes.c_void_p(pred), ctypes.c_void_p(target), C, W, H, weight,
                                     ctypes.c_void_p(grad), acc, None, None)
    assert call(pred=0) == _lib.MS_ERR_INVALID_ARG
    assert call(grad=0) == _lib.MS_ERR_INVALID_ARG
    assert call(C=0) == _lib.MS_ERR_INVALID_ARG
    assert call(C=17) == _lib.MS_ERR_INVALID_ARG
    assert call(W=0) == _lib.MS_ERR_INVALID_ARG
    assert call(H=16385) == _lib.MS_ERR_INVALID_ARG
    assert call(weight=float("inf")) == _lib.MS_ERR_INVALID_ARG
    assert call(acc=2) == _lib.MS_ERR_INVALID_ARG
    # the gradient may not overlap an input (halo reads of other workgroups)
    assert call(grad=FAKE) == _lib.MS_ERR_INVALID_ARG
    assert call(grad=FAKE + (1 << 24)) == _lib.MS_ERR_INVALID_ARG
    assert call(grad=FAKE + n_bytes - 4) == _lib.MS_ERR_INVALID_ARG
    assert call(grad=FAKE + (1 << 24) - n_bytes + 4) == _lib.MS_ERR_INVALID_ARG
    assert "overlaps" in lib.ms_last_error().decode()


def test_product_path_has_no_oracle_dependency():
    """The package never imports the oracle (test infrastructure only)."""
    pkg = os.path.join(ROOT, "paper_2412_09723_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text, f


def test_batch_rejects_bad_arguments(lib):
    jobs = (_lib.MsJob * 2)()
    for j in range(2):
        jobs[j].map = MsMap(4096, FAKE, FAKE, FAKE, FAKE, FAKE)
        jobs[j].viewmat = FAKE
        jobs[j].intr = INTR
        jobs[j].out = MsImages(FAKE, FAKE, FAKE)
    assert lib.ms_batch_workspace_bytes(2, jobs, ref(OPTS), 1 << 20) > lib.ms_workspace_bytes(4096, ref(INTR), ref(OPTS), 1 << 20)
    assert lib.ms_batch_workspace_bytes(0, jobs, ref(OPTS), 1 << 20) == 0
    assert lib.ms_batch_workspace_bytes(_lib.MS_MAX_BATCH + 1, jobs, ref(OPTS), 1 << 20) == 0
    fwd = lambda k, js, ws=FAKE, nb=1 << 40: lib.ms_forward_batch(k, js, ref(OPTS), ctypes.c_void_p(ws), nb, 1 << 20, None)
    assert fwd(0, jobs) == _lib.MS_ERR_INVALID_ARG
    assert fwd(_lib.MS_MAX_BATCH + 1, jobs) == _lib.MS_ERR_INVALID_ARG
    assert fwd(2, None) == _lib.MS_ERR_INVALID_ARG
    assert fwd(2, jobs, nb=1024) == _lib.MS_ERR_WORKSPACE
    jobs[1].out = MsImages(FAKE, 0, FAKE)
    assert fwd(2, jobs) == _lib.MS_ERR_INVALID_ARG and b"job 1" in lib.ms_last_error()
    jobs[1].out = MsImages(FAKE, FAKE, FAKE)
    jobs[1].viewmat = 0
    assert fwd(2, jobs) == _lib.MS_ERR_INVALID_ARG
    jobs[1].viewmat = FAKE
    jobs[0].intr = MsIntrinsics(0, 10, 1, 1, 0, 0)
    assert fwd(2, jobs) == _lib.MS_ERR_INVALID_ARG
    jobs[0].intr = INTR
    # backward: a job that wants map gradients needs the arrays
    assert lib.ms_backward_batch(2, jobs, ref(OPTS), ctypes.c_void_p(FAKE), 1 << 40, 1 << 20, None) \
        == _lib.MS_ERR_INVALID_ARG


def test_prune_noalloc_rejects_bad_arguments(lib):
    """The allocation-free pruning call takes ms_prune's host checks, and
    refuses maps beyond its static scratch before touching the device."""
    m = MsMap(4096, FAKE, FAKE + 0x100000, FAKE + 0x200000, FAKE + 0x300000, FAKE + 0x400000)
    out = MsMap(4096, FAKE + 0x500000, FAKE + 0x600000, FAKE + 0x700000, FAKE + 0x800000, FAKE + 0x900000)
    kept = ctypes.c_void_p(FAKE + 0xA00000)

    def call(src=m, dst=out, to=0.005, ts=0.25, te=10.0, k=kept):
        return lib.ms_prune_noalloc(ref(src) if src is not None else None, to, ts, te,
                                    ref(dst) if dst is not None else None, k, None)
    assert call(src=None) == _lib.MS_ERR_INVALID_ARG
    assert call(dst=None) == _lib.MS_ERR_INVALID_ARG
    assert call(k=None) == _lib.MS_ERR_INVALID_ARG
    assert call(dst=MsMap(4096, out.means, out.scales, m.quats, out.opacity, out.colors)) == _lib.MS_ERR_INVALID_ARG
    assert call(te=-1.0) == _lib.MS_ERR_INVALID_ARG
    big = (1 << 26) + 1
    fields = ("means", "scales", "quats", "opacity", "colors")
    assert call(src=MsMap(big, *[getattr(m, f) for f in fields]),
                dst=MsMap(big, *[getattr(out, f) for f in fields])) == _lib.MS_ERR_INVALID_ARG
    assert "static scratch" in lib.ms_last_error().decode()


def test_select_rejects_bad_arguments(lib):
    from paper_2412_09723_amd._lib import MsIntrinsics as I
    good = I(160, 120, 150.0, 150.0, 80.0, 60.0)

    def call(means=FAKE, n=4096, vm=FAKE + 0x100000, intr=good, near=0.2, dmax=3.0, margin=0.0,
             idx=FAKE + 0x200000, cnt=FAKE + 0x300000, ws=FAKE + 0x400000, wsb=1 << 20):
        return lib.ms_select_candidates(ctypes.c_void_p(means), n, ctypes.c_void_p(vm),
                                        ref(intr) if intr is not None else None, near, dmax, margin,
                                        ctypes.c_void_p(idx), ctypes.c_void_p(cnt), ctypes.c_void_p(ws), wsb, None)
    assert call(means=0) == _lib.MS_ERR_INVALID_ARG
    assert call(vm=0) == _lib.MS_ERR_INVALID_ARG
    assert call(intr=None) == _lib.MS_ERR_INVALID_ARG
    assert call(cnt=0) == _lib.MS_ERR_INVALID_ARG
    assert call(n=-1) == _lib.MS_ERR_INVALID_ARG
    assert call(n=1 << 31) == _lib.MS_ERR_INVALID_ARG
    assert call(intr=I(0, 120, 150.0, 150.0, 80.0, 60.0)) == _lib.MS_ERR_INVALID_ARG
    assert call(intr=I(160, 120, -150.0, 150.0, 80.0, 60.0)) == _lib.MS_ERR_INVALID_ARG
    assert call(near=0.0) == _lib.MS_ERR_INVALID_ARG
    assert call(dmax=-1.0) == _lib.MS_ERR_INVALID_ARG
    assert call(margin=float("nan")) == _lib.MS_ERR_INVALID_ARG
    assert call(idx=FAKE + 64) == _lib.MS_ERR_INVALID_ARG          # indices over the means
    assert call(ws=0) == _lib.MS_ERR_WORKSPACE
    assert call(wsb=lib.ms_select_workspace_bytes(4096) - 1) == _lib.MS_ERR_WORKSPACE


def test_gicp_rejects_bad_arguments(lib):
    from paper_2412_09723_amd._lib import MsGicpConfig
    cfg = MsGicpConfig(1000, 2000, 0.02, 1e-6)
    nb = lib.ms_gicp_workspace_bytes(ref(cfg))
    assert nb > 0
    assert lib.ms_gicp_workspace_bytes(ref(MsGicpConfig(1000, 2000, 0.0, 1e-6))) == 0
    pts = MsMap(1000, FAKE, 0, 0, 0, 0)
    tgt = MsMap(2000, FAKE + 0x100000, FAKE + 0x200000, FAKE + 0x300000, 0, 0)
    ws = ctypes.c_void_p(FAKE + 0x1000000)
    T = ctypes.c_void_p(FAKE + 0x400000)
    st = None

    def build(c=cfg, t=tgt, idx=None, m=2000, w=ws, wb=nb):
        return lib.ms_gicp_build(ref(c), ref(t), ctypes.c_void_p(idx or 0), m, w, wb, st)
    assert build(c=MsGicpConfig(1000, 2000, float("nan"), 1e-6)) == _lib.MS_ERR_INVALID_ARG
    assert build(c=MsGicpConfig(1000, 2000, 0.02, -1.0)) == _lib.MS_ERR_INVALID_ARG
    assert build(m=2001, t=MsMap(2001, tgt.means, tgt.scales, tgt.quats, 0, 0)) == _lib.MS_ERR_INVALID_ARG
    assert build(m=1999) == _lib.MS_ERR_INVALID_ARG                     # m != n without an index list
    assert build(t=MsMap(2000, tgt.means, tgt.scales, 0, 0, 0)) == _lib.MS_ERR_INVALID_ARG   # scales without quats
    assert build(w=ctypes.c_void_p(0)) == _lib.MS_ERR_WORKSPACE
    assert build(w=ctypes.c_void_p(FAKE + 0x1000010)) == _lib.MS_ERR_WORKSPACE   # misaligned
    assert build(wb=nb - 1) == _lib.MS_ERR_WORKSPACE
    corr = ctypes.c_void_p(FAKE + 0x500000)
    assert lib.ms_gicp_correspond(ref(cfg), ref(MsMap(1001, FAKE, 0, 0, 0, 0)), T, corr, ws, nb, st) == \
        _lib.MS_ERR_INVALID_ARG                                          # more sources than configured
    assert lib.ms_gicp_correspond(ref(cfg), ref(pts), ctypes.c_void_p(0), corr, ws, nb, st) == _lib.MS_ERR_INVALID_ARG
    out = ctypes.c_void_p(FAKE + 0x600000)
    assert lib.ms_gicp_normal_equations(ref(cfg), ref(pts), ref(tgt), T, corr, ctypes.c_void_p(0), ws, nb, st) == \
        _lib.MS_ERR_INVALID_ARG
    assert lib.ms_gicp_align(ref(cfg), ref(pts), ref(tgt), T, -1, corr, None, ws, nb, st) == _lib.MS_ERR_INVALID_ARG
    assert lib.ms_gicp_align(ref(cfg), ref(pts), ref(tgt), T, 1001, corr, None, ws, nb, st) == _lib.MS_ERR_INVALID_ARG

"""ctypes binding of libmacsplat.so (the C ABI declared in include/macsplat.h).

Argument marshalling only: every step of the render runs in the HIP kernels of
the library. Importing this module does not touch the GPU; load() fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmacsplat.so")

MS_OK = 0
MS_ERR_INVALID_ARG = 1
MS_ERR_CAPACITY = 2
MS_ERR_WORKSPACE = 3
MS_ERR_HIP = 4
MS_ERR_UNSUPPORTED = 5
MS_FLAG_POSE_GRAD_ONLY = 1
MS_FLAG_NO_POSE_GRAD = 2
MS_FLAG_SCALAR_FWD = 4
MS_FLAG_SCALAR_BWD = 8
MS_FLAG_MFMA_BWD = 16
MS_FLAG_ACCUMULATE_MAP_GRADS = 32
MS_FLAG_BWD_BF16X3 = 64
MS_FLAG_TILE_QUEUE = 128
MS_FLAG_XCD_QUEUES = 256

EXPORTED = [
    "ms_abi_version", "ms_status_string", "ms_last_error", "ms_workspace_bytes", "ms_backward_l1",
    "ms_forward", "ms_backward", "ms_read_stats", "ms_state_view_get",
    "ms_l1_loss_grad", "ms_ssim_loss_grad", "ms_pair_loss_grad", "ms_prune_workspace_bytes", "ms_prune", "ms_prune_noalloc", "ms_select_workspace_bytes", "ms_select_candidates",
    "ms_gicp_workspace_bytes", "ms_gicp_build", "ms_gicp_correspond", "ms_gicp_normal_equations", "ms_gicp_align",
    "ms_pose_adam_step",
    "ms_profiler_create", "ms_profiler_destroy", "ms_profiler_attach", "ms_profiler_read",
    "ms_batch_workspace_bytes", "ms_forward_batch", "ms_backward_batch", "ms_batch_read_stats",
]
MS_MAX_BATCH = 12

STAGES = ["project", "bin", "composite", "composite_bwd", "project_bwd", "bin_count", "bin_emit", "bin_sort",
          "pose", "loss", "pose_step", "gicp"]


class MsIntrinsics(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float)]


class MsOptions(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("wave_batch", ctypes.c_int32), ("near_z", ctypes.c_float),
                ("flags", ctypes.c_uint32), ("bin_tile", ctypes.c_int32)]


class MsMap(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("means", ctypes.c_void_p), ("scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("opacity", ctypes.c_void_p), ("colors", ctypes.c_void_p)]


class MsImages(ctypes.Structure):
    _fields_ = [("rgb", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("silhouette", ctypes.c_void_p)]


class MsGrads(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacity", ctypes.c_void_p), ("colors", ctypes.c_void_p), ("viewmat", ctypes.c_void_p),
                ("twist", ctypes.c_void_p)]


class MsGicpConfig(ctypes.Structure):
    _fields_ = [("max_src", ctypes.c_int64), ("max_tgt", ctypes.c_int64), ("d_max", ctypes.c_float),
                ("eps", ctypes.c_float)]


class MsJob(ctypes.Structure):
    _fields_ = [("map", MsMap), ("viewmat", ctypes.c_void_p), ("intr", MsIntrinsics), ("out", MsImages),
                ("grad_out", MsImages), ("grads", MsGrads), ("flags", ctypes.c_uint32)]


class MsStateView(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in (
        "depth_key", "sorted_index", "rank_of", "pair_tile", "pair_rank", "tile_range", "records",
        "tfinal", "last", "counters", "grad2d")] + [("pair_rank_bits", ctypes.c_int32),
                                                     ("list_kind", ctypes.c_int32),
                                                     ("tile_order", ctypes.c_void_p), ("tile_cost", ctypes.c_void_p),
                                                     ("tiles", ctypes.c_int32), ("tile_waves", ctypes.c_int32)]


_lib = None


class MacsplatError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"macsplat status {status}: {detail}")
        self.status = status


def load():
    """Load the in-tree library; raise if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                           "python -m paper_2412_09723_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.ms_abi_version.restype = ctypes.c_int32
    lib.ms_status_string.argtypes = [ctypes.c_int32]
    lib.ms_status_string.restype = ctypes.c_char_p
    lib.ms_last_error.restype = ctypes.c_char_p
    lib.ms_workspace_bytes.argtypes = [ctypes.c_int64, P, P, ctypes.c_int64]
    lib.ms_workspace_bytes.restype = ctypes.c_size_t
    lib.ms_forward.argtypes = [P, P, P, P, P, ctypes.c_size_t, ctypes.c_int64, P, P]
    lib.ms_forward.restype = ctypes.c_int32
    lib.ms_backward.argtypes = [P, P, P, P, P, ctypes.c_size_t, ctypes.c_int64, P, P, P]
    lib.ms_backward.restype = ctypes.c_int32
    lib.ms_backward_l1.argtypes = [P, P, P, P, P, ctypes.c_size_t, ctypes.c_int64, P, P, ctypes.c_float,
                                   ctypes.c_float, ctypes.c_float, P, P]
    lib.ms_backward_l1.restype = ctypes.c_int32
    lib.ms_read_stats.argtypes = [P, ctypes.c_size_t, ctypes.c_int64, P, P, ctypes.c_int64, P, P]
    lib.ms_read_stats.restype = ctypes.c_int32
    lib.ms_state_view_get.argtypes = [P, ctypes.c_size_t, ctypes.c_int64, P, P, ctypes.c_int64, P]
    lib.ms_state_view_get.restype = ctypes.c_int32
    F = ctypes.c_float
    lib.ms_l1_loss_grad.argtypes = [P, P, P, F, F, F, P, P, P]
    lib.ms_l1_loss_grad.restype = ctypes.c_int32
    lib.ms_ssim_loss_grad.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, F, P, ctypes.c_int32, P, P]
    lib.ms_ssim_loss_grad.restype = ctypes.c_int32
    lib.ms_pair_loss_grad.argtypes = [P, P, P, P, ctypes.c_int32, ctypes.c_int32, F, F, F, P, P, P, P,
                                      ctypes.c_int32, P, P]
    lib.ms_pair_loss_grad.restype = ctypes.c_int32
    lib.ms_prune_workspace_bytes.argtypes = [ctypes.c_int64]
    lib.ms_prune_workspace_bytes.restype = ctypes.c_size_t
    lib.ms_prune.argtypes = [ctypes.POINTER(MsMap), F, F, F, ctypes.POINTER(MsMap), P, P, ctypes.c_size_t, P]
    lib.ms_prune.restype = ctypes.c_int32
    lib.ms_prune_noalloc.argtypes = [ctypes.POINTER(MsMap), F, F, F, ctypes.POINTER(MsMap), P, P]
    lib.ms_prune_noalloc.restype = ctypes.c_int32
    lib.ms_select_workspace_bytes.argtypes = [ctypes.c_int64]
    lib.ms_select_workspace_bytes.restype = ctypes.c_size_t
    lib.ms_select_candidates.argtypes = [P, ctypes.c_int64, P, ctypes.POINTER(MsIntrinsics), F, F, F, P, P, P,
                                         ctypes.c_size_t, P]
    lib.ms_select_candidates.restype = ctypes.c_int32
    lib.ms_gicp_workspace_bytes.argtypes = [P]
    lib.ms_gicp_workspace_bytes.restype = ctypes.c_size_t
    lib.ms_gicp_build.argtypes = [P, P, P, ctypes.c_int64, P, ctypes.c_size_t, P]
    lib.ms_gicp_build.restype = ctypes.c_int32
    lib.ms_gicp_correspond.argtypes = [P, P, P, P, P, ctypes.c_size_t, P]
    lib.ms_gicp_correspond.restype = ctypes.c_int32
    lib.ms_gicp_normal_equations.argtypes = [P, P, P, P, P, P, P, ctypes.c_size_t, P]
    lib.ms_gicp_normal_equations.restype = ctypes.c_int32
    lib.ms_gicp_align.argtypes = [P, P, P, P, ctypes.c_int32, P, P, P, ctypes.c_size_t, P]
    lib.ms_gicp_align.restype = ctypes.c_int32
    lib.ms_pose_adam_step.argtypes = [P, P, P, F, F, F, F, P]
    lib.ms_pose_adam_step.restype = ctypes.c_int32
    lib.ms_profiler_create.argtypes = [ctypes.c_uint32, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]
    lib.ms_profiler_create.restype = ctypes.c_int32
    lib.ms_profiler_destroy.argtypes = [P]
    lib.ms_profiler_destroy.restype = ctypes.c_int32
    lib.ms_profiler_attach.argtypes = [P]
    lib.ms_profiler_attach.restype = ctypes.c_int32
    lib.ms_profiler_read.argtypes = [P, P, P]
    lib.ms_profiler_read.restype = ctypes.c_int32
    I32, I64, SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    lib.ms_batch_workspace_bytes.argtypes = [I32, P, P, I64]
    lib.ms_batch_workspace_bytes.restype = SZ
    lib.ms_forward_batch.argtypes = [I32, P, P, P, SZ, I64, P]
    lib.ms_forward_batch.restype = I32
    lib.ms_backward_batch.argtypes = [I32, P, P, P, SZ, I64, P]
    lib.ms_backward_batch.restype = I32
    lib.ms_batch_read_stats.argtypes = [I32, P, P, P, SZ, I64, P, P]
    lib.ms_batch_read_stats.restype = I32
    _lib = lib
    return lib


def check(status: int):
    if status != MS_OK:
        lib = load()
        raise MacsplatError(status, (lib.ms_last_error() or b"").decode())


def ref(s):
    return ctypes.byref(s)


class Profiler:
    """Per-stage HIP-event timing of the library's launches on the calling
    thread (see ms_profiler_* in the header)."""

    def __init__(self, stages=tuple(STAGES), capacity: int = 8192):
        mask = 0
        for st in stages:
            mask |= 1 << STAGES.index(st)
        self._h = ctypes.c_void_p()
        check(load().ms_profiler_create(mask, capacity, ctypes.byref(self._h)))

    def attach(self):
        load().ms_profiler_attach(self._h)
        return self

    def detach(self):
        load().ms_profiler_attach(None)

    def read(self) -> dict:
        ms = (ctypes.c_double * len(STAGES))()
        cnt = (ctypes.c_int64 * len(STAGES))()
        check(load().ms_profiler_read(self._h, ms, cnt))
        return {st: (ms[i], cnt[i]) for i, st in enumerate(STAGES)}

    def close(self):
        if self._h:
            load().ms_profiler_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self.attach()

    def __exit__(self, *exc):
        self.detach()

"""Generalized-ICP alignment (Sec. 3.4 "3) Alignment", Eqs. 3-4; Sec. 3.5
"3) Alignment", Eq. 6) over the C ABI (ms_gicp_*): a thin holder of the
configuration and the device workspace. Maps are dicts of SoA float32
tensors on the GPU: "means" [3, n] and optionally "scales" [3, n] with
"quats" [4, n] (Gaussians; without them, points). Poses are float32 [12]
tensors [R|t] (source to target), updated in place on the device."""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import MsGicpConfig, MsMap, check, ref

SUMS = 29   # H upper triangle (21), g (6), cost, correspondence count


def _cmap(m: dict) -> MsMap:
    means = m["means"]
    if means.dim() != 2 or means.shape[0] != 3 or means.dtype != torch.float32 or not means.is_contiguous():
        raise ValueError("means must be a contiguous float32 [3, n] tensor")
    n = means.shape[1]
    sc, qt = m.get("scales"), m.get("quats")
    if (sc is None) != (qt is None):
        raise ValueError("give both scales and quats, or neither")
    if sc is not None and (tuple(sc.shape) != (3, n) or tuple(qt.shape) != (4, n) or not sc.is_contiguous()
                           or not qt.is_contiguous() or sc.dtype != torch.float32 or qt.dtype != torch.float32):
        raise ValueError("scales [3, n] and quats [4, n] must be contiguous float32")
    return MsMap(n, means.data_ptr(), sc.data_ptr() if sc is not None else 0, qt.data_ptr() if qt is not None else 0,
                 0, 0)


class GeneralizedICP:
    """Workspace and configuration of the alignment: up to max_src sources
    and max_tgt targets, correspondence distance d_max (metres), covariance
    regularisation eps (m^2)."""

    def __init__(self, max_src: int, max_tgt: int, d_max: float = 0.02, eps: float = 1e-6, device="cuda"):
        self.cfg = MsGicpConfig(int(max_src), int(max_tgt), float(d_max), float(eps))
        lib = _lib.load()
        nbytes = int(lib.ms_gicp_workspace_bytes(ref(self.cfg)))
        if nbytes == 0:
            check(_lib.MS_ERR_INVALID_ARG)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.device = self.ws.device
        self._keep = None     # the target map the grid was built from

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def build(self, tgt: dict, idx: torch.Tensor | None = None, m: int | None = None):
        """Grid over the target means: all of `tgt`, or the first m entries
        of the int32 index tensor `idx`."""
        ct = _cmap(tgt)
        if idx is not None:
            if idx.dtype != torch.int32 or not idx.is_contiguous() or idx.device != self.device:
                raise ValueError("idx must be a contiguous int32 tensor on the workspace's device")
            m = idx.numel() if m is None else int(m)
        else:
            m = ct.n
        check(_lib.load().ms_gicp_build(ref(self.cfg), ref(ct), ctypes.c_void_p(idx.data_ptr() if idx is not None else 0),
                                        m, ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), self._stream()))
        self._keep = (tgt, idx)

    def correspond(self, src: dict, T: torch.Tensor) -> torch.Tensor:
        cs = _cmap(src)
        corr = torch.empty(max(cs.n, 1), dtype=torch.int32, device=self.device)
        check(_lib.load().ms_gicp_correspond(ref(self.cfg), ref(cs), ctypes.c_void_p(T.data_ptr()),
                                             ctypes.c_void_p(corr.data_ptr()), ctypes.c_void_p(self.ws.data_ptr()),
                                             self.ws.numel(), self._stream()))
        return corr[:cs.n]

    def normal_equations(self, src: dict, tgt: dict, T: torch.Tensor, corr: torch.Tensor) -> torch.Tensor:
        cs, ct = _cmap(src), _cmap(tgt)
        out = torch.empty(SUMS, dtype=torch.float64, device=self.device)
        check(_lib.load().ms_gicp_normal_equations(ref(self.cfg), ref(cs), ref(ct), ctypes.c_void_p(T.data_ptr()),
                                                   ctypes.c_void_p(corr.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                                   ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                                   self._stream()))
        return out

    def align(self, src: dict, tgt: dict, T: torch.Tensor, iters: int = 10, history: bool = False):
        """`iters` iterations from T (updated in place). Returns (corr of the
        last iteration, [iters, 29] sums per iteration or None)."""
        cs, ct = _cmap(src), _cmap(tgt)
        if T.dtype != torch.float32 or T.numel() != 12 or T.device != self.device:
            raise ValueError("T must be a float32 [12] tensor on the workspace's device")
        corr = torch.empty(max(cs.n, 1), dtype=torch.int32, device=self.device)
        hist = torch.empty((max(iters, 1), SUMS), dtype=torch.float64, device=self.device) if history else None
        check(_lib.load().ms_gicp_align(ref(self.cfg), ref(cs), ref(ct), ctypes.c_void_p(T.data_ptr()), int(iters),
                                        ctypes.c_void_p(corr.data_ptr()),
                                        ctypes.c_void_p(hist.data_ptr() if hist is not None else 0),
                                        ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), self._stream()))
        return corr[:cs.n], (hist[:iters] if hist is not None else None)

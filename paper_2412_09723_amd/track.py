"""Device-resident tracking loop: the per-agent pose optimisation that calls
the rasterizer every iteration (Sec. 3.4; rendering-based optimisation of
poses and maps).

One iteration = forward render, gradient of the L1 loss against the
observed RGB-D frame, backward (map and pose gradients), one Adam step on the
pose's left twist. Everything is enqueued on the current stream with no host
synchronisation; the pose lives in a device tensor updated in place.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import MsImages, check, ref
from .raster import Job, RenderOptions


def _imgs(t3):
    return MsImages(t3[0].data_ptr(), t3[1].data_ptr(), t3[2].data_ptr())


class Tracker:
    def __init__(self, m: dict, viewmat: torch.Tensor, target: tuple, intr, opts: RenderOptions = RenderOptions(),
                 lr: float = 1e-3, w_rgb: float = 1.0, w_depth: float = 0.5, w_sil: float = 0.0,
                 map_grads: bool = True):
        dev = m["means"].device
        self.viewmat = viewmat
        self.job = Job(m, viewmat, intr, opts)
        H, W = intr.height, intr.width
        e = lambda *shp: torch.empty(shp, dtype=torch.float32, device=dev)
        self.out = (e(3, H, W), e(H, W), e(H, W))
        self.grad = (e(3, H, W), e(H, W), e(H, W))
        self.target = target
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.adam = torch.zeros(13, dtype=torch.float32, device=dev)
        self.map_grads = map_grads
        self.g = {}
        if map_grads:
            for k in ("means", "scales", "quats", "opacity", "colors"):
                self.g[k] = torch.empty_like(m[k])
        self.g["viewmat"] = e(12)
        self.g["twist"] = e(6)
        self.lr, self.w = lr, (w_rgb, w_depth, w_sil)
        self.c_intr = self.job.c_intr
        self._out_c, self._tgt_c, self._grad_c = _imgs(self.out), _imgs(target), _imgs(self.grad)

    def iteration(self, with_loss: bool = False):
        """One iteration; with_loss also accumulates the loss value into
        self.loss (an extra reduction)."""
        lib = _lib.load()
        stream = ctypes.c_void_p(torch.cuda.current_stream(self.viewmat.device).cuda_stream)
        self.job.forward(out=self.out)
        check(lib.ms_l1_loss_grad(ref(self._out_c), ref(self._tgt_c), ref(self.c_intr), self.w[0], self.w[1],
                                  self.w[2], ref(self._grad_c),
                                  ctypes.c_void_p(self.loss.data_ptr() if with_loss else 0), stream))
        self.job.backward(*self.grad, map_grads=self.map_grads, pose_grads=True, out=self.g)
        check(lib.ms_pose_adam_step(ctypes.c_void_p(self.viewmat.data_ptr()),
                                    ctypes.c_void_p(self.g["twist"].data_ptr()),
                                    ctypes.c_void_p(self.adam.data_ptr()), self.lr, 0.9, 0.999, 1e-8, stream))

    def step(self, iters: int = 10):
        for _ in range(iters):
            self.iteration()

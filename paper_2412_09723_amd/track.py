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
        """One iteration. The L1 loss gradient is formed inside the compositing
        backward (no gradient planes); with_loss instead runs the separate
        loss kernel, which also accumulates the loss value into self.loss."""
        lib = _lib.load()
        stream = ctypes.c_void_p(torch.cuda.current_stream(self.viewmat.device).cuda_stream)
        self.job.forward(out=self.out)
        if with_loss:
            check(lib.ms_l1_loss_grad(ref(self._out_c), ref(self._tgt_c), ref(self.c_intr), self.w[0], self.w[1],
                                      self.w[2], ref(self._grad_c), ctypes.c_void_p(self.loss.data_ptr()), stream))
            self.job.backward(*self.grad, map_grads=self.map_grads, pose_grads=True, out=self.g)
        else:
            self.job.backward_l1(self.out, self.target, *self.w, map_grads=self.map_grads, pose_grads=True,
                                 out=self.g)
        check(lib.ms_pose_adam_step(ctypes.c_void_p(self.viewmat.data_ptr()),
                                    ctypes.c_void_p(self.g["twist"].data_ptr()),
                                    ctypes.c_void_p(self.adam.data_ptr()), self.lr, 0.9, 0.999, 1e-8, stream))

    def step(self, iters: int = 10):
        for _ in range(iters):
            self.iteration()


def ssim_loss_grad(pred: torch.Tensor, target: torch.Tensor, weight: float = 0.2, grad: torch.Tensor | None = None,
                   accumulate: bool = False, loss: torch.Tensor | None = None):
    """The SSIM term weight * (1 - mean SSIM(pred, target)) of the mapping
    objective (Eq. 7) and its gradient with respect to pred, through
    ms_ssim_loss_grad. pred, target: contiguous float32 [C, H, W] on the
    device. grad (same shape) is written, or added to with accumulate; loss
    (a one-element device tensor) receives the value, or is added to with
    accumulate. Returns grad."""
    if pred.dim() != 3 or pred.shape != target.shape:
        raise ValueError(f"pred {tuple(pred.shape)} and target {tuple(target.shape)} must both be [C, H, W]")
    for name, t in (("pred", pred), ("target", target)):
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 device tensor")
    if grad is None:
        if accumulate:
            raise ValueError("accumulate needs a grad tensor")
        grad = torch.empty_like(pred)
    elif grad.shape != pred.shape or grad.dtype != torch.float32 or not grad.is_contiguous():
        raise ValueError("grad must be a contiguous float32 tensor shaped like pred")
    for name, t in (("target", target), ("grad", grad)):
        if t.device != pred.device:
            raise ValueError(f"{name} is on device {t.device}, pred on device {pred.device}")
    nbytes = pred.numel() * 4
    for name, t in (("pred", pred), ("target", target)):
        if grad.data_ptr() < t.data_ptr() + nbytes and t.data_ptr() < grad.data_ptr() + nbytes:
            raise ValueError(f"grad overlaps {name}: neighbouring windows would read pixels already overwritten")
    if loss is not None and (loss.dtype != torch.float32 or loss.numel() < 1 or loss.device != pred.device):
        raise ValueError("loss must be a float32 tensor on pred's device")
    C, H, W = pred.shape
    lib = _lib.load()
    stream = ctypes.c_void_p(torch.cuda.current_stream(pred.device).cuda_stream)
    check(lib.ms_ssim_loss_grad(ctypes.c_void_p(pred.data_ptr()), ctypes.c_void_p(target.data_ptr()), int(C), int(W),
                                int(H), float(weight), ctypes.c_void_p(grad.data_ptr()), int(bool(accumulate)),
                                ctypes.c_void_p(loss.data_ptr() if loss is not None else 0), stream))
    return grad


def prune_map(m: dict, tau_o: float = 0.005, tau_s: float = 0.25, tau_e: float = 10.0) -> dict:
    """Map pruning of App. C.1 (Algorithm 1) through ms_prune: a new map of
    the surviving Gaussians in their original order. One host synchronisation
    reads the survivor count."""
    from ._lib import MsMap
    keys = ("means", "scales", "quats", "opacity", "colors")
    n = m["means"].shape[1]
    dev = m["means"].device
    for k in keys:
        if m[k].dtype != torch.float32 or not m[k].is_contiguous() or m[k].shape[-1] != n:
            raise ValueError(f"map {k} must be contiguous float32 with n = {n} columns")
    rows = {"means": 3, "scales": 3, "quats": 4, "opacity": 1, "colors": 3}
    bufs = {k: torch.empty(rows[k] * max(n, 1), dtype=torch.float32, device=dev) for k in keys}
    kept = torch.zeros(1, dtype=torch.int64, device=dev)
    lib = _lib.load()
    wsb = int(lib.ms_prune_workspace_bytes(n))
    ws = torch.empty(max(wsb, 256), dtype=torch.uint8, device=dev)
    src = MsMap(n, *[m[k].data_ptr() for k in keys])
    dst = MsMap(n, *[bufs[k].data_ptr() for k in keys])
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    check(lib.ms_prune(ref(src), float(tau_o), float(tau_s), float(tau_e), ref(dst), ctypes.c_void_p(kept.data_ptr()),
                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), stream))
    k = int(kept.item())
    return {key: (bufs[key][:rows[key] * k].view(rows[key], k) if key != "opacity" else bufs[key][:k])
            for key in keys}


def select_candidates(means: torch.Tensor, viewmat: torch.Tensor, intr, near_z: float = 0.2, max_dist: float = 3.0,
                      margin: float = 0.0, sync: bool = True):
    """Candidate selection of Sec. 3.4 ("1) Selection") through
    ms_select_candidates: indices (int32, map order) of the Gaussians whose
    mean is in the camera's field of view and within max_dist of its pose.
    means: contiguous float32 [3, N] on the device; viewmat: float32 [12] on
    the same device. With sync (one host read of the count) returns the index
    tensor trimmed to the count; otherwise (indices [N], count [1] int64),
    both on the device."""
    from ._lib import MsIntrinsics
    if means.dim() != 2 or means.shape[0] != 3 or means.dtype != torch.float32 or not means.is_contiguous():
        raise ValueError("means must be a contiguous float32 [3, N] tensor")
    if not means.is_cuda or viewmat.device != means.device or viewmat.dtype != torch.float32 or viewmat.numel() != 12:
        raise ValueError("means and a float32 [12] viewmat must be on one device")
    n = means.shape[1]
    dev = means.device
    idx = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    lib = _lib.load()
    ws = torch.empty(max(int(lib.ms_select_workspace_bytes(n)), 256), dtype=torch.uint8, device=dev)
    c_intr = MsIntrinsics(int(intr.width), int(intr.height), float(intr.fx), float(intr.fy), float(intr.cx),
                          float(intr.cy))
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    check(lib.ms_select_candidates(ctypes.c_void_p(means.data_ptr()), n, ctypes.c_void_p(viewmat.data_ptr()),
                                   ref(c_intr), float(near_z), float(max_dist), float(margin),
                                   ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(count.data_ptr()),
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(), stream))
    if not sync:
        return idx, count
    return idx[:int(count.item())]


def pair_loss_grad(rgb_i: torch.Tensor, rgb_j: torch.Tensor, depth_i: torch.Tensor, depth_j: torch.Tensor,
                   w_l1: float = 0.8, w_ssim: float = 0.2, w_geom: float = 0.1, grads: tuple | None = None,
                   accumulate: bool = False, loss: torch.Tensor | None = None):
    """Eq. 7 for one pair of rendered views through ms_pair_loss_grad:
    w_l1 mean|I_i - I_j| + w_ssim (1 - mean SSIM(I_i, I_j)) + w_geom mean|D_i - D_j|
    (the paper's weights by default) and its gradient with respect to all
    four images. rgb_*: contiguous float32 [3, H, W], depth_*: [H, W], on one
    device. grads: (g_rgb_i, g_rgb_j, g_depth_i, g_depth_j), written or added
    to; loss: a one-element device tensor. Returns the four gradients."""
    ins = (rgb_i, rgb_j, depth_i, depth_j)
    if rgb_i.dim() != 3 or rgb_i.shape[0] != 3 or rgb_j.shape != rgb_i.shape or \
            depth_i.shape != rgb_i.shape[1:] or depth_j.shape != rgb_i.shape[1:]:
        raise ValueError("rgb_* must be [3, H, W] and depth_* [H, W] of one size")
    dev = rgb_i.device
    for t in ins:
        if t.dtype != torch.float32 or not t.is_contiguous() or t.device != dev or not t.is_cuda:
            raise ValueError("inputs must be contiguous float32 tensors on one GPU")
    if grads is None:
        if accumulate:
            raise ValueError("accumulate needs gradient tensors")
        grads = (torch.empty_like(rgb_i), torch.empty_like(rgb_j), torch.empty_like(depth_i),
                 torch.empty_like(depth_j))
    for g, t in zip(grads, ins):
        if g.shape != t.shape or g.dtype != torch.float32 or not g.is_contiguous() or g.device != dev:
            raise ValueError("gradients must be contiguous float32 tensors shaped like the inputs, on their device")
    if loss is not None and (loss.dtype != torch.float32 or loss.numel() < 1 or loss.device != dev):
        raise ValueError("loss must be a float32 tensor on the inputs' device")
    H, W = rgb_i.shape[1:]
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    lib = _lib.load()
    check(lib.ms_pair_loss_grad(*[p(t) for t in ins], int(W), int(H), float(w_l1), float(w_ssim), float(w_geom),
                                *[p(g) for g in grads], int(bool(accumulate)),
                                ctypes.c_void_p(loss.data_ptr() if loss is not None else 0),
                                ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)))
    return grads

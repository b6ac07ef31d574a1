"""PyTorch-facing entry points of the rasterizer (thin layer over the C ABI).

PyTorch supplies device memory (inputs, outputs, the workspace) and the
current HIP stream; all arithmetic runs in libmacsplat's HIP kernels.

Map tensors use the ABI's structure-of-arrays layout: means/scales [3, N],
quats [4, N] (w, x, y, z), opacity [N], colors [3, N], float32, on the GPU.
`to_soa` converts [N, 3]-style tensors once.
"""
from __future__ import annotations

import ctypes
import dataclasses

import torch

from . import _lib
from ._lib import MsGrads, MsImages, MsIntrinsics, MsMap, MsOptions, MsStateView, check, ref

NEAR_Z = 0.2


@dataclasses.dataclass(frozen=True)
class RenderOptions:
    tile: int = 16
    bin_tile: int = 128                  # 0: bin at `tile`; else a power of two in [tile, 256]
    wave_batch: int = 64
    near_z: float = NEAR_Z
    pair_capacity: int | None = None     # None: sized from the map (see default_capacity)
    check: bool = False                  # read the device counters after the forward (synchronises)
    fwd_records: str = "lds"             # forward compositing record path: "lds" staging or "scalar" (SGPR)
    bwd_records: str = "mfma"            # backward compositing: "mfma" (per-Gaussian pixel reduction on the
                                         # matrix cores in binary32), "mfma_bf16x3" (the same product from
                                         # bf16 high/low parts), "lds" or "scalar" (wave reductions)
    grow: bool = True                    # with check: enlarge the pair capacity and redo on overflow
    schedule: str = "grid"               # compositing launch: "grid" (one workgroup per tile), "queue"
                                         # (persistent workgroups taking tiles longest-first from one
                                         # queue) or "xcd_queue" (eight queues, one per XCD)


def default_capacity(n: int, width: int, height: int, tile: int) -> int:
    """Pair capacity heuristic: (8 + 512/tile) pairs per Gaussian plus 64 per
    tile (a 1M-Gaussian room at 1200x680 needs about 7 pairs per Gaussian at
    tile 16 and 24 at tile 8). A checked forward grows it when exceeded."""
    tiles = ((width + tile - 1) // tile) * ((height + tile - 1) // tile)
    return int(min((8 + 512 // tile) * n + 64 * tiles + 4096, 0xFFFFFFFF))


def to_soa(t: torch.Tensor) -> torch.Tensor:
    """[N, k] -> contiguous [k, N]."""
    return t.t().contiguous() if t.dim() == 2 else t.contiguous()


def intr_struct(intr) -> MsIntrinsics:
    return MsIntrinsics(int(intr.width), int(intr.height), float(intr.fx), float(intr.fy), float(intr.cx),
                        float(intr.cy))


def opts_struct(opts: RenderOptions, flags: int = 0) -> MsOptions:
    if opts.fwd_records == "scalar":
        flags |= _lib.MS_FLAG_SCALAR_FWD
    if opts.bwd_records == "scalar":
        flags |= _lib.MS_FLAG_SCALAR_BWD
    if opts.bwd_records in ("mfma", "mfma_bf16x3"):
        flags |= _lib.MS_FLAG_MFMA_BWD
    if opts.bwd_records == "mfma_bf16x3":
        flags |= _lib.MS_FLAG_BWD_BF16X3
    if opts.schedule not in ("grid", "queue", "xcd_queue"):
        raise ValueError(f"schedule {opts.schedule!r} not in ('grid', 'queue', 'xcd_queue')")
    if opts.schedule in ("queue", "xcd_queue"):
        flags |= _lib.MS_FLAG_TILE_QUEUE
    if opts.schedule == "xcd_queue":
        flags |= _lib.MS_FLAG_XCD_QUEUES
    return MsOptions(int(opts.tile), int(opts.wave_batch), float(opts.near_z), int(flags), int(opts.bin_tile))


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream_ptr(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_map(m: dict):
    n = m["means"].shape[1]
    shapes = {"means": (3, n), "scales": (3, n), "quats": (4, n), "opacity": (n,), "colors": (3, n)}
    dev = m["means"].device
    for k, shp in shapes.items():
        t = m[k]
        if tuple(t.shape) != shp:
            raise ValueError(f"{k} has shape {tuple(t.shape)}, expected {shp}")
        if t.dtype != torch.float32 or t.device != dev:
            raise ValueError(f"{k} must be float32 on {dev}")
        if not t.is_contiguous():
            raise ValueError(f"{k} must be contiguous")
    if dev.type != "cuda":
        raise ValueError("map tensors must live on the GPU")
    return n


def _stamp(ws: torch.Tensor) -> int:
    """Marks a new forward in workspace `ws` and returns its generation."""
    gen = getattr(ws, "_ms_generation", 0) + 1
    ws._ms_generation = gen
    return gen


class Job:
    """One render job: its map, pose, intrinsics, options and workspace.

    The workspace is a caller-owned uint8 tensor; the forward state stays in
    it until the next forward in the same workspace, by this Job or another
    one sharing it. backward() raises if such a forward has run since this
    Job's forward (the state it would read is gone)."""

    def __init__(self, m: dict, viewmat: torch.Tensor, intr, opts: RenderOptions = RenderOptions(),
                 workspace: torch.Tensor | None = None):
        self.m = m
        self.n = _check_map(m)
        self.viewmat = viewmat
        if viewmat.shape != (12,) or viewmat.dtype != torch.float32 or viewmat.device != m["means"].device:
            raise ValueError("viewmat must be a float32 [12] tensor on the map's device")
        self.intr = intr
        self.opts = opts
        self.cap = opts.pair_capacity if opts.pair_capacity is not None else default_capacity(
            self.n, intr.width, intr.height, opts.bin_tile or opts.tile)
        self.c_intr = intr_struct(intr)
        self.c_map = MsMap(self.n, m["means"].data_ptr(), m["scales"].data_ptr(), m["quats"].data_ptr(),
                           m["opacity"].data_ptr(), m["colors"].data_ptr())
        lib = _lib.load()
        self.ws_bytes = lib.ms_workspace_bytes(self.n, ref(self.c_intr), ref(opts_struct(opts)), self.cap)
        if self.ws_bytes == 0:
            check(_lib.MS_ERR_INVALID_ARG)
        if workspace is None or workspace.numel() < self.ws_bytes:
            workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=m["means"].device)
        self.ws = workspace
        self._gen = None       # generation of this Job's last forward in self.ws

    # -- forward -----------------------------------------------------------
    def forward(self, out: tuple | None = None):
        H, W = self.intr.height, self.intr.width
        dev = self.m["means"].device
        if out is None:
            rgb = torch.empty((3, H, W), dtype=torch.float32, device=dev)
            depth = torch.empty((H, W), dtype=torch.float32, device=dev)
            sil = torch.empty((H, W), dtype=torch.float32, device=dev)
        else:
            rgb, depth, sil = out
        imgs = MsImages(rgb.data_ptr(), depth.data_ptr(), sil.data_ptr())
        lib = _lib.load()
        self._gen = _stamp(self.ws)
        check(lib.ms_forward(ref(self.c_map), _ptr(self.viewmat), ref(self.c_intr), ref(opts_struct(self.opts)),
                             _ptr(self.ws), self.ws_bytes, self.cap, ref(imgs), _stream_ptr(dev)))
        if self.opts.check:
            st = self.stats()
            if st["overflow"]:
                if not self.opts.grow:
                    raise _lib.MacsplatError(_lib.MS_ERR_CAPACITY,
                                             f"{st['pairs']} pairs exceed the capacity {self.cap}")
                self._resize(int(min(st["pairs"] * 5 // 4 + 4096, 0xFFFFFFFF)))
                return self.forward(out=(rgb, depth, sil))
        return rgb, depth, sil

    def _resize(self, cap: int):
        lib = _lib.load()
        self.cap = cap
        self.ws_bytes = lib.ms_workspace_bytes(self.n, ref(self.c_intr), ref(opts_struct(self.opts)), self.cap)
        if self.ws_bytes == 0:
            check(_lib.MS_ERR_INVALID_ARG)
        if self.ws.numel() < self.ws_bytes:
            self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.m["means"].device)

    # -- backward ----------------------------------------------------------
    def backward(self, g_rgb, g_depth, g_sil, map_grads: bool = True, pose_grads: bool = True,
                 out: dict | None = None) -> dict:
        if self._gen is None:
            raise RuntimeError("backward() needs a forward() on this Job first")
        if getattr(self.ws, "_ms_generation", None) != self._gen:
            raise RuntimeError("another forward has run in this Job's workspace since its forward(); the forward "
                               "state the backward reads is gone (give each pending render its own workspace)")
        dev = self.m["means"].device
        flags = 0
        if not map_grads:
            flags |= _lib.MS_FLAG_POSE_GRAD_ONLY
        if not pose_grads:
            flags |= _lib.MS_FLAG_NO_POSE_GRAD
        g = out if out is not None else {}
        if map_grads and out is None:
            for k in ("means", "scales", "quats", "opacity", "colors"):
                g[k] = torch.empty_like(self.m[k])
        if pose_grads and out is None:
            g["viewmat"] = torch.empty(12, dtype=torch.float32, device=dev)
            g["twist"] = torch.empty(6, dtype=torch.float32, device=dev)
        gi = MsImages(g_rgb.data_ptr(), g_depth.data_ptr(), g_sil.data_ptr())
        gg = MsGrads(*[g[k].data_ptr() if k in g else 0
                       for k in ("means", "scales", "quats", "opacity", "colors", "viewmat", "twist")])
        lib = _lib.load()
        check(lib.ms_backward(ref(self.c_map), _ptr(self.viewmat), ref(self.c_intr),
                              ref(opts_struct(self.opts, flags)), _ptr(self.ws), self.ws_bytes, self.cap, ref(gi),
                              ref(gg), _stream_ptr(dev)))
        return g

    def backward_l1(self, pred: tuple, target: tuple, w_rgb: float = 1.0, w_depth: float = 0.5, w_sil: float = 0.0,
                    map_grads: bool = True, pose_grads: bool = True, out: dict | None = None) -> dict:
        """Backward of the L1 loss w_rgb mean|rgb - rgb*| + w_depth mean|D - D*|
        + w_sil mean|S - S*| between the images of the last forward (`pred`,
        as it returned them) and `target`, with the loss gradient formed
        inside the compositing backward (ms_backward_l1): the same gradients,
        bit for bit, as ms_l1_loss_grad then backward()."""
        if self._gen is None or getattr(self.ws, "_ms_generation", None) != self._gen:
            raise RuntimeError("backward_l1() needs this Job's forward state, and another forward has run in its "
                               "workspace since (or none has run)")
        dev = self.m["means"].device
        flags = (0 if map_grads else _lib.MS_FLAG_POSE_GRAD_ONLY) | (0 if pose_grads else _lib.MS_FLAG_NO_POSE_GRAD)
        g = out if out is not None else {}
        if map_grads and out is None:
            for k in ("means", "scales", "quats", "opacity", "colors"):
                g[k] = torch.empty_like(self.m[k])
        if pose_grads and out is None:
            g["viewmat"] = torch.empty(12, dtype=torch.float32, device=dev)
            g["twist"] = torch.empty(6, dtype=torch.float32, device=dev)
        pi = MsImages(pred[0].data_ptr(), pred[1].data_ptr(), pred[2].data_ptr())
        ti = MsImages(target[0].data_ptr(), target[1].data_ptr(), target[2].data_ptr())
        gg = MsGrads(*[g[k].data_ptr() if k in g else 0
                       for k in ("means", "scales", "quats", "opacity", "colors", "viewmat", "twist")])
        lib = _lib.load()
        check(lib.ms_backward_l1(ref(self.c_map), _ptr(self.viewmat), ref(self.c_intr),
                                 ref(opts_struct(self.opts, flags)), _ptr(self.ws), self.ws_bytes, self.cap, ref(pi),
                                 ref(ti), float(w_rgb), float(w_depth), float(w_sil), ref(gg), _stream_ptr(dev)))
        return g

    # -- inspection ---------------------------------------------------------
    def stats(self) -> dict:
        out = (ctypes.c_int64 * 7)()
        lib = _lib.load()
        check(lib.ms_read_stats(_ptr(self.ws), self.ws_bytes, self.n, ref(self.c_intr), ref(opts_struct(self.opts)),
                                self.cap, out, _stream_ptr(self.m["means"].device)))
        return dict(visible=out[0], pairs=out[1], overflow=bool(out[2]), tiles=out[3], composited=out[4],
                    staged=out[5], reduced=out[6])

    def state(self) -> dict:
        """Device views of the forward state (see ms_state_view in the header)."""
        v = MsStateView()
        lib = _lib.load()
        check(lib.ms_state_view_get(_ptr(self.ws), self.ws_bytes, self.n, ref(self.c_intr),
                                    ref(opts_struct(self.opts)), self.cap, ref(v)))
        base = self.ws.data_ptr()
        n = max(self.n, 1)
        H, W = self.intr.height, self.intr.width
        t = self.opts.bin_tile or self.opts.tile
        tiles = ((W + t - 1) // t) * ((H + t - 1) // t)

        def view(ptr, count, dtype):
            off = ptr - base
            nbytes = count * torch.empty((), dtype=dtype).element_size()
            return self.ws[off:off + nbytes].view(dtype)

        kind = int(v.list_kind)
        pair_rank = view(v.pair_rank, max(self.cap, 1), torch.int32)
        pair_tile = view(v.pair_tile, max(self.cap, 1), torch.int32) if kind == 0 else None
        if v.pair_rank_bits > 0:       # packed pair words: tile << bits | rank
            bits = v.pair_rank_bits
            words = pair_tile.to(torch.int64) & 0xFFFFFFFF
            pair_tile = (words >> bits).to(torch.int32)
            pair_rank = (words & ((1 << bits) - 1)).to(torch.int32)
        return dict(
            list_kind=kind,
            depth_key=view(v.depth_key, n, torch.int32),
            sorted_index=view(v.sorted_index, n, torch.int32) if kind == 0 else None,
            rank_of=view(v.rank_of, n, torch.int32) if kind == 0 else None,
            pair_tile=pair_tile,
            pair_rank=pair_rank,
            tile_range=view(v.tile_range, 2 * tiles, torch.int32).view(tiles, 2),
            records=view(v.records, 16 * n, torch.float32).view(n, 16),
            tfinal=view(v.tfinal, H * W, torch.float32).view(H, W),
            last=view(v.last, H * W, torch.int32).view(H, W),
            counters=view(v.counters, 8, torch.int64),
            grad2d=view(v.grad2d, 10 * n, torch.float32).view(n, 10),
            pair_rank_bits=int(v.pair_rank_bits),
            tile_order=view(v.tile_order, int(v.tiles), torch.int32),
            tile_cost=view(v.tile_cost, int(v.tiles) * int(v.tile_waves), torch.int32).view(int(v.tiles),
                                                                                           int(v.tile_waves)),
        )


class BatchJob:
    """Several render jobs -- one map, pose and camera each, shapes and sizes
    free -- rendered through one launch sequence per pass (ms_forward_batch /
    ms_backward_batch). Every job's result equals rendering it alone. All
    jobs share `opts`; the pair capacity covers all jobs together."""

    def __init__(self, maps: list, viewmats: list, intrs: list, opts: RenderOptions = RenderOptions(),
                 workspace: torch.Tensor | None = None):
        k = len(maps)
        if not 1 <= k <= _lib.MS_MAX_BATCH or len(viewmats) != k or len(intrs) != k:
            raise ValueError(f"a batch holds 1..{_lib.MS_MAX_BATCH} jobs with one viewmat and intrinsics each")
        self.maps, self.viewmats, self.intrs, self.opts = list(maps), list(viewmats), list(intrs), opts
        self.ns = [_check_map(m) for m in maps]
        dev = maps[0]["means"].device
        for m, vm in zip(maps, viewmats):
            if m["means"].device != dev or vm.shape != (12,) or vm.dtype != torch.float32 or vm.device != dev:
                raise ValueError("all maps and viewmats must be float32 tensors on one device")
        self.device = dev
        b = opts.bin_tile or opts.tile
        self.cap = opts.pair_capacity if opts.pair_capacity is not None else min(
            sum(default_capacity(n, i.width, i.height, b) for n, i in zip(self.ns, intrs)), 0xFFFFFFFF)
        self.c_jobs = (_lib.MsJob * k)()
        for j, (m, vm, intr) in enumerate(zip(maps, viewmats, intrs)):
            self.c_jobs[j].map = MsMap(self.ns[j], m["means"].data_ptr(), m["scales"].data_ptr(),
                                       m["quats"].data_ptr(), m["opacity"].data_ptr(), m["colors"].data_ptr())
            self.c_jobs[j].viewmat = vm.data_ptr()
            self.c_jobs[j].intr = intr_struct(intr)
        self.ws = workspace
        self._gen = None
        self._size_workspace()

    def _size_workspace(self):
        lib = _lib.load()
        self.ws_bytes = lib.ms_batch_workspace_bytes(len(self.maps), self.c_jobs, ref(opts_struct(self.opts)),
                                                     self.cap)
        if self.ws_bytes == 0:
            check(_lib.MS_ERR_INVALID_ARG)
        if self.ws is None or self.ws.numel() < self.ws_bytes:
            self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)

    def forward(self, outs: list | None = None) -> list:
        """Renders every job; returns [(rgb, depth, silhouette)] in job order."""
        if outs is None:
            outs = []
            for intr in self.intrs:
                H, W = intr.height, intr.width
                outs.append((torch.empty((3, H, W), dtype=torch.float32, device=self.device),
                             torch.empty((H, W), dtype=torch.float32, device=self.device),
                             torch.empty((H, W), dtype=torch.float32, device=self.device)))
        for j, (rgb, depth, sil) in enumerate(outs):
            self.c_jobs[j].out = MsImages(rgb.data_ptr(), depth.data_ptr(), sil.data_ptr())
        lib = _lib.load()
        self._gen = _stamp(self.ws)
        check(lib.ms_forward_batch(len(self.maps), self.c_jobs, ref(opts_struct(self.opts)), _ptr(self.ws),
                                   self.ws_bytes, self.cap, _stream_ptr(self.device)))
        if self.opts.check:
            st = self.stats()
            if st["overflow"]:
                if not self.opts.grow:
                    raise _lib.MacsplatError(_lib.MS_ERR_CAPACITY,
                                             f"{st['pairs']} pairs exceed the capacity {self.cap}")
                self.cap = int(min(st["pairs"] * 5 // 4 + 4096, 0xFFFFFFFF))
                self._size_workspace()
                return self.forward(outs)
        return outs

    def backward(self, upstream: list, map_grads=True, pose_grads=True, outs: list | None = None,
                 shared_map_grads: dict | None = None) -> list:
        """Backward of the last forward. upstream: [(g_rgb, g_depth, g_sil)] in
        job order; map_grads / pose_grads: a bool or one bool per job.
        Returns one gradient dict per job, as Job.backward. shared_map_grads:
        for jobs that are views of one map, a dict of gradient tensors shaped
        like that map; it is zeroed and every job with map gradients adds its
        gradients into it (MS_FLAG_ACCUMULATE_MAP_GRADS), so it ends up with
        their sum over the views."""
        if self._gen is None or getattr(self.ws, "_ms_generation", None) != self._gen:
            raise RuntimeError("backward() needs this batch's forward state, and another forward has run in its "
                               "workspace since (or none has run)")
        k = len(self.maps)
        mg = [map_grads] * k if isinstance(map_grads, bool) else list(map_grads)
        pg = [pose_grads] * k if isinstance(pose_grads, bool) else list(pose_grads)
        if shared_map_grads is not None:
            for key in ("means", "scales", "quats", "opacity", "colors"):
                for j in range(k):
                    if mg[j] and self.maps[j][key].shape != shared_map_grads[key].shape:
                        raise ValueError(f"job {j}: map {key} shape differs from the shared gradient")
                shared_map_grads[key].zero_()
        res = []
        for j in range(k):
            g = outs[j] if outs is not None else {}
            if mg[j] and shared_map_grads is not None:
                g.update({key: shared_map_grads[key] for key in ("means", "scales", "quats", "opacity", "colors")})
            elif mg[j] and outs is None:
                for key in ("means", "scales", "quats", "opacity", "colors"):
                    g[key] = torch.empty_like(self.maps[j][key])
            if pg[j] and outs is None:
                g["viewmat"] = torch.empty(12, dtype=torch.float32, device=self.device)
                g["twist"] = torch.empty(6, dtype=torch.float32, device=self.device)
            gr, gd, gs = upstream[j]
            self.c_jobs[j].grad_out = MsImages(gr.data_ptr(), gd.data_ptr(), gs.data_ptr())
            self.c_jobs[j].grads = MsGrads(*[g[key].data_ptr() if key in g else 0 for key in
                                             ("means", "scales", "quats", "opacity", "colors", "viewmat", "twist")])
            self.c_jobs[j].flags = (0 if mg[j] else _lib.MS_FLAG_POSE_GRAD_ONLY) | \
                (0 if pg[j] else _lib.MS_FLAG_NO_POSE_GRAD) | \
                (_lib.MS_FLAG_ACCUMULATE_MAP_GRADS if mg[j] and shared_map_grads is not None else 0)
            res.append(g)
        lib = _lib.load()
        check(lib.ms_backward_batch(k, self.c_jobs, ref(opts_struct(self.opts)), _ptr(self.ws), self.ws_bytes,
                                    self.cap, _stream_ptr(self.device)))
        return res

    def stats(self) -> dict:
        out = (ctypes.c_int64 * 7)()
        lib = _lib.load()
        check(lib.ms_batch_read_stats(len(self.maps), self.c_jobs, ref(opts_struct(self.opts)), _ptr(self.ws),
                                      self.ws_bytes, self.cap, out, _stream_ptr(self.device)))
        return dict(visible=out[0], pairs=out[1], overflow=bool(out[2]), tiles=out[3], composited=out[4],
                    staged=out[5], reduced=out[6])


class RasterizeRGBD(torch.autograd.Function):
    """Differentiable RGB-D render: (map, viewmat) -> (rgb, depth, silhouette).

    The backward recomputes per-pixel transmittance from the forward's final
    transmittance and last index (no per-Gaussian per-pixel state). The
    left-twist pose gradient of the last backward is kept on the Job as
    `job.twist_grad`."""

    @staticmethod
    def forward(ctx, means, scales, quats, opacity, colors, viewmat, intr, opts, holder):
        m = dict(means=means.contiguous(), scales=scales.contiguous(), quats=quats.contiguous(),
                 opacity=opacity.contiguous(), colors=colors.contiguous())
        vm = viewmat.contiguous()
        # the holder keeps a pool of workspaces; one whose forward still awaits
        # its backward is never handed out again (two renders before one
        # backward, as in a multi-view mapping step, each get their own)
        pool = holder.setdefault("pool", [])
        free = [e for e in pool if not e["busy"]]
        entry = free[0] if free else None
        job = Job(m, vm, intr, opts, entry["ws"] if entry is not None else None)
        if entry is None:
            entry = {"ws": job.ws, "busy": False}
            pool.append(entry)
        entry["ws"] = job.ws
        holder["workspace"] = job.ws
        holder["job"] = job
        rgb, depth, sil = job.forward()
        entry["ws"] = job.ws          # a checked forward may have grown it
        if any(ctx.needs_input_grad[:6]):
            entry["busy"] = True
        ctx.job = job
        ctx.entry = entry
        ctx.needs = ctx.needs_input_grad
        # saved so that autograd refuses a backward after an in-place update of
        # the map or the pose
        ctx.save_for_backward(m["means"], m["scales"], m["quats"], m["opacity"], m["colors"], vm)
        return rgb, depth, sil

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, g_rgb, g_depth, g_sil):
        ctx.saved_tensors              # version check of the map and pose tensors
        job = ctx.job
        ctx.entry["busy"] = False
        H, W = job.intr.height, job.intr.width
        dev = job.m["means"].device
        z = lambda shp: torch.zeros(shp, dtype=torch.float32, device=dev)
        g_rgb = z((3, H, W)) if g_rgb is None else g_rgb.contiguous()
        g_depth = z((H, W)) if g_depth is None else g_depth.contiguous()
        g_sil = z((H, W)) if g_sil is None else g_sil.contiguous()
        need_map = any(ctx.needs[:5])
        need_pose = bool(ctx.needs[5])
        g = job.backward(g_rgb, g_depth, g_sil, map_grads=need_map or not need_pose, pose_grads=need_pose)
        job.twist_grad = g.get("twist")
        gm = lambda k, i: g.get(k) if ctx.needs[i] else None
        return (gm("means", 0), gm("scales", 1), gm("quats", 2), gm("opacity", 3), gm("colors", 4),
                g.get("viewmat") if need_pose else None, None, None, None)


def render(m: dict, viewmat: torch.Tensor, intr, opts: RenderOptions = RenderOptions(), holder: dict | None = None):
    """Differentiable render of a map (dict of SoA tensors) from `viewmat`.

    `holder` (optional dict) keeps workspaces across calls (a pool: a render
    whose backward is still pending keeps its own) and receives the last Job
    under "job"."""
    holder = {} if holder is None else holder
    return RasterizeRGBD.apply(m["means"], m["scales"], m["quats"], m["opacity"], m["colors"], viewmat, intr, opts,
                               holder)

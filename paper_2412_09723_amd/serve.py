"""Continuous-batching request loop for render + backward jobs of many agents.

Every agent keeps its map, its camera intrinsics, the poses of its camera
walk and its observed frame resident on the device (the agents run their
tracking and mapping independently and asynchronously, Sec. 3.6). A request
asks for one forward render at a pose of the walk, the L1 gradient against
the agent's frame and one backward: tracking requests want the pose gradient
only, mapping requests every gradient.

The loop replays arrival times on the host clock. Whenever fewer than
`inflight` rounds are on the device and requests are waiting, the scheduler
packs the waiting requests, first come first served, into one round of at
most `max_batch` requests whose estimated device bytes fit the HBM budget
left by the rounds in flight, and the executor launches the round as one
batched forward / loss / backward sequence on its own stream (two streams by
default, so a round that is admitted while another runs overlaps it on the
device). A finished round frees its memory; requests that arrived meanwhile
go into the next round. Latency is arrival to the host's first observation
of the round's completion event.

The scheduler is plain host logic, independent of the GPU (the tests drive
it with a simulated executor); `GpuExecutor` runs rounds through
`raster.BatchJob`, `PlainExecutor` runs one request at a time through
`raster.Job` (the sequential baseline).
"""
from __future__ import annotations

import collections
import ctypes
import dataclasses
import math
import time

import numpy as np
import torch

from . import _lib, raster, scenes
from ._lib import MsImages, check, ref


@dataclasses.dataclass
class Request:
    rid: int
    agent: int
    arrival: float          # seconds from the start of the run
    step: int               # index of the pose on the agent's camera walk
    mapping: bool           # True: all gradients; False: pose gradient only


@dataclasses.dataclass
class Done:
    rid: int
    agent: int
    arrival: float
    launched: float
    finished: float
    batch: int              # requests in the request's round
    outputs: dict | None = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Scheduler:
    """First-come-first-served admission into rounds of at most `max_batch`
    requests whose estimated bytes fit what the in-flight rounds leave of
    `budget_bytes`; at most `inflight` rounds on the device at once.

    A request whose own estimate exceeds the whole budget, or whose estimate
    cannot be made (an invalid job), never runs: it fails alone, with the
    reason. A request in `solo` (one whose round failed to launch) is admitted
    only as a round of its own, so that an invalid job fails alone."""

    def __init__(self, max_batch: int, budget_bytes: int, inflight: int, cost_bytes):
        if max_batch < 1 or inflight < 1 or budget_bytes <= 0:
            raise ValueError("max_batch, inflight and budget must be positive")
        self.max_batch = max_batch
        self.budget = budget_bytes
        self.inflight = inflight
        self.cost_bytes = cost_bytes
        self.solo: set[int] = set()

    def admit(self, queue: collections.deque, used_bytes: int):
        """Pops the next round off `queue`; returns (requests, bytes, failed)
        with `failed` a list of (request, reason)."""
        batch, total, failed = [], 0, []
        while queue and len(batch) < self.max_batch:
            r = queue[0]
            try:
                c = int(self.cost_bytes(r))
            except Exception as e:          # noqa: BLE001 -- the reason is reported with the request
                failed.append((queue.popleft(), f"invalid job: {e}"))
                continue
            if c > self.budget:
                failed.append((queue.popleft(), f"needs {c} bytes, over the budget of {self.budget}"))
                continue
            if r.rid in self.solo and batch:
                break
            if used_bytes + total + c > self.budget:
                break
            batch.append(queue.popleft())
            total += c
            if r.rid in self.solo:
                break
        return batch, total, failed


class Server:
    """Replays `requests` in real time through `executor` under `scheduler`.

    `executor` provides launch(requests) -> handle (raises if the round cannot
    be launched), done(handle) -> bool and collect(handle) -> per-request
    outputs or None."""

    def __init__(self, executor, scheduler: Scheduler, clock=time.perf_counter, sleep=time.sleep):
        self.executor = executor
        self.scheduler = scheduler
        self.clock = clock
        self.sleep = sleep

    def run(self, requests: list[Request]):
        """Returns (done, failed, info): completed requests, (request, reason)
        pairs that did not run, and the wall time and peak admitted bytes."""
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        queue: collections.deque = collections.deque()
        inflight = []          # [handle, requests, bytes, launched]
        done: list[Done] = []
        failed: list = []
        peak_bytes = 0
        rounds = 0
        t0 = self.clock()
        while pending or queue or inflight:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            progressed = False
            for entry in list(inflight):
                handle, reqs, nbytes, launched = entry
                if self.executor.done(handle):
                    # collect() may re-run the round (capacity overflow); the
                    # result is ready only when it returns
                    outs = self.executor.collect(handle)
                    fin = self.clock() - t0
                    for k, r in enumerate(reqs):
                        done.append(Done(r.rid, r.agent, r.arrival, launched, fin, len(reqs),
                                         outs[k] if outs is not None else None))
                    inflight.remove(entry)
                    progressed = True
            if queue and len(inflight) < self.scheduler.inflight:
                used = sum(e[2] for e in inflight)
                batch, nbytes, bad = self.scheduler.admit(queue, used)
                failed += bad
                progressed = progressed or bool(bad)
                if batch:
                    launched = self.clock() - t0
                    try:
                        handle = self.executor.launch(batch)
                    except Exception as e:      # noqa: BLE001 -- split the round; a lone failure is reported
                        if len(batch) == 1:
                            failed.append((batch[0], f"launch failed: {e}"))
                        else:
                            self.scheduler.solo.update(r.rid for r in batch)
                            queue.extendleft(reversed(batch))
                    else:
                        inflight.append([handle, batch, nbytes, launched])
                        peak_bytes = max(peak_bytes, used + nbytes)
                        rounds += 1
                    progressed = True
            if not progressed:
                if not inflight and not queue and pending:
                    self.sleep(max(0.0, pending[0].arrival - (self.clock() - t0)))
                else:
                    self.sleep(0)
        wall = self.clock() - t0
        return done, failed, dict(wall_s=wall, peak_bytes=peak_bytes, rounds=rounds)


def summarize(done: list[Done], wall_s: float) -> dict:
    """Throughput (completed jobs per second from the first arrival to the
    last completion) and latency percentiles (arrival to completion) of a run."""
    if not done:
        return dict(jobs=0)
    lat = np.array([d.latency for d in done]) * 1e3
    last = max(d.finished for d in done)
    first = min(d.arrival for d in done)
    return dict(jobs=len(done), frames_s=round(len(done) / max(last - first, 1e-9), 2),
                p50_ms=round(float(np.percentile(lat, 50)), 3), p99_ms=round(float(np.percentile(lat, 99)), 3),
                mean_ms=round(float(lat.mean()), 3), max_ms=round(float(lat.max()), 3),
                mean_batch=round(float(np.mean([d.batch for d in done])), 2), wall_s=round(wall_s, 3))


# ---------------------------------------------------------------- GPU side

@dataclasses.dataclass
class Agent:
    """Device-resident state of one agent."""
    map: dict               # SoA float32 tensors
    intr: object
    poses: torch.Tensor     # [steps, 12] world-to-camera poses of the walk
    target: tuple           # observed (rgb, depth, silhouette)

    @property
    def n(self) -> int:
        return int(self.map["means"].shape[1])


def camera_walk(base_viewmat: np.ndarray, steps: int, rng, step_m: float = 0.002, step_deg: float = 0.1):
    """Seeded random walk of the camera: each step moves it by `step_m` along
    a random direction and turns it by `step_deg` about a random axis (left
    perturbation of the world-to-camera pose)."""
    poses = np.empty((steps, 12), np.float32)
    V = np.asarray(base_viewmat, np.float64).reshape(3, 4).copy()
    th = math.radians(step_deg)
    for k in range(steps):
        poses[k] = V.reshape(12)
        d = rng.standard_normal(3)
        d *= step_m / np.linalg.norm(d)
        a = rng.standard_normal(3)
        a /= np.linalg.norm(a)
        K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
        Rx = np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * (K @ K)
        V = np.concatenate([Rx @ V[:, :3], (Rx @ V[:, 3] + d).reshape(3, 1)], axis=1)
    return poses


def make_agents(scs: list, steps: int, device="cuda", opts: raster.RenderOptions = raster.RenderOptions()):
    """Resident agents from scenes: map, camera walk from the scene's pose,
    and an observed frame rendered from a pose 2 cm / 1 degree off the walk's
    start."""
    agents = []
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    for a, sc in enumerate(scs):
        m = dict(means=t(sc.means), scales=t(sc.scales), quats=t(sc.quats), opacity=t(sc.opacity),
                 colors=t(sc.colors))
        poses = t(camera_walk(sc.viewmat, max(steps, 1), scenes.rng_for(4, a, salt=5)))
        vm_obs = t(scenes.perturb_pose(sc.viewmat, scenes.rng_for(4, a, salt=3)))
        target = raster.Job(m, vm_obs, sc.intr, dataclasses.replace(opts, check=True)).forward()
        agents.append(Agent(m, sc.intr, poses, target))
    torch.cuda.synchronize()
    return agents


def request_bytes(agent: Agent, mapping: bool, opts: raster.RenderOptions) -> int:
    """Device bytes one request needs: its workspace (its pairs' share of a
    batch's), its images and upstream images, and its gradients. Raises for a
    job the library rejects."""
    lib = _lib.load()
    b = opts.bin_tile or opts.tile
    cap = raster.default_capacity(agent.n, agent.intr.width, agent.intr.height, b)
    ws = lib.ms_workspace_bytes(agent.n, ref(raster.intr_struct(agent.intr)), ref(raster.opts_struct(opts)), cap)
    if ws == 0:
        check(_lib.MS_ERR_INVALID_ARG)
    px = agent.intr.width * agent.intr.height
    grads = 56 * agent.n + 72 if mapping else 72
    return int(ws + 2 * 5 * 4 * px + grads)


class _Round:
    __slots__ = ("event", "batch", "reqs", "outs", "ups", "grads", "stream")


class _ExecutorBase:
    def __init__(self, agents, opts, w_rgb, w_depth, keep_outputs):
        self.agents = agents
        self.opts = dataclasses.replace(opts, check=False)
        self.w = (float(w_rgb), float(w_depth), 0.0)
        self.keep_outputs = keep_outputs
        self._cost: dict = {}

    def cost(self, r: Request) -> int:
        if not 0 <= r.agent < len(self.agents):
            raise ValueError(f"no agent {r.agent}")
        key = (r.agent, r.mapping)
        if key not in self._cost:
            self._cost[key] = request_bytes(self.agents[r.agent], r.mapping, self.opts)
        return self._cost[key]

    def _pose(self, r: Request):
        a = self.agents[r.agent]
        return a.poses[r.step % a.poses.shape[0]]

    def _loss_grads(self, reqs, outs, stream):
        """L1 gradient of every rendered job against its agent's frame."""
        lib = _lib.load()
        sp = ctypes.c_void_p(stream.cuda_stream)
        ups = []
        for r, (rgb, depth, sil) in zip(reqs, outs):
            a = self.agents[r.agent]
            g = (torch.empty_like(rgb), torch.empty_like(depth), torch.empty_like(sil))
            check(lib.ms_l1_loss_grad(ref(MsImages(rgb.data_ptr(), depth.data_ptr(), sil.data_ptr())),
                                      ref(MsImages(a.target[0].data_ptr(), a.target[1].data_ptr(),
                                                   a.target[2].data_ptr())),
                                      ref(raster.intr_struct(a.intr)), *self.w,
                                      ref(MsImages(g[0].data_ptr(), g[1].data_ptr(), g[2].data_ptr())),
                                      ctypes.c_void_p(0), sp))
            ups.append(g)
        return ups

    def done(self, rnd) -> bool:
        return rnd.event.query()

    def _largest(self, k):
        order = sorted(range(len(self.agents)), key=lambda a: -self.cost(Request(0, a, 0.0, 0, True)))
        return [Request(-1 - i, a, 0.0, 0, True) for i, a in enumerate(order[:k])]


class GpuExecutor(_ExecutorBase):
    """Runs a round as one batched forward (ms_forward_batch), the L1 loss
    gradient of every job and one batched backward (ms_backward_batch) with
    per-job gradient flags, on the next of `streams` default-priority streams.
    Each stream keeps one workspace, grown as needed; rounds on one stream
    run in order, so they share it safely."""

    def __init__(self, agents: list[Agent], opts: raster.RenderOptions = raster.RenderOptions(), streams: int = 2,
                 w_rgb: float = 1.0, w_depth: float = 0.5, keep_outputs: bool = False):
        super().__init__(agents, opts, w_rgb, w_depth, keep_outputs)
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.ws = [None] * streams
        self.next = 0

    def warm(self, max_batch: int = 8):
        """Runs, on every stream, one round of the `max_batch` agents with the
        largest requests, so that the streams' workspaces and cached
        allocations have their largest size before serving starts."""
        reqs = self._largest(max_batch)
        for _ in self.streams:
            self.collect(self.launch(reqs))
        torch.cuda.synchronize()

    def _run(self, rnd, opts):
        with torch.cuda.stream(rnd.stream):
            k = self.streams.index(rnd.stream)
            vms = [self._pose(r) for r in rnd.reqs]
            rnd.batch = raster.BatchJob([self.agents[r.agent].map for r in rnd.reqs], vms,
                                        [self.agents[r.agent].intr for r in rnd.reqs], opts, self.ws[k])
            self.ws[k] = rnd.batch.ws
            rnd.outs = rnd.batch.forward()
            rnd.ups = self._loss_grads(rnd.reqs, rnd.outs, rnd.stream)
            rnd.grads = rnd.batch.backward(rnd.ups, map_grads=[r.mapping for r in rnd.reqs], pose_grads=True)
            rnd.event = torch.cuda.Event()
            rnd.event.record(rnd.stream)

    def launch(self, reqs: list[Request]):
        rnd = _Round()
        rnd.reqs = list(reqs)
        rnd.stream = self.streams[self.next]
        self.next = (self.next + 1) % len(self.streams)
        self._run(rnd, self.opts)
        return rnd

    def collect(self, rnd):
        with torch.cuda.stream(rnd.stream):
            if rnd.batch.stats()["overflow"]:
                # more pairs than the capacity estimate: redo with a checked
                # forward, which grows the capacity, then the backward
                self._run(rnd, dataclasses.replace(self.opts, check=True))
                rnd.event.synchronize()
        out = ([dict(images=o, grads=g, upstream=u) for o, g, u in zip(rnd.outs, rnd.grads, rnd.ups)]
               if self.keep_outputs else None)
        rnd.batch = rnd.outs = rnd.ups = rnd.grads = None
        return out


class PlainExecutor(_ExecutorBase):
    """The sequential baseline: each request on its own through `raster.Job`
    (plain launches of ms_forward, the loss gradient and ms_backward), all on
    one stream in arrival order, with one workspace per agent."""

    def __init__(self, agents: list[Agent], opts: raster.RenderOptions = raster.RenderOptions(),
                 w_rgb: float = 1.0, w_depth: float = 0.5, keep_outputs: bool = False):
        super().__init__(agents, opts, w_rgb, w_depth, keep_outputs)
        self.stream = torch.cuda.Stream()
        self.ws = {}

    def warm(self):
        """Runs one request of every agent, sizing the per-agent workspaces."""
        for r in self._largest(len(self.agents)):
            self.collect(self.launch([r]))
        torch.cuda.synchronize()

    def _run(self, rnd, opts):
        with torch.cuda.stream(rnd.stream):
            rnd.batch, rnd.outs, rnd.grads = [], [], []
            for r in rnd.reqs:
                a = self.agents[r.agent]
                job = raster.Job(a.map, self._pose(r), a.intr, opts, self.ws.get(r.agent))
                self.ws[r.agent] = job.ws
                rnd.batch.append(job)
                rnd.outs.append(job.forward())
            rnd.ups = self._loss_grads(rnd.reqs, rnd.outs, rnd.stream)
            for r, job, g in zip(rnd.reqs, rnd.batch, rnd.ups):
                rnd.grads.append(job.backward(*g, map_grads=r.mapping, pose_grads=True))
            rnd.event = torch.cuda.Event()
            rnd.event.record(rnd.stream)

    def launch(self, reqs: list[Request]):
        rnd = _Round()
        rnd.reqs = list(reqs)
        rnd.stream = self.stream
        self._run(rnd, self.opts)
        return rnd

    def collect(self, rnd):
        with torch.cuda.stream(rnd.stream):
            if any(job.stats()["overflow"] for job in rnd.batch):
                self._run(rnd, dataclasses.replace(self.opts, check=True))
                rnd.event.synchronize()
        out = ([dict(images=o, grads=g, upstream=u) for o, g, u in zip(rnd.outs, rnd.grads, rnd.ups)]
               if self.keep_outputs else None)
        rnd.batch = rnd.outs = rnd.ups = rnd.grads = None
        return out


def requests_from_trace(trace) -> list[Request]:
    """Requests from `scenes.poisson_trace` events (time, agent, step, mapping)."""
    return [Request(i, int(a), float(t), int(k), bool(mp)) for i, (t, a, k, mp) in enumerate(trace)]


def serve(agents, requests, opts=raster.RenderOptions(), budget_bytes: int = 200 << 30, max_batch: int = 8,
          inflight: int = 2, keep_outputs: bool = False, executor: GpuExecutor | None = None):
    """Continuous batching of `requests` over resident `agents`: rounds of up
    to `max_batch` jobs on `inflight` streams under `budget_bytes`. A given
    `executor` (with `inflight` streams) is reused with its workspaces."""
    ex = executor or GpuExecutor(agents, opts, streams=inflight, keep_outputs=keep_outputs)
    sched = Scheduler(max_batch, budget_bytes, len(ex.streams), ex.cost)
    return Server(ex, sched).run(requests)


def serve_plain(agents, requests, opts=raster.RenderOptions(), budget_bytes: int = 200 << 30, inflight: int = 2,
                keep_outputs: bool = False, executor: PlainExecutor | None = None):
    """The sequential FIFO baseline: one plain render + backward per request
    on one stream; up to `inflight` requests are enqueued ahead so the host's
    launch work overlaps the device's."""
    ex = executor or PlainExecutor(agents, opts, keep_outputs=keep_outputs)
    sched = Scheduler(1, budget_bytes, inflight, ex.cost)
    return Server(ex, sched).run(requests)

"""Launch-configuration autotuner for single and batched renders.

Tile edge and per-wave Gaussian batch decide how the compositing work is cut
(workgroups per tile, entries staged per LDS round) and how much the binning
has to sort, and their best values depend on the map sizes and image shapes.
The tuner times every candidate on the actual jobs (forward + backward, HIP
events on the current stream, median of a few repetitions after one
warm-up) and caches the winner under a shape key: the job count, each job's
image size and its Gaussian count rounded to a power of two.
"""
from __future__ import annotations

import dataclasses
import json
import math
import os

import torch

from . import raster

TILES = (8, 16, 32)
WAVE_BATCHES = (32, 64, 128)
SCHEDULES = ("grid", "queue", "xcd_queue")


def shape_key(ns, intrs) -> str:
    parts = [f"{i.width}x{i.height}:{1 << max(0, int(math.ceil(math.log2(max(n, 1)))))}" for n, i in zip(ns, intrs)]
    return f"{len(parts)}|" + ",".join(parts)


@dataclasses.dataclass
class TuneResult:
    options: raster.RenderOptions
    ms: float
    table: dict          # "tile/wave_batch" (grid launches) and "tile/wave_batch/schedule" (the other
                         # compositing schedules at the best tile and batch) -> median ms of one
                         # forward + backward of all jobs


class Autotuner:
    """Chooses RenderOptions (tile, wave_batch, compositing schedule) for a
    set of jobs: every (tile, wave_batch) pair with one workgroup per tile,
    then the persistent tile-queue schedules at the best pair.

    `base` supplies every other option (bin tile, record paths, near plane);
    the bin tile is raised to the tile edge where it is smaller."""

    def __init__(self, base: raster.RenderOptions = raster.RenderOptions(), tiles=TILES,
                 wave_batches=WAVE_BATCHES, reps: int = 3, cache_path: str | None = None, schedules=SCHEDULES):
        self.base = base
        self.candidates = [(t, w) for t in tiles for w in wave_batches]
        self.schedules = [s for s in schedules if s != "grid"]
        self.reps = reps
        self.cache_path = cache_path
        self.cache: dict[str, dict] = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    def _options(self, tile: int, wb: int, schedule: str = "grid") -> raster.RenderOptions:
        bin_tile = self.base.bin_tile if self.base.bin_tile == 0 else max(self.base.bin_tile, tile)
        return dataclasses.replace(self.base, tile=tile, wave_batch=wb, bin_tile=bin_tile, check=True,
                                   schedule=schedule)

    @staticmethod
    def _time(step, reps: int) -> float:
        step()                                  # checked warm-up: grows the pair capacity if needed
        step.unchecked()
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            step()
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        times.sort()
        return times[len(times) // 2]

    def tune_batch(self, maps, viewmats, intrs, upstream) -> TuneResult:
        """Best options for rendering `maps` as one batch (BatchJob)."""
        key = "batch|" + shape_key([m["means"].shape[1] for m in maps], intrs)
        return self._tune(key, lambda o: _BatchStep(maps, viewmats, intrs, upstream, o))

    def tune_plain(self, maps, viewmats, intrs, upstream) -> TuneResult:
        """Best single fixed options for rendering the jobs one after another."""
        key = "plain|" + shape_key([m["means"].shape[1] for m in maps], intrs)
        return self._tune(key, lambda o: _PlainStep(maps, viewmats, intrs, upstream, o))

    def _tune(self, key: str, make) -> TuneResult:
        if key in self.cache:
            c = self.cache[key]
            return TuneResult(self._options(c["tile"], c["wave_batch"], c.get("schedule", "grid")), c["ms"],
                              c["table"])
        table = {}
        best = None

        def trial(tile, wb, schedule, name):
            nonlocal best
            step = make(self._options(tile, wb, schedule))
            ms = self._time(step, self.reps)
            step.release()
            table[name] = round(ms, 4)
            if best is None or ms < best[0]:
                best = (ms, tile, wb, schedule)
            torch.cuda.empty_cache()

        for tile, wb in self.candidates:
            trial(tile, wb, "grid", f"{tile}/{wb}")
        _, tile, wb, _ = best
        for schedule in self.schedules:
            trial(tile, wb, schedule, f"{tile}/{wb}/{schedule}")
        ms, tile, wb, schedule = best
        self.cache[key] = dict(tile=tile, wave_batch=wb, schedule=schedule, ms=ms, table=table)
        if self.cache_path:
            with open(self.cache_path, "w") as f:
                json.dump(self.cache, f, indent=1)
        return TuneResult(self._options(tile, wb, schedule), ms, table)


class _BatchStep:
    def __init__(self, maps, viewmats, intrs, upstream, opts):
        self.batch = raster.BatchJob(maps, viewmats, intrs, opts)
        self.upstream = upstream
        self.outs = None

    def __call__(self):
        self.outs = self.batch.forward(self.outs)
        self.batch.backward(self.upstream)

    def unchecked(self):
        self.batch.opts = dataclasses.replace(self.batch.opts, check=False)

    def release(self):
        self.batch = None


class _PlainStep:
    def __init__(self, maps, viewmats, intrs, upstream, opts):
        self.jobs = [raster.Job(m, vm, i, opts) for m, vm, i in zip(maps, viewmats, intrs)]
        self.upstream = upstream

    def __call__(self):
        for job, up in zip(self.jobs, self.upstream):
            job.forward()
            job.backward(*up)

    def unchecked(self):
        for job in self.jobs:
            job.opts = dataclasses.replace(job.opts, check=False)

    def release(self):
        self.jobs = None

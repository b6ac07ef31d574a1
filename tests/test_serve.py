"""Host logic of the serving loop, driven by a simulated executor on a
virtual clock: admission order, batch and budget limits, rounds in flight,
invalid jobs failing alone, latency bookkeeping, trace reproducibility."""
import collections

import numpy as np
import pytest

from paper_2412_09723_amd import scenes
from paper_2412_09723_amd.serve import Request, Scheduler, Server, requests_from_trace, summarize


class Clock:
    """Virtual time: sleep(0) advances by one polling tick."""

    def __init__(self, tick=1e-5):
        self.t = 0.0
        self.tick = tick

    def now(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, self.tick)


class SimExecutor:
    """A round takes `fixed + per_job * jobs` seconds of virtual time; rounds
    run concurrently (as on separate streams). Requests of agent `bad` make
    the launch raise, as an invalid job does."""

    def __init__(self, clock, fixed=1e-3, per_job=5e-4, bad=None, cost=lambda r: 100, rerun=0.0):
        self.clock, self.fixed, self.per_job, self.bad, self._cost = clock, fixed, per_job, bad, cost
        self.rerun = rerun      # seconds a collect spends redoing the round (a capacity overflow)
        self.launches = []
        self.live = 0
        self.max_live = 0

    def cost(self, r):
        return self._cost(r)

    def launch(self, reqs):
        if self.bad is not None and any(r.agent == self.bad for r in reqs):
            raise RuntimeError("invalid job")
        self.launches.append([r.rid for r in reqs])
        self.live += 1
        self.max_live = max(self.max_live, self.live)
        return dict(end=self.clock.now() + self.fixed + self.per_job * len(reqs), reqs=reqs)

    def done(self, h):
        return self.clock.now() >= h["end"]

    def collect(self, h):
        self.live -= 1
        if self.rerun:
            self.clock.t += self.rerun
        return [dict(rid=r.rid) for r in h["reqs"]]


def _requests(n=200, agents=4, rate=2000.0, seed=0):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    return [Request(i, int(rng.integers(agents)), float(t[i]), i, bool(i % 2)) for i in range(n)]


def _run(reqs, max_batch=8, budget=10_000, inflight=2, **kw):
    clock = Clock()
    ex = SimExecutor(clock, **kw)
    sched = Scheduler(max_batch, budget, inflight, ex.cost)
    done, failed, info = Server(ex, sched, clock=clock.now, sleep=clock.sleep).run(reqs)
    return ex, done, failed, info


def test_every_request_completes_once_in_fifo_order():
    reqs = _requests()
    ex, done, failed, info = _run(reqs)
    assert not failed
    assert sorted(d.rid for d in done) == [r.rid for r in reqs]
    launched = [rid for rnd in ex.launches for rid in rnd]
    order = [r.rid for r in sorted(reqs, key=lambda r: (r.arrival, r.rid))]
    assert launched == order
    for d in done:
        assert d.arrival <= d.launched <= d.finished
        assert d.latency > 0


def test_batch_inflight_and_budget_limits():
    reqs = _requests(n=400, rate=50_000.0)         # arrivals far faster than service: rounds fill up
    ex, done, failed, info = _run(reqs, max_batch=5, budget=1_000, inflight=3, cost=lambda r: 150 + 50 * (r.rid % 3))
    assert not failed and len(done) == len(reqs)
    assert max(len(b) for b in ex.launches) <= 5
    assert ex.max_live <= 3
    assert info["peak_bytes"] <= 1_000
    cost = {r.rid: 150 + 50 * (r.rid % 3) for r in reqs}
    assert all(sum(cost[i] for i in b) <= 1_000 for b in ex.launches)
    assert max(len(b) for b in ex.launches) >= 3     # the loop does batch when work queues up


def test_forced_small_budget_runs_one_job_per_round():
    reqs = _requests(n=60, rate=50_000.0)
    ex, done, failed, info = _run(reqs, max_batch=8, budget=120, inflight=2, cost=lambda r: 100)
    assert len(done) == 60 and not failed
    assert all(len(b) == 1 for b in ex.launches)
    assert ex.max_live == 1                          # a second round would exceed the budget
    assert info["peak_bytes"] <= 120


def test_over_budget_and_invalid_jobs_fail_alone():
    reqs = _requests(n=120, agents=4, rate=20_000.0)
    big = {r.rid for r in reqs if r.rid % 17 == 5}
    ex, done, failed, info = _run(reqs, budget=1_000, bad=3,
                                  cost=lambda r: 5_000 if r.rid in big else 100)
    failed_ids = {r.rid for r, _ in failed}
    expected = big | {r.rid for r in reqs if r.agent == 3}
    assert failed_ids == expected
    assert {d.rid for d in done} == {r.rid for r in reqs} - expected
    reasons = dict((r.rid, why) for r, why in failed)
    assert all("budget" in reasons[i] for i in big)
    assert all("launch failed" in reasons[r.rid] for r in reqs if r.agent == 3 and r.rid not in big)
    # no launched round holds an invalid job
    agent_of = {r.rid: r.agent for r in reqs}
    assert all(agent_of[i] != 3 for b in ex.launches for i in b)


def test_cost_errors_fail_alone():
    reqs = _requests(n=50)

    def cost(r):
        if r.rid == 7:
            raise ValueError("bad intrinsics")
        return 10

    ex, done, failed, info = _run(reqs, cost=cost)
    assert [r.rid for r, _ in failed] == [7] and "bad intrinsics" in failed[0][1]
    assert len(done) == 49


def test_latency_matches_simulated_service_when_idle():
    # arrivals 10 ms apart, service 1.5 ms: every request runs alone at once
    reqs = [Request(i, 0, 0.01 * (i + 1), i, False) for i in range(20)]
    ex, done, failed, info = _run(reqs, fixed=1e-3, per_job=5e-4)
    assert all(len(b) == 1 for b in ex.launches)
    lat = np.array([d.latency for d in done])
    assert np.all(np.abs(lat - 1.5e-3) < 5e-5)
    s = summarize(done, info["wall_s"])
    assert s["jobs"] == 20 and abs(s["p50_ms"] - 1.5) < 0.05 and s["mean_batch"] == 1.0


def test_saturated_loop_batches_more():
    slow = _requests(n=300, rate=500.0)
    fast = _requests(n=300, rate=20_000.0)
    _, d_slow, _, _ = _run(slow)
    _, d_fast, _, _ = _run(fast)
    assert np.mean([d.batch for d in d_fast]) > np.mean([d.batch for d in d_slow])


def test_scheduler_rejects_bad_limits():
    with pytest.raises(ValueError):
        Scheduler(0, 10, 1, lambda r: 1)
    with pytest.raises(ValueError):
        Scheduler(1, 0, 1, lambda r: 1)


def test_poisson_trace_is_reproducible_and_poisson():
    a = scenes.poisson_trace(8, 30.0, 20.0, seed=4)
    b = scenes.poisson_trace(8, 30.0, 20.0, seed=4)
    c = scenes.poisson_trace(8, 30.0, 20.0, seed=5)
    assert a == b and a != c
    ts = np.array([e[0] for e in a])
    assert np.all(np.diff(ts) >= 0) and ts.min() >= 0 and ts.max() < 20.0
    per_agent = collections.Counter(e[1] for e in a)
    # 600 expected arrivals per agent, standard deviation about 24.5
    assert all(abs(per_agent[k] - 600) < 6 * 24.5 for k in range(8))
    frac_mapping = np.mean([e[3] for e in a])
    assert abs(frac_mapping - 0.5) < 0.05
    # step indices count each agent's jobs
    for k in range(8):
        assert [e[2] for e in a if e[1] == k] == list(range(per_agent[k]))
    reqs = requests_from_trace(a)
    assert [r.rid for r in reqs] == list(range(len(a))) and reqs[3].arrival == a[3][0]


def test_latency_includes_a_round_that_collect_reruns():
    """A round whose collect redoes the work (capacity overflow: a checked
    forward and the backward again) finishes when collect returns; the
    latency of its requests includes the re-run."""
    reqs = [Request(0, 0, 0.0, 0, True)]
    _, base, _, _ = _run(reqs)
    _, slow, _, _ = _run(reqs, rerun=5e-3)
    lat = lambda d: d[0].finished - d[0].arrival
    assert lat(slow) >= lat(base) + 5e-3 - 1e-9

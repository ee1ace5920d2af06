"""Scheduler logic of the serving loop, on host-only backends (no GPU)."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_1711_00005_amd.serve import Backend, Scheduler, report


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class TimedBackend(Backend):
    """Cost model: an iteration takes sum(points * steps) / rate seconds."""

    def __init__(self, clock, rate=1e9, fp_per_point=16, fail=()):
        self.clock, self.rate, self.fpp, self.fail = clock, rate, fp_per_point, set(fail)
        self.calls = []
        self.live = 0

    def footprint(self, p):
        return p.points * self.fpp

    def create(self, p):
        self.live += 1
        return {"p": p, "done": 0}

    def march(self, states, nsteps):
        self.calls.append(len(states))
        self.clock.t += sum(s["p"].points * n for s, n in zip(states, nsteps)) / self.rate
        for s, n in zip(states, nsteps):
            s["done"] += n

    def finish(self, s, rid):
        return {"finite": rid not in self.fail, "steps": s["done"]}

    def destroy(self, s):
        self.live -= 1


class AsyncBackend(Backend):
    """Marches take effect only once waited for, in enqueue order (device
    work behind an event); finishing a request before its last march has
    been waited for is an error."""

    def __init__(self, clock=None, rate=1e6):
        self.clock, self.rate = clock, rate
        self.queue = []      # (token, [(state, n), ...])
        self.tok = 0
        self.live = 0

    def footprint(self, p):
        return p.points * 16

    def create(self, p):
        self.live += 1
        return {"p": p, "done": 0, "queued": 0}

    def march(self, states, nsteps):
        self.tok += 1
        self.queue.append((self.tok, list(zip(states, nsteps))))
        for s, n in zip(states, nsteps):
            s["queued"] += n
        return self.tok

    def wait(self, token):
        while self.queue and self.queue[0][0] <= token:
            _, work = self.queue.pop(0)
            for s, n in work:
                s["done"] += n
                if self.clock is not None:
                    self.clock.t += s["p"].points * n / self.rate

    def finish(self, s, rid):
        assert s["done"] == s["queued"], f"request {rid} finished with a march still in flight"
        return {"finite": True, "steps": s["done"]}

    def destroy(self, s):
        assert s["done"] == s["queued"]
        self.live -= 1


def small_trace(n=12, seed=1):
    env = W.wedge_env(zmax=600.0)
    rng = np.random.default_rng(seed)
    out, t = [], 0.0
    for i in range(n):
        t += float(rng.exponential(0.01))
        nz = int(rng.choice([16, 24, 40]))
        nth = int(rng.choice([3, 5, 8]))
        width = W.TWO_PI if rng.uniform() < 0.5 else math.radians(60.0)
        g = W.Grid(nz=nz, ntheta=nth, theta0=float(rng.uniform(0, 6)), width=width, dr=10.0,
                   precision=W.PREC_C128)
        steps = int(rng.integers(3, 30))
        out.append(W.Request(i, t, W.Problem(env, g, float(rng.uniform(20, 60)), 50.0, steps, f"r{i}")))
    return out


def test_every_request_advances_exactly_its_steps():
    clk = VirtualClock()
    be = TimedBackend(clk)
    recs = Scheduler(be, budget_bytes=10**9, chunk_steps=7, clock=clk, sleep=clk.sleep).run(small_trace())
    for r in recs:
        assert r.status == "done" and r.summary["steps"] == r.steps
    assert be.live == 0


def test_admission_respects_the_budget_and_is_continuous():
    clk = VirtualClock()
    tr = small_trace(20, seed=3)
    fp = [r.problem.points * 16 for r in tr]
    budget = 3 * max(fp)
    be = TimedBackend(clk, rate=2e4)
    sch = Scheduler(be, budget_bytes=budget, chunk_steps=2, clock=clk, sleep=clk.sleep)
    recs = sch.run(tr)
    assert sch.max_used <= budget
    assert all(r.status == "done" for r in recs)
    # continuous batching: some request was admitted while an earlier one was still running
    overlap = any(a.admitted < b.done and a.admitted > b.admitted
                  for a in recs for b in recs if a.rid != b.rid)
    assert overlap
    assert max(be.calls) > 1
    # FIFO admission
    adm = [r.admitted for r in sorted(recs, key=lambda r: r.arrival)]
    assert adm == sorted(adm)


def test_oversized_request_is_rejected_and_failures_are_flagged():
    clk = VirtualClock()
    tr = small_trace(8, seed=4)
    big = max(tr, key=lambda r: r.problem.points)
    budget = big.problem.points * 16 - 1
    be = TimedBackend(clk, fail={tr[0].rid if tr[0].rid != big.rid else tr[1].rid})
    recs = Scheduler(be, budget_bytes=budget, chunk_steps=5, clock=clk, sleep=clk.sleep).run(tr)
    st = {r.rid: r.status for r in recs}
    assert st[big.rid] == "rejected"
    assert sum(s == "failed" for s in st.values()) == 1
    rep = report(recs)
    assert rep["rejected"] == 1 and rep["failed"] == 1 and rep["done"] == len(tr) - 2


def test_backlog_chunk_applies_only_while_requests_wait():
    """With the budget full, iterations advance backlog_chunk_steps; once
    nothing waits, chunk_steps again; every request still advances exactly
    its own steps."""
    clk = VirtualClock()
    be = TimedBackend(clk, rate=2e3)
    tr = small_trace(20, seed=3)
    budget = 3 * max(r.problem.points for r in tr) * 16
    sch = Scheduler(be, budget, 3, clock=clk, sleep=clk.sleep, backlog_chunk_steps=9)
    steps_seen = []
    march = be.march

    def spy(states, nsteps):
        steps_seen.append(max(nsteps))
        march(states, nsteps)
    be.march = spy
    recs = sch.run(tr)
    assert all(r.status == "done" for r in recs)
    assert all(r.summary["steps"] == r.steps for r in recs)
    assert sch.backlog_iterations > 0 and max(steps_seen) == 9
    assert 0 < sch.backlog_iterations < sch.iterations
    with pytest.raises(ValueError):
        Scheduler(be, budget, 5, backlog_chunk_steps=4)
    plain = Scheduler(TimedBackend(VirtualClock()), budget, 3)
    assert plain.Kb == plain.K == 3


def test_latency_percentiles():
    clk = VirtualClock()
    recs = Scheduler(TimedBackend(clk, rate=1e5), 10**9, 4, clock=clk, sleep=clk.sleep).run(small_trace(30, 5))
    rep = report(recs)
    lat = sorted(r.latency for r in recs)
    assert rep["p50_latency_s"] == pytest.approx(np.percentile(lat, 50))
    assert rep["p99_latency_s"] == pytest.approx(np.percentile(lat, 99))
    assert all(r.latency >= 0 for r in recs)


class OracleBackend(Backend):
    """Host backend running the complex128 oracle (tests only)."""

    def __init__(self):
        self.out = {}

    def footprint(self, p):
        return p.points * 32

    def create(self, p):
        st = O.setup(p.env, p.grid, p.f_hz)
        return {"st": st, "u": O.starter(st, p.zs), "j": 0}

    def march(self, states, nsteps):
        for s, n in zip(states, nsteps):
            s["u"] = O.march(s["st"], s["u"], s["j"], n)
            s["j"] += n

    def finish(self, s, rid):
        self.out[rid] = s["u"]
        return {"finite": bool(np.isfinite(s["u"]).all())}

    def destroy(self, s):
        pass


def test_served_results_equal_the_plain_march():
    tr = small_trace(10, seed=7)
    be = OracleBackend()
    clk = VirtualClock()
    Scheduler(be, 10**9, chunk_steps=4, clock=clk, sleep=clk.sleep).run(tr)
    for r in tr:
        p = r.problem
        st = O.setup(p.env, p.grid, p.f_hz)
        assert np.array_equal(be.out[r.rid], O.march(st, O.starter(st, p.zs), 0, p.nsteps))


def test_pipelined_loop_finishes_a_request_only_after_its_last_march():
    """The loop enqueues iteration k+1 before waiting for k: a request whose
    last iteration is k+1 must not be finished when k completes."""
    for seed in (1, 3, 5):
        clk = VirtualClock()
        be = AsyncBackend(clk, rate=3e4)
        tr = small_trace(25, seed=seed)
        sch = Scheduler(be, budget_bytes=4 * max(r.problem.points for r in tr) * 16, chunk_steps=3,
                        clock=clk, sleep=clk.sleep, backlog_chunk_steps=6)
        recs = sch.run(tr)
        assert all(r.status == "done" and r.summary["steps"] == r.steps for r in recs)
        assert be.live == 0 and not be.queue

"""Continuous-batching request loop for PE range marches.

The paper distributes the frequencies of a wide-band run over MPI ranks
(Sec. 3.2.3); a served stream is the on-line version of that decomposition:
march requests (one frequency, one sector or the full circle, one maximum
range) arrive over time and are advanced together on one GPU.

Scheduling, per iteration:
  1. requests whose arrival time has passed join the waiting queue (a request
     whose device footprint exceeds the whole budget is rejected);
  2. waiting requests are admitted in arrival order while their device
     footprint (coefficient tables, scratch field and the field itself) fits
     in the HBM budget - admission happens between iterations, so requests
     arriving while others run join the resident set (continuous batching);
  3. every resident request advances by min(K, steps left) range steps in one
     batched march (one launch per pass per step over all of
     them, pe3d_march_batch); while the device runs it, newly arrived
     requests are admitted and set up (they join the next iteration);
  4. the loop runs one iteration ahead: iteration k+1 is enqueued behind
     iteration k before the host waits for k (its event only, not the
     device), so the device does not idle while the host turns over; the
     requests whose last iteration was k are then checked (non-finite field
     -> failed) on a stream of their own, summarised, and released (their
     device memory goes back to the library's pool without waiting for the
     device).

The backend does the device work; `Pe3dBackend` drives libpe3d, tests use
host-only backends.  Latency of a request = completion time - arrival time.
"""
from __future__ import annotations

import json
import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclass
class Record:
    rid: int
    arrival: float
    points: int
    steps: int
    footprint: int
    admitted: Optional[float] = None
    done: Optional[float] = None
    status: str = "queued"          # queued | running | done | rejected | failed
    summary: Optional[dict] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


class Backend:
    """Device work of the scheduler (interface)."""

    def footprint(self, problem) -> int:
        raise NotImplementedError

    def create(self, problem):
        raise NotImplementedError

    def march(self, states: Sequence, nsteps: Sequence[int]):
        """Advance the states; may return before the device has finished.
        Returns a token for wait() (host-only backends: None)."""
        raise NotImplementedError

    def wait(self, token) -> None:
        """Block until the march that returned `token` has finished
        (host-only backends: no-op)."""

    def finish(self, state, rid: int) -> dict:
        """Summary of a finished request; must report {'finite': bool, ...}."""
        raise NotImplementedError

    def destroy(self, state) -> None:
        raise NotImplementedError


class Pe3dBackend(Backend):
    """libpe3d backend: one handle and one device field per resident request,
    all residents advanced by one pe3d_march_batch call per iteration."""

    def __init__(self, keep_fields: Sequence[int] = (), use_graph: bool = False):
        import torch  # (device memory and streams only)
        from . import pe3d as P
        self.P = P
        self.keep = set(keep_fields)
        self.use_graph = use_graph
        self.kept: Dict[int, np.ndarray] = {}
        # finished fields are checked on a stream of their own (default
        # priority), so that the check does not wait behind the next iteration
        self.side = torch.cuda.Stream()

    def footprint(self, problem) -> int:
        g = problem.grid
        esz = 16 if getattr(g, "precision", 0) == self.P.PE3D_C128 else 8
        return self.P.pe3d_footprint(problem.env, g, problem.f_hz) + g.nz * g.ntheta * esz

    def create(self, problem):
        m = self.P.Pe3d(problem.env, problem.grid, problem.f_hz)
        u = m.starter(problem.zs)
        return (m, u)

    def march(self, states, nsteps):
        import torch
        ms = [s[0] for s in states]
        us = [s[1] for s in states]
        self.P.march_batch(ms, list(nsteps), us, use_graph=self.use_graph)
        ev = torch.cuda.Event()
        ev.record()
        return ev

    def wait(self, token) -> None:
        if token is not None:
            token.synchronize()

    def finish(self, state, rid: int = -1) -> dict:
        """After wait() on the request's last march: its field is final."""
        import torch
        m, u = state
        with torch.cuda.stream(self.side):
            # one transfer for both checks (waits for this stream only)
            chk = torch.stack((torch.isfinite(torch.view_as_real(u)).all().double(),
                               torch.linalg.vector_norm(u).double())).cpu()
            if rid in self.keep:
                self.kept[rid] = u.detach().cpu().numpy()
        finite, nrm = bool(chk[0].item()), float(chk[1].item())
        return {"finite": finite, "norm": nrm, "step": m.step, "range_m": m.range_m}

    def destroy(self, state) -> None:
        state[0].close()


class Scheduler:
    def __init__(self, backend: Backend, budget_bytes: int, chunk_steps: int = 40,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep, log: Optional[Callable] = None,
                 backlog_chunk_steps: Optional[int] = None):
        """backlog_chunk_steps: steps per iteration while requests wait for
        admission (the budget is full), so that an overloaded loop pays its
        per-iteration cost less often; None keeps chunk_steps throughout."""
        if budget_bytes <= 0 or chunk_steps <= 0:
            raise ValueError("budget and chunk size must be positive")
        if backlog_chunk_steps is not None and backlog_chunk_steps < chunk_steps:
            raise ValueError("the backlog chunk must be at least the chunk")
        self.backend = backend
        self.budget = int(budget_bytes)
        self.K = int(chunk_steps)
        self.Kb = int(backlog_chunk_steps) if backlog_chunk_steps is not None else self.K
        self.backlog_iterations = 0
        self.clock = clock
        self.sleep = sleep
        self.log = log
        self.iterations = 0
        self.max_resident = 0
        self.max_used = 0

    def run(self, requests) -> List[Record]:
        """Serve `requests` (objects with rid, arrival_s, problem) in arrival order."""
        reqs = sorted(requests, key=lambda r: r.arrival_s)
        recs = {r.rid: Record(r.rid, r.arrival_s, r.problem.points, r.problem.nsteps, 0) for r in reqs}
        probs = {r.rid: r.problem for r in reqs}
        pending = deque(reqs)
        waiting: deque = deque()
        resident: List[list] = []   # [rid, state, steps_left, footprint]
        used = 0
        t0 = self.clock()

        def admit():
            nonlocal used
            now = self.clock() - t0
            while pending and pending[0].arrival_s <= now:
                r = pending.popleft()
                rec = recs[r.rid]
                rec.footprint = int(self.backend.footprint(r.problem))
                if rec.footprint > self.budget:
                    rec.status = "rejected"
                    rec.done = now
                else:
                    waiting.append(r)
            while waiting and used + recs[waiting[0].rid].footprint <= self.budget:
                r = waiting.popleft()
                rec = recs[r.rid]
                state = self.backend.create(r.problem)
                used += rec.footprint
                rec.admitted = self.clock() - t0
                rec.status = "running"
                resident.append([r.rid, state, probs[r.rid].nsteps, rec.footprint])
            self.max_used = max(self.max_used, used)
            self.max_resident = max(self.max_resident, len(resident))

        # the iteration on the device: (token, its entries); an entry's steps
        # left already exclude every enqueued iteration
        inflight = None
        while pending or waiting or resident:
            admit()
            nxt = [x for x in resident if x[2] > 0]
            enqueued = None
            if nxt:
                # enqueued behind the iteration in flight, before waiting for it
                K = self.Kb if waiting else self.K
                self.backlog_iterations += K != self.K
                steps = [min(K, x[2]) for x in nxt]
                token = self.backend.march([x[1] for x in nxt], steps)
                self.iterations += 1
                for x, s in zip(nxt, steps):
                    x[2] -= s
                enqueued = (token, nxt)
                # while the device works: admit and set up new arrivals
                admit()
            if inflight is None:
                if enqueued is None and pending:
                    wait = pending[0].arrival_s - (self.clock() - t0)
                    if wait > 0:
                        self.sleep(wait)
                inflight = enqueued
                continue
            self.backend.wait(inflight[0])
            now = self.clock() - t0
            # requests whose last iteration was the one just finished (not
            # those that also run in the iteration enqueued behind it)
            later = {id(x) for x in enqueued[1]} if enqueued else set()
            done_ids = {id(x) for x in inflight[1] if x[2] == 0 and id(x) not in later}
            keep = []
            for x in resident:
                if id(x) not in done_ids:
                    keep.append(x)
                    continue
                rec = recs[x[0]]
                try:
                    summ = self.backend.finish(x[1], x[0])
                finally:
                    self.backend.destroy(x[1])
                used -= x[3]
                rec.summary = summ
                rec.done = now
                rec.status = "done" if summ.get("finite", True) else "failed"
            resident = keep
            inflight = enqueued
            if self.log and self.iterations % 50 == 0:
                self.log(f"iter {self.iterations} t={now:.2f}s resident={len(resident)} "
                         f"waiting={len(waiting)} pending={len(pending)}")
        return [recs[r.rid] for r in reqs]


def report(records: Sequence[Record], makespan: Optional[float] = None) -> dict:
    """p50/p99 latency and throughput of a served run."""
    done = [r for r in records if r.status == "done"]
    lat = np.array([r.latency for r in done]) if done else np.zeros(0)
    if makespan is None:
        makespan = max((r.done for r in records if r.done is not None), default=0.0)
    work = float(sum(r.points * r.steps for r in done))
    arr = [r.arrival for r in records]
    span = (max(arr) - min(arr)) if len(arr) > 1 else 0.0
    offered = float(sum(r.points * r.steps for r in records)) / span if span > 0 else None
    return {
        "requests": len(records),
        "done": len(done),
        "rejected": sum(r.status == "rejected" for r in records),
        "failed": sum(r.status == "failed" for r in records),
        "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
        "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
        "mean_latency_s": float(lat.mean()) if lat.size else None,
        "makespan_s": makespan,
        "throughput_pt_steps_per_s": work / makespan if makespan else None,
        "offered_pt_steps_per_s": offered,
    }


def main(argv=None):
    import argparse
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads as W
    ap = argparse.ArgumentParser(description="serve a Poisson stream of PE march requests")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--budget-gib", type=float, default=1.0)
    ap.add_argument("--chunk", type=int, default=40)
    ap.add_argument("--backlog-chunk", type=int, default=100,
                    help="steps per iteration while requests wait for admission")
    ap.add_argument("--range-scale", type=float, default=1.0,
                    help="multiply every request's range (and step count) by this factor")
    a = ap.parse_args(argv)
    trace = W.config5_trace(n=a.requests, rate_hz=a.rate, seed=a.seed)
    if a.range_scale != 1.0:
        trace = [W.Request(r.rid, r.arrival_s,
                           W.Problem(r.problem.env, r.problem.grid, r.problem.f_hz, r.problem.zs,
                                     max(1, int(math.ceil(r.problem.nsteps * a.range_scale))),
                                     r.problem.name)) for r in trace]
    sch = Scheduler(Pe3dBackend(), int(a.budget_gib * 2**30), a.chunk,
                    log=lambda s: print("[serve]", s, file=sys.stderr, flush=True),
                    backlog_chunk_steps=a.backlog_chunk)
    t0 = time.perf_counter()
    recs = sch.run(trace)
    out = report(recs, time.perf_counter() - t0)
    out.update(iterations=sch.iterations, max_resident=sch.max_resident,
               max_used_bytes=sch.max_used, budget_bytes=sch.budget, chunk_steps=sch.K,
               backlog_chunk_steps=sch.Kb, backlog_iterations=sch.backlog_iterations,
               rate_hz=a.rate, range_scale=a.range_scale)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

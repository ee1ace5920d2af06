"""Per-shape choice of the kernels' lanes and azimuth solver by measurement.

The library picks the lanes per depth column (depth pass) and per depth line
(azimuth pass) by a fixed rule (the fewest lanes whose chunks stay within
the kernels' limits), and solves the azimuth systems by chunked recurrences
joined by a wavefront scan unless the grid asks for cyclic reduction.
`tune` times the alternatives for one problem shape alone on the GPU, each
pass separately (the depth pass does not depend on the azimuth lanes and
vice versa), with the library's own per-launch event timing, and returns the
fastest of each.  `tune_batch_azimuth` chooses the azimuth solver per class
of problems (same Ntheta and azimuth boundary) inside batched launches, where
a problem shares the GPU with the others; `keep_if_faster` then times the
whole batch in the library's batch schedule with the chosen solvers and with
the default ones and keeps the faster (a class that wins alone can lengthen
the schedule's launch tails in the mix).  Lanes and solver change only how
the same systems are solved, so a tuned march agrees with the default one to
rounding.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Tuple

from . import pe3d as P


def _pass_ms(stats, prefix: str) -> float:
    tot = sum(s["total_ms"] for s in stats if s["name"].startswith(prefix))
    n = sum(s["launches"] for s in stats if s["name"].startswith(prefix))
    return tot / max(n, 1)


def _time(env, grid, f_hz: float, steps: int, reps: int) -> Tuple[float, float]:
    import torch
    m = P.Pe3d(env, grid, f_hz)
    try:
        u = m.starter(env.zmax / 3.0)
        m.march(2, u)  # first use of the kernels
        torch.cuda.synchronize()
        best_a = best_b = float("inf")
        for _ in range(reps):
            P.pe3d_profile_read()
            P.pe3d_profile_enable(True)
            try:
                m.march(steps, u)
                torch.cuda.synchronize()
                stats = P.pe3d_profile_read()
            finally:
                P.pe3d_profile_enable(False)
            best_a = min(best_a, _pass_ms(stats, "pass_a"))
            best_b = min(best_b, _pass_ms(stats, "pass_b"))
        return best_a, best_b
    finally:
        m.close()


def candidates(grid) -> Tuple[list, list]:
    """Lanes the kernels accept for this shape: depth lanes from the rule's
    choice up to 256, azimuth lanes from the rule's choice up to 64."""
    L = 4
    while True:
        M = (grid.nz + 1 + L - 2) // (L - 1)
        M += M % 2 == 0
        if max(M, 3) <= 17 or L > 256:
            break
        L *= 2
    W = 1
    while (grid.ntheta + W - 1) // W > 16:
        W *= 2
    la = [x for x in (4, 8, 16, 32, 64, 128, 256) if x >= L]
    lb = [x for x in (1, 2, 4, 8, 16, 32, 64) if x >= W]
    return la, lb


def tune(env, grid, f_hz: float, steps: int = 6, reps: int = 2) -> Tuple[object, Dict]:
    """The grid with the fastest depth and azimuth lanes for this problem
    shape, and the timings (ms per launch) of every candidate."""
    la, lb = candidates(grid)
    ta = {L: _time(env, dataclasses.replace(grid, depth_lanes=L, azimuth_lanes=lb[0]), f_hz, steps, reps)[0]
          for L in la}
    # an N x 2D march has no azimuth pass: its lanes keep the rule's choice
    # (and its depth pass over a fixed medium is one launch per call, timed
    # as a whole: the same steps for every candidate)
    tb = {} if getattr(grid, "mode", 0) == P.PE3D_MODE_NX2D else {
        W: _time(env, dataclasses.replace(grid, depth_lanes=la[0], azimuth_lanes=W), f_hz, steps, reps)[1]
        for W in lb}
    best = dataclasses.replace(grid, depth_lanes=min(ta, key=ta.get),
                               azimuth_lanes=min(tb, key=tb.get) if tb else 0)
    return best, {"depth_lanes_ms": ta, "azimuth_lanes_ms": tb}


def _batch_pass_b_ms(problems, steps: int, start: int, reps: int) -> float:
    """Best whole-batch azimuth-pass launch time (ms) of the problems marched
    together from step `start` (one chain, one group: one launch per pass)."""
    import torch
    ms = [P.Pe3d(p.env, p.grid, p.f_hz) for p in problems]
    try:
        us = [m.starter(p.zs) for m, p in zip(ms, problems)]
        if start:
            for m in ms:
                m.set_step(start)
        P.set_batch_schedule(1, 0)
        P.march_batch(ms, 1, us, use_graph=False)  # first step of a call and first use
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            P.pe3d_profile_read()
            P.pe3d_profile_enable(True)
            try:
                P.march_batch(ms, steps, us, use_graph=False)
                torch.cuda.synchronize()
                stats = P.pe3d_profile_read()
            finally:
                P.pe3d_profile_enable(False)
            best = min(best, _pass_ms(stats, "pass_b"))
        return best
    finally:
        P.set_batch_schedule(2, 112 << 20)
        for m in ms:
            m.close()


def tune_batch_azimuth(problems, steps: int = 6, far: int = 0, reps: int = 2):
    """Azimuth solver per class of problems (same Ntheta and boundary) by
    measurement inside a batch: the class's problems marched together with
    each solver near the source (from step 1, where the azimuth coupling is
    strong and cyclic reduction needs the most levels) and from step `far`
    (default: half the problems' steps), the solver with the smaller sum
    chosen.  Returns the problems with the chosen solver in their grids and a
    report {class: {solver: [near_ms, far_ms]}, ...}."""
    import dataclasses as dc
    far = far or max(1, min(p.nsteps for p in problems) // 2)
    classes = {}
    for i, p in enumerate(problems):
        periodic = p.grid.width >= 2 * 3.141592653589793 * (1 - 1e-12)
        classes.setdefault((p.grid.ntheta, periodic), []).append(i)
    out = list(problems)
    report = {}
    for (nt, periodic), idx in sorted(classes.items()):
        times = {}
        for solver in (P.PE3D_AZIMUTH_CHUNKED, P.PE3D_AZIMUTH_PCR):
            ps = [dc.replace(problems[i], grid=dc.replace(problems[i].grid, azimuth_solver=solver,
                                                         azimuth_lanes=0)) for i in idx]
            times[solver] = [_batch_pass_b_ms(ps, steps, 0, reps), _batch_pass_b_ms(ps, steps, far, reps)]
        best = min(times, key=lambda k: sum(times[k]))
        for i in idx:
            out[i] = dc.replace(problems[i], grid=dc.replace(problems[i].grid, azimuth_solver=best))
        key = f"ntheta {nt} {'periodic' if periodic else 'sector'} ({len(idx)} problems)"
        report[key] = {"chunked_ms": [round(t, 4) for t in times[P.PE3D_AZIMUTH_CHUNKED]],
                       "pcr_ms": [round(t, 4) for t in times[P.PE3D_AZIMUTH_PCR]],
                       "chosen": "pcr" if best == P.PE3D_AZIMUTH_PCR else "chunked"}
    return out, {"near_steps_from": 1, "far_steps_from": far, "classes": report}


def _batch_ms_per_step(problems, steps: int, reps: int) -> float:
    """Best ms per batch step of the problems marched together in the
    library's current batch schedule, calls of `steps` steps replayed from a
    captured graph (events around the calls)."""
    import torch
    ms = [P.Pe3d(p.env, p.grid, p.f_hz) for p in problems]
    try:
        us = [m.starter(p.zs) for m, p in zip(ms, problems)]
        P.prepare_batch(ms, steps, us)
        P.march_batch(ms, steps, us)  # first replay
        torch.cuda.synchronize()
        best = float("inf")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(reps):
            e0.record()
            P.march_batch(ms, steps, us)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) / steps)
        return best
    finally:
        for m in ms:
            m.close()


def keep_if_faster(default, tuned, steps: int = 20, reps: int = 3):
    """The tuned problems if the whole batch marches faster with them than
    with the default solvers (same schedule, same calls), else the default
    ones; and a report {default_ms_per_step, tuned_ms_per_step, kept}.  The
    two sets are timed alternately."""
    changed = any(a.grid != b.grid for a, b in zip(default, tuned))
    if not changed:
        return tuned, {"kept": "tuned", "note": "the choice equals the default"}
    td, tt = float("inf"), float("inf")
    for _ in range(2):
        td = min(td, _batch_ms_per_step(default, steps, reps))
        tt = min(tt, _batch_ms_per_step(tuned, steps, reps))
    kept = "tuned" if tt < td else "default"
    return (tuned if kept == "tuned" else default), {
        "default_ms_per_step": round(td, 4), "tuned_ms_per_step": round(tt, 4), "kept": kept,
        "how": f"whole batch, library batch schedule, calls of {steps} steps replayed from a graph, "
               f"best of {2 * reps} per set, sets alternated"}

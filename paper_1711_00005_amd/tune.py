"""Per-shape choice of the kernels' lanes by measurement.

The library picks the lanes per depth column (depth pass) and per depth line
(azimuth pass) by a fixed rule (the fewest lanes whose chunks stay within
the kernels' limits).  `tune` times the alternatives for one problem shape on
the GPU, each pass separately (the depth pass does not depend on the azimuth
lanes and vice versa), with the library's own per-launch event timing, and
returns the fastest of each.  The lanes change only the split of the same
recurrences over lanes, so a tuned march agrees with the default one to
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

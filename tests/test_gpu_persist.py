"""The persistent batched march (one kernel per call walking a task list,
pe3d_set_batch_kernel) against the launch-per-pass batched march, bit for
bit: both run the same pass bodies on the same values, so every field and
step counter must agree exactly.  Also: a batch with range rows falls back to
the launches, and a wait limit of zero ends the kernel early with the
timeouts reported (the kernel's bounded waits, forced from the host)."""
import dataclasses
import math
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a ROCm GPU"
    return _t


@pytest.fixture(scope="module")
def P(torch):
    import paper_1711_00005_amd.pe3d as _P
    yield _P
    _P.set_batch_kernel(_P.PE3D_BATCH_LAUNCHES)
    _P.set_batch_schedule()


def to_dev(torch, u, prec):
    dt = torch.complex128 if prec == W.PREC_C128 else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(u)).to(device="cuda", dtype=dt).contiguous()


def problems(prec):
    """Shapes that reach every pass body of the persistent kernel: several
    depth-lane counts, chunked azimuth classes (exact and general), a sector,
    cyclic reduction, an N x 2D problem, and 0 steps."""
    env = W.wedge_env()
    specs = [
        dict(nz=200, ntheta=24, theta0=0.0, width=W.TWO_PI, dr=10.0),
        dict(nz=1100, ntheta=40, theta0=0.5, width=W.TWO_PI, dr=5.0),
        dict(nz=64, ntheta=9, theta0=1.0, width=math.radians(30.0), dr=12.0),
        dict(nz=333, ntheta=300, theta0=2.0, width=W.TWO_PI, dr=8.0),
        dict(nz=130, ntheta=64, theta0=0.0, width=W.TWO_PI, dr=6.0, azimuth_solver=W.AZ_PCR),
        dict(nz=90, ntheta=33, theta0=0.2, width=math.radians(90.0), dr=5.0, mode=W.MODE_NX2D),
        dict(nz=700, ntheta=1024, theta0=0.0, width=W.TWO_PI, dr=10.0),
        dict(nz=50, ntheta=16, theta0=0.0, width=W.TWO_PI, dr=10.0),
    ]
    fs = [40.0, 90.0, 25.0, 60.0, 45.0, 70.0, 30.0, 20.0]
    steps = [5, 3, 7, 4, 6, 5, 2, 0]
    out = []
    for s, f, n in zip(specs, fs, steps):
        g = W.Grid(precision=prec, **s)
        out.append((env, g, f, n))
    return out


def fields(torch, probs, prec, seed):
    us = []
    for i, (env, grid, f, n) in enumerate(probs):
        st = O.setup(env, grid, f)
        u0 = O.starter(st, 0.3 * env.zmax) + 0.1 * W.random_field(grid.ntheta, grid.nz, seed + i)
        us.append(to_dev(torch, u0, prec))
    return us


def run(torch, P, probs, u0s, kind, use_graph, calls):
    P.set_batch_kernel(kind)
    ms = [P.Pe3d(env, grid, f) for env, grid, f, n in probs]
    us = [u.clone() for u in u0s]
    steps = [n for *_, n in probs]
    for _ in range(calls):
        P.march_batch(ms, steps, us, use_graph=use_graph)
    torch.cuda.synchronize()
    js = [m.step for m in ms]
    for m in ms:
        m.close()
    P.set_batch_kernel(P.PE3D_BATCH_LAUNCHES)
    return us, js


@pytest.mark.parametrize("prec", [W.PREC_C64, W.PREC_C128])
@pytest.mark.parametrize("use_graph", [False, True])
@pytest.mark.parametrize("chains", [1, 2])
def test_persistent_equals_launches(torch, P, prec, use_graph, chains):
    probs = problems(prec)
    u0s = fields(torch, probs, prec, 700)
    say("persistent vs launches", prec, "graph" if use_graph else "direct", "chains", chains)
    P.set_batch_schedule(chains, 112 << 20)
    try:
        # two calls: the second replays the captured graph (use_graph) and
        # starts from the first call's fields and step counters
        ref, jr = run(torch, P, probs, u0s, P.PE3D_BATCH_LAUNCHES, use_graph, 2)
        got, jg = run(torch, P, probs, u0s, P.PE3D_BATCH_PERSISTENT, use_graph, 2)
    finally:
        P.set_batch_schedule()
    assert jg == jr == [2 * n for *_, n in probs]
    for i, (a, b) in enumerate(zip(ref, got)):
        assert torch.equal(a, b), f"problem {i}"
    assert P.pe3d_batch_wait_timeouts() == 0


def test_persistent_small_groups_and_profile(torch, P):
    """A schedule of many groups per chain (16 KiB of field per group) for
    the launches, which the persistent kernel replaces by one group per
    chain; the profiled call records one persistent launch with the call's
    algorithmic bytes."""
    prec = W.PREC_C64
    probs = problems(prec)
    u0s = fields(torch, probs, prec, 900)
    P.set_batch_schedule(2, 16 << 10)
    try:
        ref, _ = run(torch, P, probs, u0s, P.PE3D_BATCH_LAUNCHES, False, 1)
        P.pe3d_profile_read()
        P.pe3d_profile_enable(True)
        try:
            got, _ = run(torch, P, probs, u0s, P.PE3D_BATCH_PERSISTENT, False, 1)
            stats = P.pe3d_profile_read()
        finally:
            P.pe3d_profile_enable(False)
    finally:
        P.set_batch_schedule()
    for i, (a, b) in enumerate(zip(ref, got)):
        assert torch.equal(a, b), f"problem {i}"
    names = {s["name"]: s for s in stats}
    assert set(names) == {"persist<c64,batch>"}, names
    s = names["persist<c64,batch>"]
    assert s["launches"] == 1
    expect = sum(n * (2.0 if g.mode == W.MODE_NX2D else 4.0) * 8.0 * g.nz * g.ntheta
                 for env, g, f, n in probs)
    assert s["algo_bytes"] == pytest.approx(expect)


def test_persistent_config4_equals_launches(torch, P):
    """The 64-frequency batch at full size, 2 steps, graph replay."""
    probs = W.config4_problems(nsteps=2, precision=W.PREC_C64)
    say("persistent config4")
    outs = []
    for kind in (P.PE3D_BATCH_LAUNCHES, P.PE3D_BATCH_PERSISTENT):
        P.set_batch_kernel(kind)
        ms = [P.Pe3d(p.env, p.grid, p.f_hz) for p in probs]
        us = [m.starter(p.zs) for m, p in zip(ms, probs)]
        P.march_batch(ms, 2, us, use_graph=True)
        torch.cuda.synchronize()
        outs.append(us)
        for m in ms:
            m.close()
    P.set_batch_kernel(P.PE3D_BATCH_LAUNCHES)
    for i, (a, b) in enumerate(zip(*outs)):
        assert torch.equal(a, b), f"problem {i}"
    assert P.pe3d_batch_wait_timeouts() == 0


def test_batch_with_range_rows_uses_the_launches(torch, P):
    """A range-dependent problem in the batch: the call runs the launches
    (the medium changes per step), with the same results."""
    prec = W.PREC_C64
    probs = problems(prec)[:3]
    env_r = W.random_ssp_range_env(52, nr=4, row_dr=15.0)
    probs.append((env_r, W.Grid(nz=45, ntheta=7, theta0=1.0, width=1.0, dr=4.0, precision=prec), 50.0, 6))
    u0s = fields(torch, probs, prec, 800)
    ref, jr = run(torch, P, probs, u0s, P.PE3D_BATCH_LAUNCHES, False, 1)
    P.pe3d_profile_read()
    P.pe3d_profile_enable(True)
    try:
        got, jg = run(torch, P, probs, u0s, P.PE3D_BATCH_PERSISTENT, False, 1)
        stats = P.pe3d_profile_read()
    finally:
        P.pe3d_profile_enable(False)
    assert jr == jg
    for i, (a, b) in enumerate(zip(ref, got)):
        assert torch.equal(a, b), f"problem {i}"
    assert not any(s["name"].startswith("persist") for s in stats)


def test_wait_limit_zero_ends_the_kernel_and_is_reported(torch, P):
    """With a wait limit of zero the first task that has to wait gives up,
    raises the abort flag and every workgroup leaves: the call returns, the
    timeouts are counted, and the next calls with the default limit are
    exact again."""
    prec = W.PREC_C64
    env = W.wedge_env()
    grid = W.Grid(nz=1500, ntheta=256, theta0=0.0, width=W.TWO_PI, dr=10.0, precision=prec)
    probs = [(env, grid, 50.0, 4)]
    u0s = fields(torch, probs, prec, 1000)
    assert P.pe3d_batch_wait_timeouts() == 0
    say("persistent wait limit 0")
    P.set_batch_kernel(P.PE3D_BATCH_PERSISTENT, 0.0)
    try:
        ms = [P.Pe3d(env, grid, 50.0)]
        us = [u0s[0].clone()]
        P.march_batch(ms, [4], us, use_graph=False)
        torch.cuda.synchronize()
        ms[0].close()
    finally:
        P.set_batch_kernel(P.PE3D_BATCH_LAUNCHES)
    assert P.pe3d_batch_wait_timeouts() >= 1
    assert P.pe3d_batch_wait_timeouts() == 0  # reset by the read
    ref, _ = run(torch, P, probs, u0s, P.PE3D_BATCH_LAUNCHES, False, 1)
    got, _ = run(torch, P, probs, u0s, P.PE3D_BATCH_PERSISTENT, False, 1)
    assert torch.equal(ref[0], got[0])
    assert P.pe3d_batch_wait_timeouts() == 0

"""Parity of the HIP march (through the C ABI) with the complex128 oracle.

Tolerances (relative L2 over the whole field, reading A18/A19): complex128
mode <= 1e-12, complex64 mode <= 1e-5, both against the oracle on identical
seeded inputs.  Integer-valued state (the step counter) and the batched vs
plain and graph vs direct paths are compared bit for bit.
"""
import dataclasses
import math
import os
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.modal import modal_march

pytestmark = pytest.mark.gpu

TOL = {W.PREC_C128: 1e-12, W.PREC_C64: 1e-5}


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
    return _P


def to_dev(torch, u, prec):
    dt = torch.complex128 if prec == W.PREC_C128 else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(u)).to(device="cuda", dtype=dt).contiguous()


def to_host(torch, u):
    torch.cuda.synchronize()
    return u.detach().cpu().numpy().astype(np.complex128)


def run_pair(torch, P, env, grid, f, u0, nsteps, name):
    st = O.setup(env, grid, f)
    ref = O.march(st, u0, 0, nsteps)
    say(name, f"nz={grid.nz} nth={grid.ntheta} prec={grid.precision} steps={nsteps}")
    m = P.Pe3d(env, grid, f)
    u = to_dev(torch, u0, grid.precision)
    m.march(nsteps, u)
    got = to_host(torch, u)
    assert m.step == nsteps
    m.close()
    return got, ref


# ---------------------------------------------------------------- starter
@pytest.mark.parametrize("prec", [W.PREC_C128, W.PREC_C64])
def test_starter_matches_oracle(torch, P, prec):
    env = W.wedge_env()
    grid = W.Grid(nz=300, ntheta=7, theta0=0.0, width=W.TWO_PI, dr=10.0, precision=prec)
    st = O.setup(env, grid, 100.0)
    say("starter", prec)
    m = P.Pe3d(env, grid, 100.0)
    u = m.starter(100.0)
    got = to_host(torch, u)
    assert O.rel_l2(got, O.starter(st, 100.0)) < (1e-14 if prec == W.PREC_C128 else 1e-7)
    m.close()


# ---------------------------------------------------------------- config 1
def test_config1_fp64_matches_oracle_and_closed_form(torch, P):
    p = W.config1()
    st = O.setup(p.env, p.grid, p.f_hz)
    th = st.theta[:, None]
    u0 = O.starter(st, p.zs) * (1 + 0.5 * np.cos(th))
    got, ref = run_pair(torch, P, p.env, p.grid, p.f_hz, u0, p.nsteps, "config1")
    assert O.rel_l2(got, ref) < 1e-12
    cf = modal_march(st, u0, p.nsteps, p.env.floor)
    assert O.rel_l2(got, cf) < 1e-12


def test_config1_gpu_starter(torch, P):
    p = W.config1()
    st = O.setup(p.env, p.grid, p.f_hz)
    say("config1 gpu starter")
    m = P.Pe3d(p.env, p.grid, p.f_hz)
    u = m.starter(p.zs)
    m.march(p.nsteps, u)
    got = to_host(torch, u)
    ref = O.march(st, O.starter(st, p.zs), 0, p.nsteps)
    assert O.rel_l2(got, ref) < 1e-12
    m.close()


# ---------------------------------------------------------------- small cases
CASES = [
    # name, env, grid kwargs, f, steps
    ("wedge", W.wedge_env(), dict(nz=70, ntheta=12, theta0=0.0, width=W.TWO_PI, dr=10.0), 30.0, 6),
    ("wedge_rigid", W.wedge_env(floor=W.FLOOR_RIGID),
     dict(nz=130, ntheta=9, theta0=0.2, width=W.TWO_PI, dr=10.0), 20.0, 5),
    ("sector", W.random_env(3), dict(nz=45, ntheta=7, theta0=1.0, width=math.radians(60.0), dr=5.0), 50.0, 5),
    ("sector_1az", W.random_env(4), dict(nz=33, ntheta=1, theta0=0.5, width=math.radians(30.0), dr=5.0), 40.0, 4),
    ("min_periodic", W.random_env(5), dict(nz=2, ntheta=3, theta0=0.0, width=W.TWO_PI, dr=5.0), 60.0, 3),
    ("nth5_r0", W.random_env(6), dict(nz=17, ntheta=5, theta0=0.0, width=W.TWO_PI, dr=5.0, r0=250.0), 60.0, 4),
    ("nth33", W.wedge_env(zmax=500.0, d_max=300.0, d_min=50.0),
     dict(nz=100, ntheta=33, theta0=0.0, width=W.TWO_PI, dr=8.0), 40.0, 5),
    ("no_water", W.flat_layered_env(depth=3.0), dict(nz=40, ntheta=5, theta0=0.0, width=W.TWO_PI, dr=5.0), 40.0, 4),
    ("all_water", W.isovelocity_env(c=1510.0, atten=0.1), dict(nz=64, ntheta=8, theta0=0.0, width=W.TWO_PI, dr=5.0), 25.0, 5),
    ("multi_tile", W.wedge_env(), dict(nz=300, ntheta=70, theta0=0.3, width=W.TWO_PI, dr=10.0), 60.0, 4),
    ("sector_90", W.wedge_env(zmax=2400.0), dict(nz=192, ntheta=64, theta0=2.0, width=math.radians(90.0), dr=10.0), 50.0, 4),
]


def _seed(name):
    return sum(map(ord, name)) % 1000


@pytest.mark.parametrize("prec", [W.PREC_C128, W.PREC_C64])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_small_case_matches_oracle(torch, P, case, prec):
    """A field that is smooth in azimuth (a starter with a random azimuthal
    modulation of low order), as the march produces: the strict bars."""
    name, env, gk, f, steps = case
    grid = W.Grid(precision=prec, **gk)
    st = O.setup(env, grid, f)
    rng = np.random.default_rng(_seed(name))
    th = st.theta[:, None]
    mod = 1 + 0.3 * np.cos(th + rng.uniform(0, 6)) + 0.2j * np.sin(2 * th)
    u0 = O.starter(st, 0.3 * env.zmax) * mod + 0.05 * W.random_field(1, grid.nz, _seed(name))
    got, ref = run_pair(torch, P, env, grid, f, u0, steps, name)
    assert O.rel_l2(got, ref) < TOL[prec], name


@pytest.mark.parametrize("prec", [W.PREC_C128, W.PREC_C64])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_small_case_rough_field(torch, P, case, prec):
    """White-noise field (every azimuth and depth mode excited) at the same
    strict bars.  Highest azimuth modes leave the azimuth solve 1 + 4 sigma_j
    times smaller than they enter it (sigma_0 = 204 on sector_90), so a solve
    that formed u as a difference of two terms of the size of v would lose
    that many digits here."""
    name, env, gk, f, steps = case
    grid = W.Grid(precision=prec, **gk)
    u0 = W.random_field(grid.ntheta, grid.nz, seed=_seed(name))
    got, ref = run_pair(torch, P, env, grid, f, u0, steps, name + "_rough")
    assert O.rel_l2(got, ref) < TOL[prec], name


def worst_sector_request():
    """The config-5 request (served stream, seed 0) whose first azimuth step
    has the largest sigma_0 among the sectors: 30 degrees, 367 Hz,
    Nz = 2368, Ntheta = 64, dr = 4.09 m, sigma_0 = 613."""
    best = None
    for rq in W.config5_trace():
        p = rq.problem
        if p.grid.width >= W.TWO_PI - 1e-9:
            continue
        st = O.setup(p.env, p.grid, p.f_hz)
        sg = abs(st.s(0))
        if best is None or sg > best[0]:
            best = (sg, p)
    return best[1]


@pytest.mark.parametrize("prec", [W.PREC_C64, W.PREC_C128])
def test_config5_worst_sector_request(torch, P, prec):
    """The served stream's sector with the largest azimuth coefficient, at
    its full grid, from the GPU starter (the zero edge azimuths put edge
    structure into the field from step 1), 20 steps, whole field."""
    p = worst_sector_request()
    grid = dataclasses.replace(p.grid, precision=prec)
    st = O.setup(p.env, grid, p.f_hz)
    assert abs(st.s(0)) > 600.0 and grid.ntheta == 64
    say("config5 worst sector", p.name, f"nz={grid.nz} nth={grid.ntheta} prec={prec}")
    m = P.Pe3d(p.env, grid, p.f_hz)
    u = m.starter(p.zs)
    u0 = to_host(torch, u)
    m.march(20, u)
    got = to_host(torch, u)
    m.close()
    ref = O.march(st, u0, 0, 20)
    assert O.rel_l2(got, ref) < TOL[prec]


# ---------------------------------------------------------------- azimuth solver: cyclic reduction
@pytest.mark.parametrize("rough", [False, True])
@pytest.mark.parametrize("prec", [W.PREC_C128, W.PREC_C64])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_pcr_azimuth_solver_matches_oracle(torch, P, case, prec, rough):
    """The azimuth pass by parallel cyclic reduction (periodic lines and
    sectors through their odd extension), smooth and white-noise fields, at
    the strict bars."""
    name, env, gk, f, steps = case
    grid = W.Grid(precision=prec, azimuth_solver=W.AZ_PCR, **gk)
    st = O.setup(env, grid, f)
    if rough:
        u0 = W.random_field(grid.ntheta, grid.nz, seed=_seed(name))
    else:
        u0 = O.starter(st, 0.3 * env.zmax) * (1 + 0.4 * np.cos(st.theta) + 0.2 * np.sin(3 * st.theta))[:, None]
    got, ref = run_pair(torch, P, env, grid, f, u0, steps, name + "_pcr")
    assert O.rel_l2(got, ref) < TOL[prec], name


@pytest.mark.parametrize("prec", [W.PREC_C64, W.PREC_C128])
def test_pcr_config5_worst_sector_request(torch, P, prec):
    """Cyclic reduction on the served stream's sector with sigma_0 = 613."""
    p = worst_sector_request()
    grid = dataclasses.replace(p.grid, precision=prec, azimuth_solver=W.AZ_PCR)
    st = O.setup(p.env, grid, p.f_hz)
    say("config5 worst sector, pcr", p.name, f"nz={grid.nz} nth={grid.ntheta} prec={prec}")
    m = P.Pe3d(p.env, grid, p.f_hz)
    u = m.starter(p.zs)
    u0 = to_host(torch, u)
    m.march(20, u)
    got = to_host(torch, u)
    m.close()
    assert O.rel_l2(got, O.march(st, u0, 0, 20)) < TOL[prec]


@pytest.mark.parametrize("prec", [W.PREC_C64, W.PREC_C128])
def test_pcr_size_limits_and_batch(torch, P, prec):
    """Cyclic reduction at the largest Ntheta (2 depths per tile) and a
    ragged depth count, alone against the oracle, then batched together with
    chunked problems: every field equals its plain march bit for bit."""
    env = W.wedge_env()
    specs = [
        dict(nz=20, ntheta=1024, theta0=0.0, width=W.TWO_PI, dr=10.0, azimuth_solver=W.AZ_PCR),
        dict(nz=333, ntheta=300, theta0=2.0, width=W.TWO_PI, dr=8.0, azimuth_solver=W.AZ_PCR),
        dict(nz=64, ntheta=9, theta0=1.0, width=math.radians(30.0), dr=12.0, azimuth_solver=W.AZ_PCR),
        dict(nz=200, ntheta=24, theta0=0.0, width=W.TWO_PI, dr=10.0),
    ]
    fs = [50.0, 60.0, 25.0, 40.0]
    steps = [3, 4, 6, 5]
    probs = [(W.Grid(precision=prec, **g), f) for g, f in zip(specs, fs)]
    fields0, plain = [], []
    for (grid, f), n in zip(probs, steps):
        st = O.setup(env, grid, f)
        u0 = (O.starter(st, 0.3 * env.zmax) * (1 + 0.3 * np.cos(2 * st.theta))[:, None]
              + 0.05 * W.random_field(grid.ntheta, grid.nz, grid.nz))
        fields0.append(u0)
        say("pcr alone", grid.nz, grid.ntheta, prec)
        got, ref = run_pair(torch, P, env, grid, f, u0, n, "pcr_alone")
        assert O.rel_l2(got, ref) < TOL[prec]
        m = P.Pe3d(env, grid, f)
        u = to_dev(torch, u0, prec)
        m.march(n, u)
        torch.cuda.synchronize()
        plain.append(u)
        m.close()
    for use_graph in (False, True):
        ms = [P.Pe3d(env, grid, f) for grid, f in probs]
        us = [to_dev(torch, u0, prec) for u0 in fields0]
        P.march_batch(ms, steps, us, use_graph=use_graph)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(plain, us)):
            assert torch.equal(a, b), f"problem {i} graph={use_graph}"
        for m in ms:
            m.close()


# ---------------------------------------------------------------- size limits
LIMITS = [
    ("max_nz_c64", W.PREC_C64, dict(nz=4096, ntheta=4, theta0=0.0, width=W.TWO_PI, dr=10.0), 100.0),
    ("max_nz_c128", W.PREC_C128, dict(nz=2048, ntheta=4, theta0=0.0, width=W.TWO_PI, dr=10.0), 100.0),
    ("max_nth_c64", W.PREC_C64, dict(nz=20, ntheta=1024, theta0=0.0, width=W.TWO_PI, dr=10.0), 50.0),
    ("max_nth_c128", W.PREC_C128, dict(nz=20, ntheta=1024, theta0=0.0, width=W.TWO_PI, dr=10.0), 50.0),
    ("ragged_c64", W.PREC_C64, dict(nz=1999, ntheta=777, theta0=0.1, width=W.TWO_PI, dr=10.0), 100.0),
    ("max_nz_c128_4096", W.PREC_C128, dict(nz=4096, ntheta=4, theta0=0.0, width=W.TWO_PI, dr=10.0), 100.0),
]


@pytest.mark.parametrize("case", LIMITS, ids=[c[0] for c in LIMITS])
def test_size_limits_match_oracle(torch, P, case):
    name, prec, gk, f = case
    grid = W.Grid(precision=prec, **gk)
    env = W.wedge_env()
    st = O.setup(env, grid, f)
    u0 = O.starter(st, 100.0) * (1 + 0.3 * np.cos(2 * st.theta))[:, None]
    got, ref = run_pair(torch, P, env, grid, f, u0, 3, name)
    assert O.rel_l2(got, ref) < TOL[prec], name


# Depth-pass shapes whose complex64 bodies keep multipliers in LDS between the
# sweeps (chunks of M = 15 and 17 rows) at every lane count the rule gives for
# them, under a wedge whose interface row moves over many chunk offsets from
# column to column (so that every lane role, idle lanes included, occurs).
CHUNKS = [
    # name, nz (lanes L, rows per lane M)
    ("L16_M15", 224), ("L16_M17", 254), ("L32_M15", 448), ("L32_M17", 512),
    ("L64_M15", 944), ("L64_M17", 1070), ("L128_M15", 1904), ("L128_M17", 2158),
    ("L256_M15", 3824), ("L256_M17", 4096),
]


@pytest.mark.parametrize("prec", [W.PREC_C64, W.PREC_C128])
@pytest.mark.parametrize("case", CHUNKS, ids=[c[0] for c in CHUNKS])
def test_depth_chunk_shapes_match_oracle(torch, P, case, prec):
    name, nz = case
    env = W.wedge_env()
    grid = W.Grid(nz=nz, ntheta=48, theta0=0.1, width=W.TWO_PI, dr=10.0, precision=prec)
    m = P.Pe3d(env, grid, 80.0)
    info = m.info()
    m.close()
    assert (info.pass_a_lanes, info.pass_a_chunk) == tuple(int(x) for x in name[1:].split("_M")), name
    st = O.setup(env, grid, 80.0)
    u0 = O.starter(st, 100.0) * (1 + 0.3 * np.cos(st.theta))[:, None] + 0.05 * W.random_field(48, nz, nz)
    got, ref = run_pair(torch, P, env, grid, 80.0, u0, 3, name)
    assert np.isfinite(got).all(), name
    assert O.rel_l2(got, ref) < TOL[prec], name


# ---------------------------------------------------------------- state and batching
@pytest.mark.parametrize("prec", [W.PREC_C64, W.PREC_C128])
@pytest.mark.parametrize("lanes", [(0, 0), (64, 0), (256, 0), (0, 32), (0, 64), (128, 64)])
def test_kernel_lanes_overrides_match_oracle(torch, P, prec, lanes):
    """Every kernel shape the sizes allow gives the oracle's field (the lanes
    only split the same recurrences differently)."""
    env = W.wedge_env()
    grid = W.Grid(nz=300, ntheta=70, theta0=0.3, width=W.TWO_PI, dr=10.0, precision=prec,
                  depth_lanes=lanes[0], azimuth_lanes=lanes[1])
    st = O.setup(env, grid, 60.0)
    u0 = O.starter(st, 100.0) * (1 + 0.2 * np.cos(st.theta))[:, None]
    say("kernel lanes", lanes, prec)
    m = P.Pe3d(env, grid, 60.0)
    if lanes[0]:
        assert m.info().pass_a_lanes == lanes[0]
    u = to_dev(torch, u0, prec)
    m.march(4, u)
    torch.cuda.synchronize()
    assert O.rel_l2(to_host(torch, u), O.march(st, u0, 0, 4)) < TOL[prec]
    m.close()


def test_tune_returns_a_shape_that_matches_oracle(torch, P):
    from paper_1711_00005_amd import tune as T
    env = W.wedge_env()
    grid = W.Grid(nz=700, ntheta=384, theta0=0.0, width=W.TWO_PI, dr=10.0)
    say("tune")
    best, tim = T.tune(env, grid, 80.0, steps=3, reps=1)
    la, lb = T.candidates(grid)
    assert best.depth_lanes in la and best.azimuth_lanes in lb
    assert set(tim["depth_lanes_ms"]) == set(la) and set(tim["azimuth_lanes_ms"]) == set(lb)
    st = O.setup(env, best, 80.0)
    u0 = O.starter(st, 100.0)
    m = P.Pe3d(env, best, 80.0)
    u = to_dev(torch, u0, W.PREC_C64)
    m.march(3, u)
    torch.cuda.synchronize()
    assert O.rel_l2(to_host(torch, u), O.march(st, u0, 0, 3)) < TOL[W.PREC_C64]
    m.close()


def test_tune_batch_azimuth_chooses_per_class_by_measurement(torch, P):
    """The in-batch choice of the azimuth solver: one entry per (Ntheta,
    boundary) class with both solvers timed near the source and further out,
    the problems returned with the faster solver, and a march with the
    chosen solvers matches the oracle."""
    from paper_1711_00005_amd import tune as T
    env = W.wedge_env()
    probs = [W.Problem(env, W.Grid(nz=200, ntheta=nt, theta0=0.0, width=w, dr=10.0), 40.0, 100.0, 30, f"p{i}")
             for i, (nt, w) in enumerate([(24, W.TWO_PI), (24, W.TWO_PI), (64, W.TWO_PI), (32, 1.0)])]
    say("tune batch azimuth")
    out, rep = T.tune_batch_azimuth(probs, steps=3, far=20, reps=1)
    assert len(rep["classes"]) == 3
    for c in rep["classes"].values():
        assert all(t > 0 for t in c["chunked_ms"] + c["pcr_ms"]) and c["chosen"] in ("chunked", "pcr")
        # the report rounds each time to 1e-4 ms and the tuner compares the
        # unrounded sums: the chosen solver's rounded sum exceeds the other's
        # by at most the rounding of the four times
        other = "pcr" if c["chosen"] == "chunked" else "chunked"
        assert sum(c[c["chosen"] + "_ms"]) <= sum(c[other + "_ms"]) + 2e-4, c
    assert out[0].grid.azimuth_solver == out[1].grid.azimuth_solver
    p = out[3]
    st = O.setup(p.env, p.grid, p.f_hz)
    u0 = O.starter(st, p.zs)
    got, ref = run_pair(torch, P, p.env, p.grid, p.f_hz, u0, 5, "tuned sector")
    assert O.rel_l2(got, ref) < TOL[p.grid.precision]


def test_keep_if_faster_times_the_whole_batch(torch, P):
    """The whole-batch check of the in-batch solver choice: both sets timed in
    the batch schedule, the faster kept and reported; an unchanged choice is
    kept without timing."""
    from paper_1711_00005_amd import tune as T
    env = W.wedge_env()
    base = [W.Problem(env, W.Grid(nz=200, ntheta=nt, theta0=0.0, width=W.TWO_PI, dr=10.0), 40.0, 100.0, 30, f"p{i}")
            for i, nt in enumerate([24, 64, 64])]
    tuned = [dataclasses.replace(p, grid=dataclasses.replace(p.grid, azimuth_solver=W.AZ_PCR))
             if p.grid.ntheta == 64 else p for p in base]
    say("keep if faster")
    out, rep = T.keep_if_faster(base, tuned, steps=5, reps=1)
    assert rep["kept"] in ("tuned", "default")
    assert rep["default_ms_per_step"] > 0 and rep["tuned_ms_per_step"] > 0
    assert out is (tuned if rep["kept"] == "tuned" else base)
    assert (rep["tuned_ms_per_step"] < rep["default_ms_per_step"]) == (rep["kept"] == "tuned")
    same, rep2 = T.keep_if_faster(base, list(base))
    assert rep2["kept"] == "tuned" and "note" in rep2 and same == base


def test_tune_nx2d_times_the_depth_pass_only(torch, P):
    """The tuner of an N x 2D shape searches the depth lanes only (there is
    no azimuth pass) and its choice matches the oracle."""
    from paper_1711_00005_amd import tune as T
    env = W.wedge_env()
    grid = W.Grid(nz=700, ntheta=96, theta0=0.0, width=W.TWO_PI, dr=10.0, mode=W.MODE_NX2D)
    say("tune nx2d")
    best, tim = T.tune(env, grid, 80.0, steps=4, reps=1)
    la, _ = T.candidates(grid)
    assert best.depth_lanes in la and best.azimuth_lanes == 0 and best.mode == W.MODE_NX2D
    assert set(tim["depth_lanes_ms"]) == set(la) and tim["azimuth_lanes_ms"] == {}
    assert all(v > 0 for v in tim["depth_lanes_ms"].values())
    st = O.setup(env, best, 80.0)
    u0 = O.starter(st, 100.0)
    m = P.Pe3d(env, best, 80.0)
    u = to_dev(torch, u0, W.PREC_C64)
    m.march(4, u)
    torch.cuda.synchronize()
    assert O.rel_l2(to_host(torch, u), O.march(st, u0, 0, 4)) < TOL[W.PREC_C64]
    m.close()


def test_resume_is_bitwise(torch, P):
    env = W.wedge_env()
    grid = W.Grid(nz=200, ntheta=24, theta0=0.0, width=W.TWO_PI, dr=10.0)
    st = O.setup(env, grid, 50.0)
    u0 = to_dev(torch, O.starter(st, 100.0), W.PREC_C64)
    say("resume")
    a = P.Pe3d(env, grid, 50.0)
    ua = u0.clone()
    a.march(10, ua)
    b = P.Pe3d(env, grid, 50.0)
    ub = u0.clone()
    b.march(4, ub)
    b.march(6, ub)
    torch.cuda.synchronize()
    assert torch.equal(ua, ub)
    # set_step: a fresh handle at step 4 continues the first march exactly
    c = P.Pe3d(env, grid, 50.0)
    uc = u0.clone()
    c.march(4, uc)
    d = P.Pe3d(env, grid, 50.0)
    d.set_step(4)
    d.march(6, uc)
    torch.cuda.synchronize()
    assert torch.equal(ua, uc)
    assert d.step == 10
    for m in (a, b, c, d):
        m.close()


def _batch_problems(prec):
    env = W.wedge_env()
    specs = [
        dict(nz=200, ntheta=24, theta0=0.0, width=W.TWO_PI, dr=10.0),
        dict(nz=1100, ntheta=40, theta0=0.5, width=W.TWO_PI, dr=5.0),
        dict(nz=64, ntheta=9, theta0=1.0, width=math.radians(30.0), dr=12.0),
        dict(nz=333, ntheta=300, theta0=2.0, width=W.TWO_PI, dr=8.0),
    ]
    if prec == W.PREC_C64:
        specs.append(dict(nz=2500, ntheta=20, theta0=0.0, width=W.TWO_PI, dr=10.0))
    fs = [40.0, 90.0, 25.0, 60.0, 120.0]
    return [(env, W.Grid(precision=prec, **s), fs[i]) for i, s in enumerate(specs)]


@pytest.mark.parametrize("prec", [W.PREC_C64, W.PREC_C128])
@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_is_bitwise_equal_to_plain(torch, P, prec, use_graph):
    probs = _batch_problems(prec)
    steps = [5, 3, 7, 0, 4][:len(probs)]
    fields0 = []
    for env, grid, f in probs:
        st = O.setup(env, grid, f)
        fields0.append(to_dev(torch, O.starter(st, 60.0) * (1 + 0.2 * np.sin(st.theta))[:, None], prec))
    say("batch vs plain", prec, use_graph)
    plain = []
    for (env, grid, f), u0, n in zip(probs, fields0, steps):
        m = P.Pe3d(env, grid, f)
        u = u0.clone()
        m.march(n, u)
        plain.append(u)
        m.close()
    ms = [P.Pe3d(env, grid, f) for env, grid, f in probs]
    us = [u0.clone() for u0 in fields0]
    P.march_batch(ms, steps, us, use_graph=use_graph)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(plain, us)):
        assert torch.equal(a, b), f"problem {i}"
    assert [m.step for m in ms] == steps
    for m in ms:
        m.close()


# ---------------------------------------------------------------- N x 2D mode
NX2D = [c for c in CASES if c[0] in ("wedge", "sector", "sector_1az", "min_periodic", "multi_tile", "sector_90")]


@pytest.mark.parametrize("prec", [W.PREC_C128, W.PREC_C64])
@pytest.mark.parametrize("case", NX2D, ids=[c[0] for c in NX2D])
def test_nx2d_matches_oracle(torch, P, case, prec):
    """N x 2D mode (Y = 0): depth pass only.  A one-step call (the depth pass
    reads and writes the caller's field in place), then the rest."""
    name, env, gk, f, steps = case
    grid = W.Grid(precision=prec, mode=W.MODE_NX2D, **gk)
    st = O.setup(env, grid, f)
    u0 = O.starter(st, 0.3 * env.zmax) + 0.3 * W.random_field(grid.ntheta, grid.nz, _seed(name))
    say("nx2d", name, prec)
    m = P.Pe3d(env, grid, f)
    assert m.info().mode == W.MODE_NX2D
    u = to_dev(torch, u0, prec)
    m.march(1, u)
    m.march(steps - 1, u)
    torch.cuda.synchronize()
    ref = O.march(st, u0, 0, steps)
    assert O.rel_l2(to_host(torch, u), ref) < TOL[prec], name
    m.close()


@pytest.mark.parametrize("prec", [W.PREC_C64, W.PREC_C128])
def test_batch_mixing_nx2d_and_3d(torch, P, prec):
    """A batch holding both modes equals the plain marches bit for bit, and its
    N x 2D problems match the oracle."""
    probs = _batch_problems(prec)
    modes = [W.MODE_NX2D, W.MODE_3D, W.MODE_NX2D, W.MODE_3D, W.MODE_NX2D][:len(probs)]
    probs = [(env, dataclasses.replace(g, mode=md), f) for (env, g, f), md in zip(probs, modes)]
    steps = [6, 3, 1, 4, 5][:len(probs)]
    u0s = []
    for env, grid, f in probs:
        st = O.setup(env, grid, f)
        u0s.append(O.starter(st, 60.0) * (1 + 0.2 * np.sin(st.theta))[:, None])
    say("batch nx2d/3d", prec)
    plain = []
    for (env, grid, f), u0, n in zip(probs, u0s, steps):
        m = P.Pe3d(env, grid, f)
        u = to_dev(torch, u0, prec)
        m.march(n, u)
        plain.append(u)
        m.close()
    for use_graph in (False, True):
        ms = [P.Pe3d(env, grid, f) for env, grid, f in probs]
        us = [to_dev(torch, u0, prec) for u0 in u0s]
        P.march_batch(ms, steps, us, use_graph=use_graph)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(plain, us)):
            assert torch.equal(a, b), f"problem {i} graph={use_graph}"
        for m in ms:
            m.close()
    for i, ((env, grid, f), u0, n) in enumerate(zip(probs, u0s, steps)):
        if grid.mode == W.MODE_NX2D:
            ref = O.march(O.setup(env, grid, f), u0, 0, n)
            assert O.rel_l2(to_host(torch, plain[i]), ref) < TOL[prec], f"problem {i}"


# ---------------------------------------------------------------- range-dependent depth
def _tie_env():
    """Rigid floor with dz = 5 m exactly (nz = 60, zmax = 300) and depth rows
    on whole multiples of dz at r = 40, 65, 90 m: with dr = 5 m the steps
    reach the rows exactly and the water-node decisions there are ties."""
    base = W.random_env(32, zmax=300.0, floor=W.FLOOR_RIGID, nbathy=4)
    rows = 5.0 * np.array([[10, 20, 30, 40], [11, 25, 7, 59], [3, 60, 33, 12]], dtype=float)
    return dataclasses.replace(base, bathy_theta=(-3.0, -1.0, 0.5, 2.0), bathy_depth=tuple(rows.ravel()),
                               bathy_nr=3, bathy_r0=40.0, bathy_dr=25.0)


RANGE = [
    # name, env, grid kwargs, f, steps of the successive calls
    ("rd_periodic", W.random_range_env(41, nr=6, row_dr=20.0),
     dict(nz=60, ntheta=12, theta0=0.0, width=W.TWO_PI, dr=5.0), 40.0, (3, 14)),
    ("rd_sector_r0", W.random_range_env(42, nr=5, row_dr=15.0, r0=30.0, floor=W.FLOOR_RIGID),
     dict(nz=45, ntheta=7, theta0=1.0, width=1.0, dr=4.0, r0=22.0), 50.0, (1, 8, 12)),
    ("rd_ties", _tie_env(), dict(nz=60, ntheta=16, theta0=0.0, width=W.TWO_PI, dr=5.0), 40.0, (9, 11)),
    ("rd_multi_tile", W.random_range_env(43, zmax=600.0, nr=8, row_dr=25.0),
     dict(nz=300, ntheta=70, theta0=0.3, width=W.TWO_PI, dr=10.0), 60.0, (4, 5)),
    ("rd_slope", W.slope_env(rmax=2000.0), dict(nz=256, ntheta=64, theta0=0.0, width=W.TWO_PI, dr=25.0), 30.0,
     (10, 10)),
]


@pytest.mark.parametrize("mode", [W.MODE_3D, W.MODE_NX2D])
@pytest.mark.parametrize("prec", [W.PREC_C128, W.PREC_C64])
@pytest.mark.parametrize("case", RANGE, ids=[c[0] for c in RANGE])
def test_range_dependent_depth_matches_oracle(torch, P, case, prec, mode):
    """Depth D(r, theta) with range rows: every step uses the medium at
    r_{j+1}; the march is split over several calls."""
    name, env, gk, f, calls = case
    grid = W.Grid(precision=prec, mode=mode, **gk)
    st = O.setup(env, grid, f)
    th = st.theta[:, None]
    u0 = O.starter(st, 0.3 * env.zmax) * (1 + 0.3 * np.cos(th)) + 0.05 * W.random_field(1, grid.nz, _seed(name))
    say("range-dependent", name, prec, mode)
    m = P.Pe3d(env, grid, f)
    u = to_dev(torch, u0, prec)
    for n in calls:
        m.march(n, u)
    torch.cuda.synchronize()
    ref = O.march(st, u0, 0, sum(calls))
    assert O.rel_l2(to_host(torch, u), ref) < TOL[prec], name
    m.close()


@pytest.mark.parametrize("prec", [W.PREC_C64, W.PREC_C128])
def test_config4_batch_matches_oracle_on_samples(torch, P, prec):
    """The 64-frequency batch at full size (107,589,632 points) in the launch
    configuration bench.py times (one batched call replaying the graphs of
    the default schedule): 2 steps, then the smallest, two middle and the
    largest problems against the oracle over their whole fields."""
    probs = W.config4_problems(nsteps=2, precision=prec)
    say("config4 batch, 64 problems", prec)
    ms = [P.Pe3d(p.env, p.grid, p.f_hz) for p in probs]
    us = [m.starter(p.zs) for m, p in zip(ms, probs)]
    P.march_batch(ms, 2, us, use_graph=True)
    torch.cuda.synchronize()
    # every field finite (a NaN anywhere would also reach the sampled norms)
    assert all(bool(torch.isfinite(torch.view_as_real(u)).all()) for u in us)
    for i in (0, 21, 42, 63):
        p = probs[i]
        st = O.setup(p.env, p.grid, p.f_hz)
        ref = O.march(st, O.starter(st, p.zs), 0, 2)
        err = O.rel_l2(to_host(torch, us[i]), ref)
        say("config4 problem", i, p.grid.nz, p.grid.ntheta, err)
        assert err < TOL[prec], (i, err)
    for m in ms:
        m.close()


# ---------------------------------------------------------------- range-dependent water
WATER = [
    # name, env, grid kwargs, f, steps of the successive calls
    ("wr_periodic", W.random_ssp_range_env(51, nr=5, row_dr=20.0),
     dict(nz=60, ntheta=12, theta0=0.0, width=W.TWO_PI, dr=5.0), 40.0, (3, 14)),
    ("wr_sector_r0", W.random_ssp_range_env(52, nr=4, row_dr=15.0, r0=30.0, floor=W.FLOOR_RIGID),
     dict(nz=45, ntheta=7, theta0=1.0, width=1.0, dr=4.0, r0=22.0), 50.0, (1, 8, 12)),
    ("wr_with_depth_rows", W.random_ssp_range_env(53, nr=6, row_dr=12.0, depth_rows=5),
     dict(nz=70, ntheta=16, theta0=0.0, width=W.TWO_PI, dr=4.0), 45.0, (7, 10)),
    ("wr_multi_tile", W.random_ssp_range_env(54, zmax=600.0, nr=4, row_dr=30.0),
     dict(nz=300, ntheta=70, theta0=0.3, width=W.TWO_PI, dr=10.0), 60.0, (4, 5)),
]


@pytest.mark.parametrize("mode", [W.MODE_3D, W.MODE_NX2D])
@pytest.mark.parametrize("prec", [W.PREC_C128, W.PREC_C64])
@pytest.mark.parametrize("case", WATER, ids=[c[0] for c in WATER])
def test_range_dependent_water_matches_oracle(torch, P, case, prec, mode):
    """Water profiles on range rows (a stair-step in range): every step uses
    the row in force at r_{j+1}, also when r_{j+1} is a row's range exactly;
    the march is split over several calls."""
    name, env, gk, f, calls = case
    grid = W.Grid(precision=prec, mode=mode, **gk)
    st = O.setup(env, grid, f)
    rows = {st.ssp_row_at(st.r(j + 1)) for j in range(sum(calls))}
    assert len(rows) >= 3, rows  # the march crosses rows
    th = st.theta[:, None]
    u0 = O.starter(st, 0.3 * env.zmax) * (1 + 0.3 * np.cos(th)) + 0.05 * W.random_field(1, grid.nz, _seed(name))
    say("range-dependent water", name, prec, mode)
    m = P.Pe3d(env, grid, f)
    u = to_dev(torch, u0, prec)
    for n in calls:
        m.march(n, u)
    torch.cuda.synchronize()
    ref = O.march(st, u0, 0, sum(calls))
    assert O.rel_l2(to_host(torch, u), ref) < TOL[prec], name
    m.close()


@pytest.mark.parametrize("prec", [W.PREC_C64, W.PREC_C128])
def test_equal_water_rows_are_bitwise_range_independent(torch, P, prec):
    base = W.wedge_env()
    rd = dataclasses.replace(base, ssp_c=base.ssp_c * 3, ssp_nr=3, ssp_r0=0.0, ssp_dr=20.0)
    grid = W.Grid(nz=400, ntheta=64, theta0=0.0, width=W.TWO_PI, dr=10.0, precision=prec)
    st = O.setup(base, grid, 60.0)
    u0 = to_dev(torch, O.starter(st, 100.0), prec)
    say("equal water rows", prec)
    out = []
    for env in (base, rd):
        m = P.Pe3d(env, grid, 60.0)
        u = u0.clone()
        m.march(9, u)
        out.append(u)
        m.close()
    torch.cuda.synchronize()
    assert torch.equal(out[0], out[1])


@pytest.mark.parametrize("prec", [W.PREC_C64, W.PREC_C128])
def test_water_profile_per_range_step(torch, P, prec):
    """A water profile that varies continuously in range, given as one row
    per range step (rows at r0 + i dr): the step j -> j+1 takes the profile
    at r_{j+1} exactly, i.e. the matrix update of every step with the medium
    interpolated to its range, each row's factorisation built at create
    time.  Against the oracle marching the same medium."""
    base = W.random_env(61, zmax=400.0)
    nsteps, dr = 40, 6.0
    z = np.asarray(base.ssp_z)
    ca = np.asarray(base.ssp_c)
    cb = ca[::-1].copy() + 15.0
    r = dr * np.arange(nsteps + 1)
    rows = ca[None, :] + (r / r[-1])[:, None] * (cb - ca)[None, :]
    env = dataclasses.replace(base, ssp_c=tuple(rows.ravel()), ssp_nr=nsteps + 1, ssp_r0=0.0, ssp_dr=dr)
    grid = W.Grid(nz=90, ntheta=16, theta0=0.0, width=W.TWO_PI, dr=dr, precision=prec)
    st = O.setup(env, grid, 45.0)
    assert [st.ssp_row_at(st.r(j + 1)) for j in range(nsteps)] == list(range(1, nsteps + 1))
    u0 = O.starter(st, 120.0) * (1 + 0.2 * np.cos(st.theta))[:, None]
    say("water profile per range step", prec)
    m = P.Pe3d(env, grid, 45.0)
    u = to_dev(torch, u0, prec)
    m.march(17, u)
    m.march(nsteps - 17, u)
    torch.cuda.synchronize()
    assert O.rel_l2(to_host(torch, u), O.march(st, u0, 0, nsteps)) < TOL[prec]
    m.close()


@pytest.mark.parametrize("prec", [W.PREC_C64, W.PREC_C128])
def test_full_size_front_matches_oracle(torch, P, prec):
    """The config-2 grid (Nz 2048, Ntheta 512) over the wedge under the
    range-dependent water of an ocean front (a profile every 1 km), started
    at r0 = 980 m: the second step reaches the 1 km row exactly and the
    march continues on it; 4 steps against the oracle over the whole field."""
    p = W.config2_front(nsteps=4, precision=prec)
    grid = dataclasses.replace(p.grid, r0=980.0)
    st = O.setup(p.env, grid, p.f_hz)
    assert [st.ssp_row_at(st.r(j + 1)) for j in range(4)] == [0, 1, 1, 1]
    u0 = O.starter(st, p.zs)
    say("full-size front", prec)
    m = P.Pe3d(p.env, grid, p.f_hz)
    u = to_dev(torch, u0, prec)
    m.march(4, u)
    torch.cuda.synchronize()
    assert O.rel_l2(to_host(torch, u), O.march(st, u0, 0, 4)) < TOL[prec]
    m.close()


@pytest.mark.parametrize("prec", [W.PREC_C64, W.PREC_C128])
def test_full_size_sloping_bottom_matches_oracle(torch, P, prec):
    """The config-2 grid (Nz 2048, Ntheta 512) over the range-dependent
    sloping bottom, started at r0 = 2 km (so every column meets the slope):
    3 steps against the oracle over the whole field."""
    p = W.config2_slope(nsteps=3, precision=prec)
    grid = dataclasses.replace(p.grid, r0=2000.0)
    st = O.setup(p.env, grid, p.f_hz)
    u0 = O.starter(st, p.zs)
    say("full-size slope", prec)
    m = P.Pe3d(p.env, grid, p.f_hz)
    u = to_dev(torch, u0, prec)
    m.march(3, u)
    torch.cuda.synchronize()
    assert O.rel_l2(to_host(torch, u), O.march(st, u0, 0, 3)) < TOL[prec]
    m.close()


@pytest.mark.parametrize("prec", [W.PREC_C64, W.PREC_C128])
def test_batch_mixing_range_dependent_problems(torch, P, prec):
    """Range-dependent and range-independent problems (3D and N x 2D) in one
    batch equal their plain marches bit for bit, graph or not."""
    probs = [
        (RANGE[0][1], W.Grid(precision=prec, **RANGE[0][2]), RANGE[0][3]),
        (W.wedge_env(), W.Grid(nz=200, ntheta=24, theta0=0.0, width=W.TWO_PI, dr=10.0, precision=prec), 40.0),
        (RANGE[3][1], W.Grid(precision=prec, mode=W.MODE_NX2D, **RANGE[3][2]), RANGE[3][3]),
        (RANGE[2][1], W.Grid(precision=prec, **RANGE[2][2]), RANGE[2][3]),
    ]
    steps = [7, 5, 9, 12]
    u0s = []
    for env, grid, f in probs:
        st = O.setup(env, grid, f)
        u0s.append(O.starter(st, 0.3 * env.zmax) * (1 + 0.2 * np.sin(st.theta))[:, None])
    say("batch range-dependent", prec)
    plain = []
    for (env, grid, f), u0, n in zip(probs, u0s, steps):
        m = P.Pe3d(env, grid, f)
        u = to_dev(torch, u0, prec)
        m.march(n, u)
        plain.append(u)
        m.close()
    for use_graph in (False, True):
        ms = [P.Pe3d(env, grid, f) for env, grid, f in probs]
        us = [to_dev(torch, u0, prec) for u0 in u0s]
        P.march_batch(ms, steps, us, use_graph=use_graph)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(plain, us)):
            assert torch.equal(a, b), f"problem {i} graph={use_graph}"
        for m in ms:
            m.close()
    env, grid, f = probs[0]
    ref = O.march(O.setup(env, grid, f), u0s[0], 0, steps[0])
    assert O.rel_l2(to_host(torch, plain[0]), ref) < TOL[prec]


@pytest.fixture
def schedule(P):
    yield P.set_batch_schedule
    P.set_batch_schedule()  # library defaults


@pytest.mark.parametrize("chains,group_bytes", [(1, 0), (2, 0), (3, 1 << 20), (4, 64 << 10), (2, 112 << 20)])
def test_batch_schedules_are_bitwise_equal(torch, P, schedule, chains, group_bytes):
    """Every schedule (chains on concurrent streams, groups marched through
    all of their steps in turn) gives the plain marches bit for bit, graph or
    not.  The fields are written on the caller's stream just before the call
    and read on it just after, with no synchronisation in between: the side
    streams of a graph replay must wait for the first and be waited for by
    the second."""
    prec = W.PREC_C64
    probs = [
        (RANGE[0][1], W.Grid(precision=prec, **RANGE[0][2]), RANGE[0][3]),
        (W.wedge_env(), W.Grid(nz=200, ntheta=24, theta0=0.0, width=W.TWO_PI, dr=10.0, precision=prec), 40.0),
        (RANGE[3][1], W.Grid(precision=prec, mode=W.MODE_NX2D, **RANGE[3][2]), RANGE[3][3]),
        (RANGE[2][1], W.Grid(precision=prec, **RANGE[2][2]), RANGE[2][3]),
        (W.wedge_env(), W.Grid(nz=700, ntheta=64, theta0=0.0, width=W.TWO_PI, dr=10.0, precision=prec), 60.0),
        (W.wedge_env(), W.Grid(nz=90, ntheta=16, theta0=0.0, width=W.TWO_PI, dr=10.0, precision=prec), 25.0),
        (WATER[2][1], W.Grid(precision=prec, **WATER[2][2]), WATER[2][3]),
        (WATER[0][1], W.Grid(precision=prec, mode=W.MODE_NX2D, **WATER[0][2]), WATER[0][3]),
    ]
    steps = [7, 5, 9, 12, 6, 0, 11, 8]
    u0s = []
    for env, grid, f in probs:
        st = O.setup(env, grid, f)
        u0s.append(to_dev(torch, O.starter(st, 0.3 * env.zmax) * (1 + 0.2 * np.sin(st.theta))[:, None], prec))
    say("batch schedule", chains, group_bytes)
    plain = []
    for (env, grid, f), u0, n in zip(probs, u0s, steps):
        m = P.Pe3d(env, grid, f)
        u = u0.clone()
        m.march(n, u)
        plain.append(u)
        m.close()
    torch.cuda.synchronize()
    schedule(chains, group_bytes)
    for use_graph in (False, True):
        ms = [P.Pe3d(env, grid, f) for env, grid, f in probs]
        for rep in range(2):
            for m in ms:
                m.set_step(0)
            us = [u0.clone() for u0 in u0s]
            P.march_batch(ms, steps, us, use_graph=use_graph)
            snap = [u.clone() for u in us]
            torch.cuda.synchronize()
            for i, (a, b) in enumerate(zip(plain, snap)):
                assert torch.equal(a, b), f"problem {i} graph={use_graph} replay {rep}"
            assert [m.step for m in ms] == steps
        for m in ms:
            m.close()


def test_plan_cache_eviction_and_handle_destruction(torch, P):
    """More distinct batched calls than the plan cache holds (64), with
    graphs, evict the oldest plans while their handles live on; destroying a
    handle drops its plans; every call still equals the plain march."""
    env = W.wedge_env()
    grids = [W.Grid(nz=64 + 8 * i, ntheta=16, theta0=0.0, width=W.TWO_PI, dr=10.0) for i in range(3)]
    ms = [P.Pe3d(env, g, 40.0) for g in grids]
    ref = [P.Pe3d(env, g, 40.0) for g in grids]
    us = [m.starter(60.0) for m in ms]
    rs = [m.starter(60.0) for m in ref]
    say("plan cache eviction")
    for call in range(70):
        steps = [1 + call % 5, 1 + (call // 5) % 7, 1 + call % 3]
        P.march_batch(ms, steps, us, use_graph=True)
        for m, r, n in zip(ref, rs, steps):
            m.march(n, r)
    torch.cuda.synchronize()
    for a, b in zip(us, rs):
        assert torch.equal(a, b)
    ms[1].close()
    P.march_batch([ms[0], ms[2]], [2, 3], [us[0], us[2]], use_graph=True)
    ref[0].march(2, rs[0])
    ref[2].march(3, rs[2])
    torch.cuda.synchronize()
    assert torch.equal(us[0], rs[0]) and torch.equal(us[2], rs[2])
    for m in [ms[0], ms[2]] + ref:
        m.close()


def test_pooled_blocks_of_a_destroyed_handle_serve_a_new_one(torch, P):
    """Destroying a handle returns its device memory to the library's pool
    without waiting for the device; a new handle of the same size reuses it
    while another problem's batched march is still queued, and every field
    still equals the plain march."""
    env = W.wedge_env()
    g = W.Grid(nz=300, ntheta=40, theta0=0.0, width=W.TWO_PI, dr=10.0)
    a, b = P.Pe3d(env, g, 50.0), P.Pe3d(env, g, 50.0)
    ua, ub = a.starter(80.0), b.starter(80.0)
    say("pooled blocks")
    P.march_batch([a, b], [3, 5], [ua, ub], use_graph=False)
    torch.cuda.synchronize()
    a.close()                        # its plan goes to the graveyard with its blocks
    P.march_batch([b], [40], [ub], use_graph=False)   # queued, not waited for
    for _ in range(3):               # new handles of a's size while b's work runs
        c = P.Pe3d(env, g, 50.0)
        uc = c.starter(80.0)
        P.march_batch([c], [4], [uc], use_graph=False)
        ref = P.Pe3d(env, g, 50.0)
        ur = ref.starter(80.0)
        ref.march(4, ur)
        torch.cuda.synchronize()
        assert torch.equal(uc, ur)
        c.close()
        ref.close()
    rb = P.Pe3d(env, g, 50.0)
    urb = rb.starter(80.0)
    rb.march(45, urb)
    torch.cuda.synchronize()
    assert torch.equal(ub, urb)
    b.close()
    rb.close()
    # the idle pool goes back to the runtime, and marching works after it
    torch.cuda.synchronize()
    assert P.pe3d_release_pooled_memory() > 0
    assert P.pe3d_release_pooled_memory() == 0
    c = P.Pe3d(env, g, 50.0)
    uc = c.starter(80.0)
    c.march(3, uc)
    got = to_host(torch, uc)
    st = O.setup(env, g, 50.0)
    assert O.rel_l2(got, O.march(st, O.starter(st, 80.0), 0, 3)) < TOL[g.precision]
    c.close()


def test_prepared_graph_runs_nothing_then_replays(torch, P):
    """Capture-only (use_graph == 2) leaves fields and step counters alone;
    the next identical call replays it and equals direct launches bitwise."""
    probs = _batch_problems(W.PREC_C64)
    ms = [P.Pe3d(env, grid, f) for env, grid, f in probs]
    ref = [P.Pe3d(env, grid, f) for env, grid, f in probs]
    us, rs = [], []
    for env, grid, f in probs:
        st = O.setup(env, grid, f)
        u0 = to_dev(torch, O.starter(st, 60.0), W.PREC_C64)
        us.append(u0.clone())
        rs.append(u0.clone())
    say("prepare_batch")
    before = [u.clone() for u in us]
    P.prepare_batch(ms, 3, us)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(us, before))
    assert [m.step for m in ms] == [0] * len(ms)
    P.march_batch(ms, 3, us, use_graph=True)
    P.march_batch(ref, 3, rs, use_graph=False)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(us, rs))
    assert [m.step for m in ms] == [3] * len(ms)
    for m in ms + ref:
        m.close()


def test_graph_replays_match_direct_calls(torch, P):
    probs = _batch_problems(W.PREC_C64)
    steps = [4, 4, 4, 4, 4]
    ms = [P.Pe3d(env, grid, f) for env, grid, f in probs]
    ref = [P.Pe3d(env, grid, f) for env, grid, f in probs]
    us, rs = [], []
    for env, grid, f in probs:
        st = O.setup(env, grid, f)
        u0 = to_dev(torch, O.starter(st, 60.0), W.PREC_C64)
        us.append(u0.clone())
        rs.append(u0.clone())
    for rep in range(3):
        say("graph replay", rep)
        P.march_batch(ms, steps, us, use_graph=True)
        # eager work and a synchronisation between replays
        for m, r in zip(ref, rs):
            m.march(4, r)
        torch.cuda.synchronize()
        for a, b in zip(us, rs):
            assert torch.equal(a, b)
    for m in ms + ref:
        m.close()


def test_tl_matches_oracle(torch, P):
    env = W.wedge_env()
    grid = W.Grid(nz=128, ntheta=16, theta0=0.0, width=W.TWO_PI, dr=10.0, precision=W.PREC_C128)
    st = O.setup(env, grid, 50.0)
    u0 = O.starter(st, 100.0)
    say("tl")
    m = P.Pe3d(env, grid, 50.0)
    u = to_dev(torch, u0, W.PREC_C128)
    m.march(8, u)
    tl = m.tl(u)
    torch.cuda.synchronize()
    ref = O.tl(st, O.march(st, u0, 0, 8), 8)
    got = tl.cpu().numpy()
    mask = np.isfinite(ref) & (ref < np.nanmin(ref) + 60.0)
    assert np.abs(got[mask] - ref[mask]).max() < 1e-3
    m.close()


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [W.PREC_C128, W.PREC_C64])
def test_pressure_matches_oracle(torch, P, prec):
    env = W.wedge_env()
    grid = W.Grid(nz=128, ntheta=16, theta0=0.0, width=W.TWO_PI, dr=10.0, precision=prec)
    st = O.setup(env, grid, 50.0)
    u0 = O.starter(st, 100.0)
    say("pressure", prec)
    m = P.Pe3d(env, grid, 50.0)
    u = to_dev(torch, u0, prec)
    with pytest.raises(P.Pe3dError):
        m.pressure(u)  # r_0 = 0: H0^(1) is singular
    m.march(8, u)
    p = m.pressure(u)
    torch.cuda.synchronize()
    ref = O.pressure(st, O.march(st, u0, 0, 8), 8)
    assert O.rel_l2(to_host(torch, p), ref) < TOL[prec]
    m.close()


def test_c_abi_rejects_bad_arguments_on_gpu(torch, P):
    env = W.wedge_env()
    grid = W.Grid(nz=64, ntheta=8, theta0=0.0, width=W.TWO_PI, dr=10.0)
    say("abi errors")
    m = P.Pe3d(env, grid, 50.0)
    u = m.new_field()
    stream = torch.cuda.current_stream().cuda_stream
    with pytest.raises(P.Pe3dError) as e:
        P.pe3d_march(m.h, -1, u.data_ptr(), stream)
    assert e.value.status == P.PE3D_EINVAL
    with pytest.raises(P.Pe3dError) as e:
        P.pe3d_march(m.h, 1, u.data_ptr() + 8, stream)   # misaligned
    assert e.value.status == P.PE3D_EINVAL
    with pytest.raises(P.Pe3dError):
        P.pe3d_march_batch([m.h, m.h], [1, 1], [u.data_ptr(), u.data_ptr()], True, stream)
    P.pe3d_march(m.h, 0, u.data_ptr(), stream)           # no-op
    assert m.step == 0
    m.close()


# ---------------------------------------------------------------- config 2 / 3
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "config2_oracle_samples.npz")


@pytest.mark.parametrize("prec", [W.PREC_C64, W.PREC_C128])
def test_config2_matches_oracle_checkpoints(torch, P, prec):
    """Config 2 at full size (Nz=2048, Ntheta=512) marched from the GPU
    starter, compared with the oracle's stored checkpoints on every 4th
    azimuth and 16th depth node: c64 <= 1e-5, FP64 within fp64_bar(steps)."""
    g = np.load(GOLDEN)
    cps = [int(c) for c in g["checkpoints"]]
    ts, zs_ = int(g["th_stride"]), int(g["z_stride"])
    p = W.config2(precision=prec)
    say("config2", prec)
    m = P.Pe3d(p.env, p.grid, p.f_hz)
    u = m.starter(p.zs)
    done = 0
    errs = {}
    for c in cps:
        m.march(c - done, u)
        done = c
        got = to_host(torch, u)
        errs[c] = O.rel_l2(got[::ts, ::zs_], g[f"u{c}"])
        nrm = np.linalg.norm(got)
        assert abs(nrm - float(g[f"norm{c}"])) < 1e-4 * float(g[f"norm{c}"])
    say("config2 errors", prec, errs)
    for c, e in errs.items():
        assert e < (1e-5 if prec == W.PREC_C64 else fp64_bar(c)), errs
    m.close()


def fp64_bar(steps):
    """FP64 mode against the complex128 oracle after `steps` steps.  Two FP64
    implementations of one step (here the twisted and circulant
    factorisations against Thomas and Sherman-Morrison) differ by a fixed
    perturbation of a few units in the last place of the step operator, the
    same at every step, so their difference grows linearly: bar = 9 ulp (1e-15)
    per step plus 1e-13 for the starter (the device's exp against NumPy's;
    4e-14 after one step on config 2, where the narrow Gaussian dominates)."""
    return 1e-13 + 1e-15 * steps


GOLDEN3 = os.path.join(os.path.dirname(__file__), "golden", "config3_oracle_samples.npz")


@pytest.mark.parametrize("prec", [W.PREC_C64, W.PREC_C128])
def test_config3_precision_study(torch, P, prec):
    """Config 2 marched to 5000 steps (50 km) from the GPU starter; at every
    500 steps the sampled field (every 4th azimuth, 16th depth) against the
    stored complex128 oracle field: complex64 <= 1e-5 at every checkpoint,
    FP64 within fp64_bar; the full-field norm within 1e-4."""
    g = np.load(GOLDEN3)
    cps = [int(c) for c in g["checkpoints"]]
    ts, zs_ = int(g["th_stride"]), int(g["z_stride"])
    p = W.config2(nsteps=max(cps), precision=prec)
    say("config3 precision", prec)
    m = P.Pe3d(p.env, p.grid, p.f_hz)
    u = m.starter(p.zs)
    done, errs = 0, {}
    for c in cps:
        m.march(c - done, u)
        done = c
        got = to_host(torch, u)
        errs[c] = O.rel_l2(got[::ts, ::zs_], g[f"u{c}"])
        nrm = np.linalg.norm(got)
        assert abs(nrm - float(g[f"norm{c}"])) < 1e-4 * float(g[f"norm{c}"])
    say("config3 errors", prec, errs)
    for c, e in errs.items():
        assert e < (1e-5 if prec == W.PREC_C64 else fp64_bar(c)), errs
    m.close()

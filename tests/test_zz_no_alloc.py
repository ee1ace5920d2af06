"""pe3d_march_static (the allocation-free march: its scratch field is the
library's file-scope device array) against pe3d_march through the C ABI.

Both run the same kernels, so the bar is bit-for-bit equality (reading A18:
bitwise for the same kernel variant), plus the oracle's tolerance on the
smaller problems.  Two or more calls in a row, each later one on a smaller
field than the one before, so that a later call runs on an array still
holding the previous call's larger field.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

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


# name, env, grid kwargs, f, march calls, check against the oracle
CALLS = [
    ("wedge_large_c64", W.wedge_env(),
     dict(nz=1100, ntheta=300, theta0=0.5, width=W.TWO_PI, dr=5.0, precision=W.PREC_C64), 90.0, (3, 4), False),
    ("range_sector_c128", W.random_range_env(42, nr=5, row_dr=15.0, r0=30.0, floor=W.FLOOR_RIGID),
     dict(nz=150, ntheta=20, theta0=1.0, width=1.0, dr=4.0, r0=22.0, precision=W.PREC_C128), 50.0, (2, 5), True),
    ("range_nx2d_c64", W.random_range_env(43, zmax=600.0, nr=8, row_dr=25.0),
     dict(nz=96, ntheta=9, theta0=0.3, width=W.TWO_PI, dr=10.0, precision=W.PREC_C64, mode=W.MODE_NX2D), 60.0,
     (4,), True),
]


def _start(name, env, grid, f):
    st = O.setup(env, grid, f)
    th = st.theta[:, None]
    seed = sum(map(ord, name)) % 1000
    u0 = O.starter(st, 0.3 * env.zmax) * (1 + 0.3 * np.cos(th)) + 0.05 * W.random_field(grid.ntheta, grid.nz, seed)
    return st, u0


def test_static_march_equals_march_on_successive_smaller_fields(torch, P):
    sizes = []
    for name, env, gk, f, calls, oracle_check in CALLS:
        grid = W.Grid(**gk)
        st, u0 = _start(name, env, grid, f)
        sizes.append(grid.nz * grid.ntheta * (16 if grid.precision == W.PREC_C128 else 8))
        say("static march", name, f"nz={grid.nz} nth={grid.ntheta} prec={grid.precision} calls={calls}")
        plain = P.Pe3d(env, grid, f)
        stat = P.Pe3d(env, grid, f)
        ua = to_dev(torch, u0, grid.precision)
        ub = ua.clone()
        for n in calls:
            plain.march(n, ua)
            stat.march_static(n, ub)
        torch.cuda.synchronize()
        assert plain.step == stat.step == sum(calls)
        assert torch.equal(ua, ub), name
        if oracle_check:
            ref = O.march(st, u0, 0, sum(calls))
            assert O.rel_l2(to_host(torch, ub), ref) < TOL[grid.precision], name
        plain.close()
        stat.close()
    # every later call ran on a smaller field than the one before it
    assert all(b < a for a, b in zip(sizes, sizes[1:]))


def test_static_march_rejects_fields_beyond_the_array(torch, P):
    env = W.wedge_env()
    grid = W.Grid(nz=4096, ntheta=1024, theta0=0.0, width=W.TWO_PI, dr=10.0, precision=W.PREC_C128)
    assert grid.nz * grid.ntheta * 16 > P.PE3D_STATIC_SCRATCH_BYTES
    say("static march: oversize field is refused")
    m = P.Pe3d(env, grid, 100.0)
    u = m.starter(100.0)
    torch.cuda.synchronize()
    before = u.clone()
    with pytest.raises(P.Pe3dError) as e:
        m.march_static(3, u)
    assert e.value.status == P.PE3D_EUNSUPPORTED
    torch.cuda.synchronize()
    assert m.step == 0
    assert torch.equal(u, before)
    m.close()
    # the largest complex64 shape the kernels accept fits
    grid64 = W.Grid(nz=4096, ntheta=1024, theta0=0.0, width=W.TWO_PI, dr=10.0, precision=W.PREC_C64)
    assert grid64.nz * grid64.ntheta * 8 <= P.PE3D_STATIC_SCRATCH_BYTES


def test_static_march_argument_errors(torch, P):
    env = W.wedge_env()
    grid = W.Grid(nz=64, ntheta=8, theta0=0.0, width=W.TWO_PI, dr=10.0, precision=W.PREC_C64)
    m = P.Pe3d(env, grid, 40.0)
    u = m.starter(100.0)
    for args in ((m.h, -1, u.data_ptr(), 0), (m.h, 1, 0, 0), (m.h, 1, u.data_ptr() + 8, 0), (None, 1, u.data_ptr(), 0)):
        assert P._lib.pe3d_march_static(args[0], args[1], args[2], args[3]) == P.PE3D_EINVAL
    assert P._lib.pe3d_march_static(m.h, 0, u.data_ptr(), 0) == P.PE3D_OK
    assert m.step == 0
    m.close()

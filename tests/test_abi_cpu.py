"""CPU-only checks of the C ABI: the built library loads, exports every
function include/pe3d.h declares, and rejects invalid arguments before any
device call (so these run without a GPU)."""
import ctypes as ct
import math
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pe3d.h")
LIB = os.path.join(ROOT, "paper_1711_00005_amd", "libpe3d.so")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pe3d_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def P():
    if not os.path.exists(LIB):
        pytest.fail("libpe3d.so is not built (run __graft_entry__.build())")
    import paper_1711_00005_amd.pe3d as _P
    return _P


def test_library_exports_every_declared_function(P):
    lib = ct.CDLL(LIB)
    names = declared_functions()
    assert "pe3d_create" in names and "pe3d_march" in names and "pe3d_destroy" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(P.EXPORTED) == set(names)


def test_strerror(P):
    for s in (0, -1, -2, -3, -4, -5):
        assert P.pe3d_strerror(s)
    assert P.pe3d_strerror(7) == "unknown status"


def test_batch_schedule_validation(P):
    lib = P._lib
    assert lib.pe3d_set_batch_schedule(0, 0) == P.PE3D_EINVAL
    assert lib.pe3d_set_batch_schedule(5, 0) == P.PE3D_EINVAL
    assert lib.pe3d_set_batch_schedule(2, -1) == P.PE3D_EINVAL
    assert lib.pe3d_set_batch_schedule(4, 0) == 0
    P.set_batch_schedule()
    with pytest.raises(Exception):
        P.set_batch_schedule(0)


def test_footprint_is_tables_plus_one_field(P):
    p = W.config2()
    b = P.pe3d_footprint(p.env, p.grid, p.f_hz)
    field = 2048 * 512 * 8
    assert field < b < field + 2 * 1024 * 1024
    b128 = P.pe3d_footprint(p.env, W.Grid(nz=2048, ntheta=512, theta0=0, width=W.TWO_PI, dr=10,
                                           precision=W.PREC_C128), p.f_hz)
    assert b128 > 2 * field


def _status(P, env, grid, f=100.0):
    return P.pe3d_create_status(env, grid, f)


def test_create_rejects_invalid_arguments_without_a_device(P):
    env = W.wedge_env()
    ok = dict(nz=64, ntheta=8, theta0=0.0, width=W.TWO_PI, dr=10.0)
    bad_grids = [
        dict(ok, nz=1), dict(ok, ntheta=2), dict(ok, dr=0.0), dict(ok, dr=float("nan")),
        dict(ok, r0=-1.0), dict(ok, width=0.0), dict(ok, precision=7), dict(ok, mode=2), dict(ok, mode=-1),
    ]
    for g in bad_grids:
        assert _status(P, env, W.Grid(**g)) == P.PE3D_EINVAL, g
    g = W.Grid(**ok)
    assert _status(P, env, g, f=0.0) == P.PE3D_EINVAL
    assert _status(P, env, g, f=float("inf")) == P.PE3D_EINVAL
    from dataclasses import replace
    for e in (replace(env, c0=0.0), replace(env, ssp_z=(10.0, 5.0), ssp_c=(1500.0, 1500.0)),
              replace(env, rho_b=-1.0), replace(env, atten_b=-0.1), replace(env, floor=3),
              replace(env, bathy_theta=(0.0, 7.0), bathy_depth=(10.0, 20.0)), replace(env, zmax=0.0)):
        assert _status(P, e, g) == P.PE3D_EINVAL, e
    # sector with one azimuth is valid; a periodic grid needs three
    sec = W.Grid(nz=64, ntheta=1, theta0=0.0, width=math.radians(30), dr=10.0)
    assert _status(P, env, sec) != P.PE3D_EINVAL


def test_water_rows_are_validated(P):
    from dataclasses import replace
    env = W.random_ssp_range_env(5, nr=3)
    g = W.Grid(nz=64, ntheta=8, theta0=0.0, width=W.TWO_PI, dr=10.0)
    assert _status(P, env, g) != P.PE3D_EINVAL
    c = list(env.ssp_c)
    bad = [replace(env, ssp_dr=0.0), replace(env, ssp_dr=float("nan")), replace(env, ssp_r0=float("inf")),
           replace(env, ssp_c=tuple(c[:-1] + [float("nan")])), replace(env, ssp_c=tuple(c[:5] + [-1.0] + c[6:]))]
    for e in bad:
        assert _status(P, e, g) == P.PE3D_EINVAL, e
    e = replace(env, ssp_nr=-1, ssp_c=tuple(c[:len(env.ssp_z)]))
    assert _status(P, e, g) == P.PE3D_EINVAL
    # the binding refuses arrays whose length does not match the row count
    with pytest.raises(ValueError):
        _status(P, replace(env, ssp_c=tuple(c[:-1])), g)
    with pytest.raises(ValueError):
        _status(P, replace(W.random_range_env(5, nr=3), bathy_nr=4), g)


def test_footprint_counts_one_table_block_per_water_row(P):
    from dataclasses import replace
    g = W.Grid(nz=2048, ntheta=512, theta0=0.0, width=W.TWO_PI, dr=10.0)
    one = W.wedge_env()
    fp = {}
    for nr in (1, 2, 5):
        e = replace(one, ssp_c=one.ssp_c * nr, ssp_nr=nr if nr > 1 else 0, ssp_r0=0.0, ssp_dr=1000.0)
        fp[nr] = P.pe3d_footprint(e, g, 100.0)
    block = fp[2] - fp[1]
    assert 0 < block < 2 * 1024 * 1024
    assert fp[5] - fp[1] == 4 * block


def test_kernel_lanes_overrides_are_validated(P):
    env = W.wedge_env()
    g = dict(nz=300, ntheta=70, theta0=0.0, width=W.TWO_PI, dr=10.0)
    for la, lb in ((0, 0), (32, 0), (256, 0), (0, 8), (0, 64), (64, 16)):
        assert _status(P, env, W.Grid(depth_lanes=la, azimuth_lanes=lb, **g)) not in (
            P.PE3D_EINVAL, P.PE3D_EUNSUPPORTED), (la, lb)
    for la, lb in ((3, 0), (512, 0), (0, 3), (0, 128), (-4, 0)):
        assert _status(P, env, W.Grid(depth_lanes=la, azimuth_lanes=lb, **g)) == P.PE3D_EINVAL, (la, lb)
    # 16 lanes for 300 depths would need 21 rows per lane; 4 azimuth lanes 18 azimuths each
    for la, lb in ((16, 0), (0, 4)):
        assert _status(P, env, W.Grid(depth_lanes=la, azimuth_lanes=lb, **g)) == P.PE3D_EUNSUPPORTED, (la, lb)
    b0 = P.pe3d_footprint(env, W.Grid(**g), 40.0)
    b1 = P.pe3d_footprint(env, W.Grid(depth_lanes=256, **g), 40.0)
    assert b0 > 0 and b1 > 0


def test_azimuth_solver_is_validated(P):
    env = W.wedge_env()
    g = dict(nz=300, ntheta=70, theta0=0.0, width=W.TWO_PI, dr=10.0)
    for solver, lb in ((W.AZ_CHUNKED, 0), (W.AZ_PCR, 0), (W.AZ_CHUNKED, 8)):
        assert _status(P, env, W.Grid(azimuth_solver=solver, azimuth_lanes=lb, **g)) not in (
            P.PE3D_EINVAL, P.PE3D_EUNSUPPORTED), (solver, lb)
    # unknown solver; lanes are a parameter of the chunked solver only
    for solver, lb in ((2, 0), (-1, 0), (W.AZ_PCR, 8)):
        assert _status(P, env, W.Grid(azimuth_solver=solver, azimuth_lanes=lb, **g)) == P.PE3D_EINVAL, (solver, lb)
    assert (P.PE3D_AZIMUTH_CHUNKED, P.PE3D_AZIMUTH_PCR) == (W.AZ_CHUNKED, W.AZ_PCR)


def test_create_reports_unsupported_sizes(P):
    env = W.wedge_env()
    assert _status(P, env, W.Grid(nz=4097, ntheta=8, theta0=0, width=W.TWO_PI, dr=10.0)) == P.PE3D_EUNSUPPORTED
    assert _status(P, env, W.Grid(nz=64, ntheta=1025, theta0=0, width=W.TWO_PI, dr=10.0)) == P.PE3D_EUNSUPPORTED
    assert _status(P, env, W.Grid(nz=4097, ntheta=8, theta0=0, width=W.TWO_PI, dr=10.0,
                                  precision=W.PREC_C128)) == P.PE3D_EUNSUPPORTED


def test_pressure_rejects_null_arguments(P):
    with pytest.raises(P.Pe3dError):
        P.pe3d_pressure(None, 16, 16, None)


def test_null_handles_are_rejected(P):
    with pytest.raises(P.Pe3dError):
        P.pe3d_march(None, 1, 16, None)
    with pytest.raises(P.Pe3dError):
        P.pe3d_get_step(None)
    P.pe3d_destroy(None)


def test_tuner_candidates_are_the_shapes_the_library_accepts(P):
    """tune.candidates lists exactly the lane counts that pe3d_create accepts
    for a shape: every candidate passes validation, and the next smaller
    power of two is refused as unsupported (checked without a device)."""
    from dataclasses import replace
    from paper_1711_00005_amd import tune as T
    env = W.wedge_env()
    for nz, nth in ((64, 8), (300, 70), (700, 384), (2048, 512), (4096, 1024), (320, 17)):
        g = W.Grid(nz=nz, ntheta=nth, theta0=0.0, width=W.TWO_PI, dr=10.0)
        la, lb = T.candidates(g)
        assert la and la[-1] == 256 and lb and lb[-1] == 64, (nz, nth)
        for L in la:
            assert _status(P, env, replace(g, depth_lanes=L)) not in (P.PE3D_EINVAL, P.PE3D_EUNSUPPORTED), (nz, L)
        for Wl in lb:
            assert _status(P, env, replace(g, azimuth_lanes=Wl)) not in (
                P.PE3D_EINVAL, P.PE3D_EUNSUPPORTED), (nth, Wl)
        if la[0] > 4:
            assert _status(P, env, replace(g, depth_lanes=la[0] // 2)) == P.PE3D_EUNSUPPORTED, (nz, la)
        if lb[0] > 1:
            assert _status(P, env, replace(g, azimuth_lanes=lb[0] // 2)) == P.PE3D_EUNSUPPORTED, (nth, lb)

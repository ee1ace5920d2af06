"""CPU checks of the FP64 coefficient builder behind pe3d_create, read
through pe3d_host_tables (no device): every exported quantity is rebuilt
from the oracle's operators (Eqs. (4), (5), (7)) and compared.

The exported interface record of column m holds, for row k then row k+1,
the RHS diagonal, the coefficients on the previous and next row of that
row's elimination order, the elimination multiplier (all four divided by
nbmh = -beta_- h) and the two entries of the 2x2 inverse that give the row's
value (times nbmh).  The last test solves every column's depth system with
exactly those numbers (twisted factorisation: top-down above the interface,
bottom-up below) and compares with a dense solve."""
import dataclasses

import numpy as np
import pytest

import oracle as O
import workloads as W


@pytest.fixture(scope="module")
def P():
    import paper_1711_00005_amd.pe3d as _P
    return _P


CASES = [
    ("wedge_pr", W.wedge_env(), W.Grid(nz=96, ntheta=10, theta0=0.2, width=W.TWO_PI, dr=10.0), 60.0),
    ("wedge_rigid", dataclasses.replace(W.wedge_env(), floor=W.FLOOR_RIGID),
     W.Grid(nz=80, ntheta=9, theta0=0.0, width=W.TWO_PI, dr=7.0), 45.0),
    ("sector_layered", W.flat_layered_env(), W.Grid(nz=70, ntheta=6, theta0=1.0, width=1.2, dr=5.0), 30.0),
    ("near_floor_rigid", dataclasses.replace(W.wedge_env(), bathy_theta=(0.0, 3.0), bathy_depth=(2990.0, 1.0),
                                            floor=W.FLOOR_RIGID, zmax=3000.0),
     W.Grid(nz=60, ntheta=16, theta0=0.0, width=W.TWO_PI, dr=10.0), 40.0),
    ("range_rows", W.random_range_env(31, nr=5, row_dr=30.0, r0=20.0),
     W.Grid(nz=64, ntheta=12, theta0=0.3, width=W.TWO_PI, dr=5.0, r0=57.0), 50.0),
]


def _tie_env():
    """Rigid floor, dz = 5 m exactly, depth rows on whole multiples of dz:
    water-node decisions that are exact ties at the range nodes."""
    base = W.random_env(32, zmax=300.0, floor=W.FLOOR_RIGID, nbathy=4)
    rows = 5.0 * np.array([[10, 20, 30, 40], [11, 25, 7, 59], [3, 60, 33, 12]], dtype=float)
    return dataclasses.replace(base, bathy_theta=(-3.0, -1.0, 0.5, 2.0), bathy_depth=tuple(rows.ravel()),
                               bathy_nr=3, bathy_r0=40.0, bathy_dr=25.0)


@pytest.mark.parametrize("r0", [0.0, 40.0, 52.5, 64.999, 65.0, 77.0, 90.0, 1000.0])
def test_water_nodes_at_a_range_match_the_oracle(P, r0):
    """The host's D(r) between range rows and its water count give the
    oracle's mask at r0: exact nodes, ties l dz == D, inside, both ends."""
    env = _tie_env()
    grid = W.Grid(nz=60, ntheta=4, theta0=0.0, width=W.TWO_PI, dr=5.0, r0=r0)
    st = O.setup(env, grid, 40.0)
    T = P.pe3d_host_tables(env, grid, 40.0)
    nw = st.water.sum(axis=1)
    assert np.array_equal(T["kcol"], np.clip(nw - 1, 0, 58)), (T["kcol"], nw)


def _lu_pivots(a, b, c):
    """Top-down pivots of the tridiagonal (a: lower, b: diagonal, c: upper)."""
    n = len(b)
    p = np.zeros(n, complex)
    for i in range(n):
        p[i] = b[i] if i == 0 else b[i] - a[i] * c[i - 1] / p[i - 1]
    return p


@pytest.mark.parametrize("name,env,grid,f", CASES, ids=[c[0] for c in CASES])
def test_host_tables_match_the_oracle_operators(P, name, env, grid, f):
    st = O.setup(env, grid, f)
    T = P.pe3d_host_tables(env, grid, f)
    N, NT = st.nz, st.nth
    bm, bp, h = st.beta_m, st.beta_p, st.h
    nbmh = -bm * h
    # interface row per column from the water mask
    nw = st.water.sum(axis=1)
    k = np.clip(nw - 1, 0, N - 2)
    assert np.array_equal(T["kcol"], k)
    # n^2 - 1 of the water column: equals the oracle's q on water nodes
    for m in range(NT):
        wet = st.water[m]
        # q = n^2 - 1 cancels where c is near c0: compare to an ulp of n^2
        assert np.allclose(T["qw"][wet], st.q[m][wet], rtol=1e-14, atol=1e-15)
    # all-water column, top-down pivots of I + beta_- X (uniform density)
    qw = T["qw"]
    xl = np.full(N, h, complex); xl[0] = 0.0
    xu = np.full(N, h, complex); xu[-1] = 0.0
    xd = qw - 2.0 * h
    if env.floor == W.FLOOR_RIGID:
        xl[-1] = 2.0 * h
    pw = _lu_pivots(bm * xl, 1.0 + bm * xd, bm * xu)
    np.testing.assert_allclose(T["pw"], 1.0 / pw, rtol=1e-13)
    # all-bottom column, bottom-up pivots (reverse the system); the rigid floor
    # row is halved so that its lower coefficient is beta_- h
    qb = (env.c0 / env.c_b) ** 2 * (1 + 1j * O.ETA * env.atten_b) ** 2 - 1.0
    bxd = np.full(N, qb - 2.0 * h, complex)
    a_ = bm * np.full(N, h, complex); a_[0] = 0.0
    c_ = bm * np.full(N, h, complex); c_[-1] = 0.0
    d_ = 1.0 + bm * bxd
    if env.floor == W.FLOOR_RIGID:
        a_[-1] = bm * h          # 2 beta_- h halved
        d_[-1] = 0.5 * d_[-1]
    pb_rev = _lu_pivots(c_[::-1], d_[::-1], a_[::-1])
    np.testing.assert_allclose(T["pb"], 1.0 / pb_rev[::-1], rtol=1e-13)


@pytest.mark.parametrize("name,env,grid,f", CASES, ids=[c[0] for c in CASES])
def test_interface_records_solve_every_column(P, name, env, grid, f):
    st = O.setup(env, grid, f)
    T = P.pe3d_host_tables(env, grid, f)
    N, NT = st.nz, st.nth
    bm, bp, h = st.beta_m, st.beta_p, st.h
    nbmh = -bm * h
    rng = np.random.default_rng(7)
    rigid = env.floor == W.FLOOR_RIGID
    for m in range(NT):
        k = int(T["kcol"][m])
        rec = T["blk"][m] * np.array([nbmh] * 4 + [1 / nbmh] * 2 + [nbmh] * 4 + [1 / nbmh] * 2)
        c0t, cpt, cnt, cft, iat, ibt, c0b, cpb, cnb, cfb, iab, ibb = rec
        A_l, A_d, A_u = bm * st.xl[m], 1.0 + bm * st.xd[m], bm * st.xu[m]
        B_l, B_d, B_u = bp * st.xl[m], 1.0 + bp * st.xd[m], bp * st.xu[m]
        # the record's RHS rows are the column's own rows k and k+1 of [I + beta_+ X]
        assert np.isclose(c0t, B_d[k], rtol=1e-13) and np.isclose(cnt, B_u[k], rtol=1e-13, atol=1e-300)
        assert np.isclose(cpt, B_l[k], rtol=1e-13, atol=1e-300)
        assert np.isclose(c0b, B_d[k + 1], rtol=1e-13) and np.isclose(cnb, B_l[k + 1], rtol=1e-13)
        assert np.isclose(cpb, B_u[k + 1], rtol=1e-13, atol=1e-300)
        R = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        # twisted solve with the exported pivots and record
        Gw, Gb = T["pw"], T["pb"]
        y = np.zeros(N, complex)
        for r in range(k):          # top chain, top-down: y_r = R_r - A_l[r] y_{r-1} / p_{r-1}
            y[r] = R[r] - (A_l[r] * y[r - 1] * Gw[r - 1] if r > 0 else 0.0)
        z = np.zeros(N, complex)
        bscale = np.ones(N)
        if rigid:
            bscale[N - 1] = 0.5      # the bottom system halves the floor row
        for r in range(N - 1, k + 1, -1):   # bottom chain, bottom-up
            Rr = R[r] * bscale[r]
            z[r] = Rr - ((bm * h) * z[r + 1] * Gb[r + 1] if r < N - 1 else 0.0)
        rk = R[k] + (cft * y[k - 1] * Gw[k - 1] if k >= 1 else 0.0)
        rk1 = R[k + 1] + (cfb * z[k + 2] * Gb[k + 2] if k + 2 <= N - 1 else 0.0)
        v = np.zeros(N, complex)
        v[k] = iat * rk + ibt * rk1
        v[k + 1] = iab * rk1 + ibb * rk
        for r in range(k - 1, -1, -1):      # back substitution, top chain upward
            v[r] = Gw[r] * (y[r] - (bm * h) * v[r + 1])
        for r in range(k + 2, N):           # bottom chain downward
            v[r] = Gb[r] * (z[r] - (bm * h) * v[r - 1])
        dense = np.diag(A_d) + np.diag(A_l[1:], -1) + np.diag(A_u[:-1], 1)
        ref = np.linalg.solve(dense, R)
        assert np.linalg.norm(v - ref) / np.linalg.norm(ref) < 1e-12, (name, m, k)


def test_water_rows_keep_row_zero_tables_and_are_validated_per_row(P):
    """With water-profile rows the exported tables are row 0's, equal to a
    single-profile environment of that row; every row is built (and its
    pivots checked) at create time, so an invalid later row is refused."""
    base = W.random_env(71)
    rows = [tuple(base.ssp_c), tuple(c + 20.0 for c in base.ssp_c), tuple(c - 15.0 for c in base.ssp_c)]
    env = dataclasses.replace(base, ssp_c=sum(rows, ()), ssp_nr=3, ssp_r0=0.0, ssp_dr=50.0)
    grid = W.Grid(nz=64, ntheta=8, theta0=0.0, width=W.TWO_PI, dr=5.0)
    a = P.pe3d_host_tables(env, grid, 40.0)
    b = P.pe3d_host_tables(base, grid, 40.0)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    bad = dataclasses.replace(env, ssp_c=rows[0] + rows[1] + tuple([0.0] * len(base.ssp_z)))
    assert P.pe3d_create_status(bad, grid, 40.0) == P.PE3D_EINVAL

"""Pins of the complex128 oracle against facts fixed by the mathematics.

None of these re-derives the oracle's own code path: each checks the oracle
against an independent route (a dense LAPACK solve, the FFT diagonalisation of
a circulant, the closed-form modal solution of a separable problem, an exact
conservation law, a physical interface condition, symmetries).
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.modal import modal_march as _modal_march


def _rng(seed):
    return np.random.default_rng(seed)


def _crand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# --------------------------------------------------------------- P1: dense LU
@pytest.mark.parametrize("n", [1, 2, 3, 7, 64])
def test_thomas_matches_dense_solve(n):
    rng = _rng(n)
    a, b, c, d = (_crand(rng, 5, n) for _ in range(4))
    b = b + 4.0  # keep systems safely nonsingular without pivoting
    x = O.thomas(a, b, c, d)
    for k in range(5):
        M = np.diag(b[k]) + np.diag(a[k, 1:], -1) + np.diag(c[k, :-1], 1)
        ref = np.linalg.solve(M, d[k])
        assert np.allclose(x[k], ref, rtol=1e-13, atol=1e-13)


def test_thomas_non_dominant_system():
    # the depth systems are not diagonally dominant (h > 1); Thomas without
    # pivoting must still agree with LU with partial pivoting
    rng = _rng(11)
    n = 40
    a = np.full(n, 3.0 - 2.0j)
    c = np.full(n, 3.0 - 2.0j)
    b = 1.0 - 2.0 * a + 0.1 * _crand(rng, n)
    d = _crand(rng, n)
    M = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
    assert np.allclose(O.thomas(a, b, c, d), np.linalg.solve(M, d), rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("n", [3, 4, 5, 33, 128])
def test_periodic_sm_matches_dense_solve(n):
    rng = _rng(100 + n)
    a, b, c = (_crand(rng, n) for _ in range(3))
    b = b + 5.0
    d = _crand(rng, 3, n)
    x = O.periodic_thomas_sm(a, b, c, d)
    M = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
    M[0, n - 1] = a[0]
    M[n - 1, 0] = c[n - 1]
    for k in range(3):
        assert np.allclose(x[k], np.linalg.solve(M, d[k]), rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------- P8: FFT circulant
@pytest.mark.parametrize("sigma", [1.6e-5, 0.3, 25.0, 396.0])
@pytest.mark.parametrize("n", [5, 32, 512])
def test_periodic_azimuth_solve_matches_fft(sigma, n):
    """(I - s D_theta) is circulant with eigenvalues 1 + 4 i sigma sin^2(pi q/n)
    for s = i sigma; solving by DFT is exact and independent of Thomas+SM."""
    s = 1j * sigma
    rng = _rng(int(sigma * 7) + n)
    v = _crand(rng, 4, n)
    lo = np.full(n, -s)
    di = np.full(n, 1.0 + 2.0 * s)
    x = O.periodic_thomas_sm(lo, di, lo, v)
    q = np.arange(n)
    lam = 1.0 + 4.0j * sigma * np.sin(np.pi * q / n) ** 2
    ref = np.fft.ifft(np.fft.fft(v, axis=-1) / lam, axis=-1)
    assert np.allclose(x, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


# --------------------------------------------------------------- medium / grid
def test_attenuation_conversion_constant():
    # 1 dB per wavelength is an amplitude decay exp(-k_i lambda) with
    # 20 log10(e) k_i lambda = 1, i.e. k_i / k_r = 1/(40 pi log10 e)
    assert abs(O.ETA - 0.0183233) < 1e-6
    k_r = 1.0
    lam = 2 * math.pi / k_r
    k_i = O.ETA * k_r
    assert abs(20 * math.log10(math.e) * k_i * lam - 1.0) < 1e-12


def test_wedge_depth_and_node_classes():
    env = W.wedge_env()
    th = np.array([0.0, math.pi / 2, -math.pi / 2, math.pi, -math.pi, 3 * math.pi])
    d = O.interp_bathy(th, env.bathy_theta, env.bathy_depth)
    assert np.allclose(d, [2000.0, 1100.0, 1100.0, 200.0, 200.0, 200.0])
    grid = W.Grid(nz=30, ntheta=8, theta0=0.0, width=W.TWO_PI, dr=10.0)
    st = O.setup(env, grid, 100.0)
    dz = 3000.0 / 31
    assert abs(st.dz - dz) < 1e-12
    # column 0 (theta=0, D=2000): nodes with l*dz <= 2000 are water
    nw = int(math.floor(2000.0 / dz))
    assert st.water[0].sum() == nw
    assert st.water[4].sum() == int(math.floor(200.0 / dz))  # theta = pi
    # bottom node value of n^2 - 1 with 0.5 dB/lambda
    qb = (1500.0 / 1700.0) ** 2 * (1 + 1j * O.ETA * 0.5) ** 2 - 1.0
    assert abs(st.q[0, -1] - qb) < 1e-15
    # Munk axis: minimum speed 1490 at 1000 m
    c = O.interp_ssp(np.array([1000.0]), env.ssp_z, env.ssp_c)
    assert abs(c[0] - 1490.0) < 1e-9


def test_sector_grid_edges():
    env = W.isovelocity_env()
    grid = W.Grid(nz=8, ntheta=5, theta0=1.0, width=math.radians(30.0), dr=5.0)
    st = O.setup(env, grid, 25.0)
    assert not st.periodic
    dth = math.radians(30.0) / 6
    assert np.allclose(st.theta, 1.0 - math.radians(15.0) + dth * np.arange(1, 6))


# --------------------------------------------------------------- interface condition
@pytest.mark.parametrize("floor", [W.FLOOR_RIGID, W.FLOOR_PRESSURE_RELEASE])
def test_density_weighted_operator_annihilates_flux_continuous_profile(floor):
    """With q = 0, a profile that is continuous with continuous normal
    velocity (1/rho) du/dz across a density jump solves d/dz((1/rho) du/dz) = 0;
    between nodes the jump sits midway, so u_{l+1} - u_l = dz g (rho_l +
    rho_{l+1})/2.  The discrete X must return 0 at every interior node."""
    env = W.Env(c0=1500.0, ssp_z=(0.0,), ssp_c=(1500.0,), rho_w=1.0, atten_w=0.0,
                c_b=1500.0, rho_b=1.8, atten_b=0.0, bathy_theta=(0.0,),
                bathy_depth=(120.0,), zmax=200.0, floor=floor)
    grid = W.Grid(nz=40, ntheta=3, theta0=0.0, width=W.TWO_PI, dr=5.0)
    st = O.setup(env, grid, 30.0)
    rho = st.rho[0]
    assert rho.min() == 1.0 and rho.max() == 1.8
    rpad = np.concatenate([[rho[0]], rho])
    du = st.dz * 0.37 * 0.5 * (rpad[:-1] + rpad[1:])  # u_l - u_{l-1}, u_0 = 0
    u = np.cumsum(du)
    xu = O.apply_tridiag(st.xl[0], st.xd[0], st.xu[0], u.astype(complex))
    assert np.abs(xu[:-1]).max() < 1e-10 * st.h * np.abs(u).max()
    # the harmonic mean (a plausible mistake) would not annihilate it
    assert abs(st.h) > 1.0


# --------------------------------------------------------------- P3: closed form
@pytest.mark.parametrize("floor", [W.FLOOR_RIGID, W.FLOOR_PRESSURE_RELEASE])
@pytest.mark.parametrize("c,att", [(1500.0, 0.0), (1523.0, 0.2)])
def test_closed_form_modal_march(floor, c, att):
    env = W.isovelocity_env(depth=200.0, c=c, atten=att, floor=floor)
    grid = W.Grid(nz=64, ntheta=32, theta0=0.0, width=W.TWO_PI, dr=5.0,
                  precision=W.PREC_C128)
    st = O.setup(env, grid, 25.0)
    u0 = O.starter(st, 50.0)
    th = st.theta[:, None]
    u0 = u0 * (1 + 0.5 * np.cos(th)) + 0.2j * u0 * np.sin(3 * th)
    nsteps = 200
    u = O.march(st, u0, 0, nsteps)
    ref = _modal_march(st, u0, nsteps, floor)
    assert O.rel_l2(u, ref) < 1e-12


@pytest.mark.parametrize("width", [W.TWO_PI, 1.0])
def test_nx2d_closed_form_per_azimuth(width):
    """N x 2D mode (Y = 0, Sec. 1): every azimuth column follows the 2D
    Crank-Nicolson march alone, G_k^j per depth mode, whatever its
    neighbours hold; and the 3D march of the same field differs."""
    env = W.isovelocity_env(depth=200.0, c=1510.0, atten=0.1, floor=W.FLOOR_RIGID)
    kw = dict(nz=48, ntheta=10, theta0=0.2, width=width, dr=5.0, r0=40.0, precision=W.PREC_C128)
    st = O.setup(env, W.Grid(mode=W.MODE_NX2D, **kw), 25.0)
    assert st.s(0) == 0.0
    u0 = O.starter(st, 50.0) * (1.0 + np.arange(10)[:, None]) + 0.3j * W.random_field(10, 48, seed=9)
    u = O.march(st, u0, 0, 60)
    assert O.rel_l2(u, _modal_march(st, u0, 60, W.FLOOR_RIGID, coupled=False)) < 1e-12
    # a column evolves alone: zeroing the others changes nothing in it
    v0 = np.zeros_like(u0)
    v0[4] = u0[4]
    v = O.march(st, v0, 0, 60)
    assert np.array_equal(v[4], u[4]) and not v[3].any()
    u3 = O.march(O.setup(env, W.Grid(**kw), 25.0), u0, 0, 60)
    assert O.rel_l2(u3, u) > 1e-4


def test_nx2d_equals_3d_for_azimuth_uniform_field():
    """Periodic grid, azimuth-independent medium and field: D_theta u = 0 at
    every step, so the coupled march reduces to the N x 2D one."""
    env = W.isovelocity_env(depth=120.0, c=1480.0, floor=W.FLOOR_PRESSURE_RELEASE)
    kw = dict(nz=40, ntheta=8, theta0=0.0, width=W.TWO_PI, dr=4.0, precision=W.PREC_C128)
    s3 = O.setup(env, W.Grid(**kw), 30.0)
    s2 = O.setup(env, W.Grid(mode=W.MODE_NX2D, **kw), 30.0)
    u0 = np.repeat(O.starter(s3, 30.0)[:1], 8, axis=0)
    u3, u2 = O.march(s3, u0, 0, 40), O.march(s2, u0, 0, 40)
    assert O.rel_l2(u3, u2) < 1e-13


def test_closed_form_nonzero_start_range():
    env = W.isovelocity_env(depth=150.0, c=1490.0, floor=W.FLOOR_PRESSURE_RELEASE)
    grid = W.Grid(nz=20, ntheta=12, theta0=0.3, width=W.TWO_PI, dr=7.0, r0=350.0)
    st = O.setup(env, grid, 40.0)
    u0 = W.random_field(12, 20, seed=3)
    u = O.march(st, u0, 0, 30)
    assert O.rel_l2(u, _modal_march(st, u0, 30, W.FLOOR_PRESSURE_RELEASE)) < 1e-12


# --------------------------------------------------------------- P9: one-way factor
def test_small_angle_mode_follows_one_way_propagator():
    """A low depth mode in deep isovelocity water has tiny lambda; the step's
    amplification must track exp(i k0 dr (sqrt(1+lambda) - 1)) (the one-way
    factor of Eq. (3) with e^{-i omega t}); the complex conjugate would not."""
    env = W.isovelocity_env(depth=1000.0, c=1500.0, floor=W.FLOOR_PRESSURE_RELEASE)
    grid = W.Grid(nz=400, ntheta=3, theta0=0.0, width=W.TWO_PI, dr=10.0)
    st = O.setup(env, grid, 100.0)
    ang = math.pi / (st.nz + 1)
    mode = np.sin(ang * np.arange(1, st.nz + 1))
    u0 = np.repeat(mode[None, :].astype(complex), 3, axis=0)
    u1 = O.step(st, u0, 5)
    g = (u1[0] @ mode) / (mode @ mode)
    lam = -4 * st.h * math.sin(ang / 2) ** 2
    exact = np.exp(1j * st.k0 * st.dr * (math.sqrt(1 + lam) - 1))
    assert abs(g - exact) < 1e-3 * abs(exact - 1)
    assert abs(g - np.conj(exact)) > 0.5 * abs(exact - 1)


# --------------------------------------------------------------- P4: energy identity
def _weights(st, floor):
    rho = st.rho
    w = 1.0 / rho
    if floor == W.FLOOR_RIGID:
        w = w.copy()
        w[:, -1] = 2.0 / (3.0 * rho[:, -1] + rho[:, -2])
    return w


@pytest.mark.parametrize("floor", [W.FLOOR_RIGID, W.FLOOR_PRESSURE_RELEASE])
@pytest.mark.parametrize("periodic", [True, False])
def test_lossless_weighted_energy_identity(floor, periodic):
    """For real n^2, X is symmetric in the weight W = diag(1/rho) (rigid floor
    node adjusted), so [I + beta_-X]^{-1}[I + beta_+X] is W-unitary column by
    column and  || (I - s D) u^{j+1} ||_W = || (I + s D) u^j ||_W  exactly,
    also for an azimuth-dependent medium with density jumps."""
    env = W.random_env(seed=5, zmax=300.0, lossless=True, floor=floor)
    width = W.TWO_PI if periodic else math.radians(90.0)
    grid = W.Grid(nz=50, ntheta=17, theta0=0.4, width=width, dr=8.0)
    st = O.setup(env, grid, 60.0)
    assert np.abs(st.q.imag).max() == 0.0
    assert len(np.unique(st.water.sum(axis=1))) > 3
    wts = _weights(st, floor)
    u = W.random_field(17, 50, seed=9)
    for j in range(3, 8):
        s = st.s(j)
        un = O.step(st, u, j)
        lhs = np.sum(wts * np.abs(O.y_apply(st, un, s, -1.0)) ** 2)
        rhs = np.sum(wts * np.abs(O.y_apply(st, u, s, +1.0)) ** 2)
        assert abs(lhs - rhs) < 1e-13 * rhs
        u = un


def test_attenuation_dissipates_weighted_energy():
    env = W.random_env(seed=6, zmax=300.0, lossless=False)
    grid = W.Grid(nz=50, ntheta=16, theta0=0.0, width=W.TWO_PI, dr=8.0)
    st = O.setup(env, grid, 60.0)
    wts = 1.0 / st.rho
    u = O.starter(st, 60.0)
    for j in range(2, 6):
        s = st.s(j)
        un = O.step(st, u, j)
        lhs = np.sum(wts * np.abs(O.y_apply(st, un, s, -1.0)) ** 2)
        rhs = np.sum(wts * np.abs(O.y_apply(st, u, s, +1.0)) ** 2)
        assert lhs < rhs
        u = un


# --------------------------------------------------------------- P2/P6: dense step
def _dense_ops(st, s):
    nz, nth = st.nz, st.nth
    X = np.zeros((nth * nz, nth * nz), dtype=complex)
    for m in range(nth):
        blk = (np.diag(st.xd[m]) + np.diag(st.xl[m, 1:], -1) + np.diag(st.xu[m, :-1], 1))
        X[m * nz:(m + 1) * nz, m * nz:(m + 1) * nz] = blk
    D = -2.0 * np.eye(nth) + np.eye(nth, k=1) + np.eye(nth, k=-1)
    if st.periodic:
        D[0, -1] = D[-1, 0] = 1.0
    Y = np.kron(D, np.eye(nz))
    I = np.eye(nth * nz)
    return X, Y, I


@pytest.mark.parametrize("periodic", [True, False])
def test_step_equals_dense_kronecker_solve(periodic):
    env = W.random_env(seed=21, zmax=120.0)
    width = W.TWO_PI if periodic else math.radians(60.0)
    grid = W.Grid(nz=7, ntheta=6, theta0=0.0, width=width, dr=4.0)
    st = O.setup(env, grid, 80.0)
    u = W.random_field(6, 7, seed=2)
    j = 2
    s = st.s(j)
    X, Y, I = _dense_ops(st, s)
    L = (I + st.beta_m * X) @ (I - s * Y)
    R = (I + st.beta_p * X) @ (I + s * Y)
    ref = np.linalg.solve(L, R @ u.ravel()).reshape(6, 7)
    assert O.rel_l2(O.step(st, u, j), ref) < 1e-13
    # the other factor order (X before Y on the right) is a different scheme
    R2 = (I + s * Y) @ (I + st.beta_p * X)
    alt = np.linalg.solve(L, R2 @ u.ravel()).reshape(6, 7)
    assert O.rel_l2(alt, ref) > 1e-6


def test_residual_of_step():
    env = W.wedge_env(zmax=3000.0)
    grid = W.Grid(nz=96, ntheta=40, theta0=0.0, width=W.TWO_PI, dr=10.0)
    st = O.setup(env, grid, 20.0)
    u = O.starter(st, 100.0)
    for j in range(0, 3):
        s = st.s(j)
        un = O.step(st, u, j)
        lhs = O.x_apply(st, O.y_apply(st, un, s, -1.0), st.beta_m)
        rhs = O.x_apply(st, O.y_apply(st, u, s, +1.0), st.beta_p)
        assert O.rel_l2(lhs, rhs) < 1e-13
        u = un


# --------------------------------------------------------------- P5/P7: symmetries
def test_azimuth_independent_medium_and_starter_give_independent_field():
    env = W.flat_layered_env()
    grid = W.Grid(nz=60, ntheta=16, theta0=0.0, width=W.TWO_PI, dr=5.0)
    st = O.setup(env, grid, 50.0)
    u0 = O.starter(st, 30.0)
    u = O.march(st, u0, 0, 40)
    assert np.abs(u - u[0:1]).max() < 1e-13 * np.abs(u).max()
    # and equals the march without azimuth coupling, by dense depth solves
    col = u0[0].copy()
    A = (np.eye(60) + st.beta_m * (np.diag(st.xd[0]) + np.diag(st.xl[0, 1:], -1)
                                   + np.diag(st.xu[0, :-1], 1)))
    Ap = (np.eye(60) + st.beta_p * (np.diag(st.xd[0]) + np.diag(st.xl[0, 1:], -1)
                                    + np.diag(st.xu[0, :-1], 1)))
    for _ in range(40):
        col = np.linalg.solve(A, Ap @ col)
    assert np.abs(u[5] - col).max() < 1e-12 * np.abs(col).max()


@pytest.mark.parametrize("shift", [1, 5])
def test_rotation_equivariance(shift):
    env = W.flat_layered_env()
    grid = W.Grid(nz=30, ntheta=12, theta0=0.0, width=W.TWO_PI, dr=5.0)
    st = O.setup(env, grid, 50.0)
    u0 = W.random_field(12, 30, seed=4)
    a = O.march(st, u0, 0, 6)
    b = O.march(st, np.roll(u0, shift, axis=0), 0, 6)
    assert np.abs(np.roll(a, shift, axis=0) - b).max() < 1e-13 * np.abs(a).max()


def test_resume_is_bitwise():
    env = W.wedge_env()
    grid = W.Grid(nz=40, ntheta=16, theta0=0.0, width=W.TWO_PI, dr=10.0)
    st = O.setup(env, grid, 30.0)
    u0 = O.starter(st, 100.0)
    full = O.march(st, u0, 0, 10)
    half = O.march(st, O.march(st, u0, 0, 5), 5, 5)
    assert np.array_equal(full, half)


def test_starter_shape_and_image():
    env = W.isovelocity_env()
    grid = W.Grid(nz=64, ntheta=4, theta0=0.0, width=W.TWO_PI, dr=5.0)
    st = O.setup(env, grid, 25.0)
    u0 = O.starter(st, 50.0)
    assert u0.shape == (4, 64)
    assert np.all(u0 == u0[0:1])
    peak = st.z[np.argmax(np.abs(u0[0]))]
    assert abs(peak - 50.0) <= st.dz
    # the surface image makes the starter odd about z = 0: a source at the
    # surface gives a zero field
    assert np.abs(O.starter(st, 0.0)).max() == 0.0


def test_node_exactly_on_the_bottom_is_water():
    # reading: a node is water iff z_l <= D(theta); with dz = 5 m node 24 sits
    # exactly on a 120 m bottom
    env = W.flat_layered_env(depth=120.0, zmax=200.0)
    grid = W.Grid(nz=39, ntheta=3, theta0=0.0, width=W.TWO_PI, dr=5.0)
    st = O.setup(env, grid, 30.0)
    assert st.dz == 5.0 and st.z[23] == 120.0
    assert st.water[0].sum() == 24


def test_pressure_hankel_factor_textbook_values():
    """p = u H0^(1)(k0 r): with k0 = 1 m^-1 (c0 = 2 pi m/s, f = 1 Hz) and
    dr = 1 m, step j has k0 r_j = j.  Tabulated J0, Y0 (Abramowitz & Stegun,
    Table 9.1): H0^(1)(1) = 0.7651976866 + 0.0882569642 i,
    H0^(1)(10) = -0.2459357645 + 0.0556711673 i.  Large argument:
    |H0^(1)(x)|^2 = 2/(pi x) (1 - 1/(8 x^2) + O(x^-4)) (A&S 9.2.28)."""
    env = W.isovelocity_env(c0=2.0 * math.pi)
    grid = W.Grid(nz=4, ntheta=3, theta0=0.0, width=W.TWO_PI, dr=1.0, precision=W.PREC_C128)
    st = O.setup(env, grid, 1.0)
    assert abs(st.k0 - 1.0) < 1e-15
    one = np.ones((3, 4), complex)
    h1 = O.pressure(st, one, 1)[0, 0]
    h10 = O.pressure(st, one, 10)[0, 0]
    assert abs(h1 - (0.7651976866 + 0.0882569642j)) < 1e-9
    assert abs(h10 - (-0.2459357645 + 0.0556711673j)) < 1e-9
    x = 1000.0
    hx = O.pressure(st, one, 1000)[0, 0]
    assert abs(abs(hx) ** 2 * math.pi * x / 2.0 - (1.0 - 1.0 / (8.0 * x * x))) < 1e-11
    with pytest.raises(ValueError):
        O.pressure(st, one, 0)


def _tl_plant_20logr(st, u, j):
    with np.errstate(divide="ignore"):
        return -20.0 * np.log10(np.abs(u)) + 20.0 * math.log10(st.r(j))


def _tl_plant_sign(st, u, j):
    with np.errstate(divide="ignore"):
        return 20.0 * np.log10(np.abs(u)) + 10.0 * math.log10(st.r(j))


def _tl_hankel_defect(tlfun):
    """Largest deviation of tl(u) + 20 log10|p| from its large-argument
    constant.  The pressure p = u H0^(1)(k0 r_j) is pinned above to the
    tables; with |H0^(1)(x)|^2 = 2/(pi x) (1 - 1/(8 x^2) + O(x^-4))
    (A&S 9.2.28) the loss of the envelope, -20 log10|u| + 10 log10 r (Tappert
    factor ~ r^-1/2, Sec. 2.1), differs from the loss of the pressure,
    -20 log10|p|, by 10 log10(2 / (pi k0)) + 10 log10(1 - 1/(8 x^2)) + O(x^-4),
    whatever u is."""
    env = W.isovelocity_env()
    grid = W.Grid(nz=16, ntheta=5, theta0=0.0, width=W.TWO_PI, dr=25.0, precision=W.PREC_C128)
    st = O.setup(env, grid, 60.0)
    u = W.random_field(5, 16, seed=11)
    worst = 0.0
    for j in (200, 1000, 4000, 20000):
        x = st.k0 * st.r(j)
        assert x > 1e3
        lhs = O.tl(st, u, j) + 20.0 * np.log10(np.abs(O.pressure(st, u, j)))
        const = 10.0 * math.log10(2.0 / (math.pi * st.k0)) + 10.0 * math.log10(1.0 - 1.0 / (8.0 * x * x))
        worst = max(worst, float(np.abs(lhs - const).max()))
    return worst


def test_tl_is_the_pressure_loss_up_to_the_hankel_constant():
    assert _tl_hankel_defect(O.tl) < 1e-9


@pytest.mark.parametrize("plant", [_tl_plant_20logr, _tl_plant_sign])
def test_tl_pin_catches_planted_mistakes(plant, monkeypatch):
    monkeypatch.setattr(O, "tl", plant)
    assert _tl_hankel_defect(O.tl) > 1.0


# --------------------------------------------------------------- depth grid vs the continuous waveguide
def _lowest_x_eigenvalues(st, k):
    n = st.nz
    a = np.diag(st.xd[0]) + np.diag(st.xl[0, 1:], -1) + np.diag(st.xu[0, :-1], 1)
    ev = np.linalg.eigvals(a)
    return np.sort(ev.real)[::-1][:k]


def _waveguide_defect(floor, nz, plant_extra_nodes=0):
    """Largest relative distance of the 4 highest eigenvalues of the oracle's
    X from the continuous ones, over the second-order bound; a plant moves
    the grid to dz = zmax / (Nz + conventional offset + plant_extra_nodes)."""
    zmax = 200.0
    env = dataclasses.replace(W.isovelocity_env(depth=zmax, c=1500.0), floor=floor)
    grid = W.Grid(nz=nz, ntheta=3, theta0=0.0, width=W.TWO_PI, dr=5.0, precision=W.PREC_C128)
    st = O.setup(env, grid, 25.0)
    if plant_extra_nodes:
        st.dz = zmax / (nz + (0 if floor == W.FLOOR_RIGID else 1) + plant_extra_nodes)
        st.z = st.dz * np.arange(1, nz + 1)
        st.water, st.rho, st.q, st.xl, st.xd, st.xu = st.medium(st.depth_at(st.r0))
    k = np.arange(1, 5)
    kz = ((k - 0.5) if floor == W.FLOOR_RIGID else k) * math.pi / zmax
    cont = -(kz / st.k0) ** 2
    rel = np.abs(_lowest_x_eigenvalues(st, 4) - cont) / np.abs(cont)
    # second order: (kz dz)^2 / 12 relative
    return float(np.max(rel / (0.2 * (kz * zmax / nz) ** 2)))


@pytest.mark.parametrize("floor", [W.FLOOR_RIGID, W.FLOOR_PRESSURE_RELEASE])
@pytest.mark.parametrize("extra", [1, -1])
def test_waveguide_pin_catches_a_shifted_floor(floor, extra):
    assert _waveguide_defect(floor, 200, plant_extra_nodes=extra) > 1.0


@pytest.mark.parametrize("floor", [W.FLOOR_RIGID, W.FLOOR_PRESSURE_RELEASE])
def test_depth_grid_converges_to_the_continuous_waveguide(floor):
    """An isovelocity layer 0 < z < zmax with u(0) = 0 and a rigid floor
    (du/dz = 0 at zmax) has the continuous modes sin(kz z) with
    kz = (k - 1/2) pi / zmax; a pressure-release floor (u(zmax) = 0) has
    kz = k pi / zmax.  X = (n^2 - 1) + k0^-2 d_zz then has the eigenvalues
    (n^2 - 1) - (kz / k0)^2.  The discrete X converges to them at second
    order only when the ghost rule's plane of symmetry (rigid: node Nz;
    pressure release: node Nz + 1) lies exactly at zmax, i.e. with the grid
    conventions dz = zmax/Nz (rigid) and zmax/(Nz + 1) (pressure release).
    One node too many or too few moves the floor by dz and the eigenvalues
    by O(1/Nz), 100x more than allowed here."""
    for nz in (200, 400):
        assert _waveguide_defect(floor, nz) < 1.0, nz
    # config 1: Nz = 64 nodes over a 200 m rigid-floored layer
    p = W.config1()
    st = O.setup(p.env, p.grid, p.f_hz)
    assert p.env.floor == W.FLOOR_RIGID and st.dz == 3.125 and st.z[-1] == p.env.zmax


# --------------------------------------------------------------- range-dependent depth
def test_equal_range_rows_reduce_to_range_independent():
    base = W.random_env(21, floor=W.FLOOR_RIGID)
    rd = dataclasses.replace(base, bathy_depth=base.bathy_depth * 3, bathy_nr=3,
                             bathy_r0=10.0, bathy_dr=40.0)
    g = W.Grid(nz=40, ntheta=9, theta0=0.1, width=W.TWO_PI, dr=7.0, precision=W.PREC_C128)
    u0 = W.random_field(9, 40, seed=5)
    a = O.march(O.setup(base, g, 45.0), u0, 0, 30)
    b = O.march(O.setup(rd, g, 45.0), u0, 0, 30)
    assert np.array_equal(a, b)


def test_range_dependent_step_uses_the_medium_at_the_next_range():
    """Fig. 2 advances r, then updates the matrices: the step j -> j+1 is the
    range-independent step of the medium at r_{j+1}.  Rows one range step
    apart put row j+1 exactly there (and the last row beyond the rows)."""
    base = W.random_env(22)
    nr, nb = 5, len(base.bathy_theta)
    rng = np.random.default_rng(3)
    rows = rng.uniform(0.05 * base.zmax, 0.95 * base.zmax, (nr, nb))
    dr, r0 = 6.0, 18.0
    rd = dataclasses.replace(base, bathy_depth=tuple(rows.ravel()), bathy_nr=nr,
                             bathy_r0=r0, bathy_dr=dr)
    g = W.Grid(nz=50, ntheta=8, theta0=0.0, width=W.TWO_PI, dr=dr, r0=r0, precision=W.PREC_C128)
    st = O.setup(rd, g, 40.0)
    u = u0 = W.random_field(8, 50, seed=6)
    for j in range(7):
        row = rows[min(j + 1, nr - 1)]
        sj = O.setup(dataclasses.replace(base, bathy_depth=tuple(row)), g, 40.0)
        u = O.step(sj, u, j)
    got = O.march(st, u0, 0, 7)
    assert np.array_equal(got, u)
    # the columns really change their water nodes along the way
    counts = {tuple(st.medium(st.depth_at(st.r(j)))[0].sum(axis=1)) for j in range(1, 5)}
    assert len(counts) == 4


def test_depth_is_linear_in_range_between_rows():
    base = W.random_env(23)
    a = np.array(base.bathy_depth)
    b = a[::-1].copy()
    rd = dataclasses.replace(base, bathy_depth=tuple(np.concatenate([a, b])), bathy_nr=2,
                             bathy_r0=100.0, bathy_dr=50.0)
    st = O.setup(rd, W.Grid(nz=20, ntheta=16, theta0=0.0, width=W.TWO_PI, dr=5.0), 30.0)
    da = O.interp_bathy(st.theta, base.bathy_theta, a)
    db = O.interp_bathy(st.theta, base.bathy_theta, b)
    assert np.array_equal(st.depth_at(100.0), da) and np.array_equal(st.depth_at(0.0), da)
    assert np.array_equal(st.depth_at(150.0), db) and np.array_equal(st.depth_at(1e6), db)
    assert np.allclose(st.depth_at(125.0), 0.5 * (da + db), rtol=1e-14, atol=1e-12)
    assert np.allclose(st.depth_at(110.0), 0.8 * da + 0.2 * db, rtol=1e-14, atol=1e-12)


# --------------------------------------------------------------- range-dependent water (reading A25)
def test_equal_water_rows_reduce_to_range_independent():
    base = W.random_env(31, floor=W.FLOOR_RIGID)
    rd = dataclasses.replace(base, ssp_c=base.ssp_c * 4, ssp_nr=4, ssp_r0=5.0, ssp_dr=20.0)
    g = W.Grid(nz=40, ntheta=9, theta0=0.1, width=W.TWO_PI, dr=7.0, precision=W.PREC_C128)
    u0 = W.random_field(9, 40, seed=5)
    a = O.march(O.setup(base, g, 45.0), u0, 0, 25)
    b = O.march(O.setup(rd, g, 45.0), u0, 0, 25)
    assert np.array_equal(a, b)


def test_water_rows_are_a_stair_step_in_range():
    """A profile holds from its row's range until the next row's: with rows
    at 0, 30, 60 m and dr = 5 m the step j -> j+1 (medium at r_{j+1} =
    5 (j+1)) uses row 0 for j = 0..4, row 1 from j = 5 (r_6 = 30 exactly,
    the row's own range) to j = 10, and row 2 (the last) from j = 11 on.  The
    march equals range-independent marches of each profile over those steps,
    composed."""
    base = W.random_env(32)
    nz_s = len(base.ssp_z)
    rng = np.random.default_rng(4)
    rows = rng.uniform(1470.0, 1560.0, (3, nz_s))
    rd = dataclasses.replace(base, ssp_c=tuple(rows.ravel()), ssp_nr=3, ssp_r0=0.0, ssp_dr=30.0)
    g = W.Grid(nz=36, ntheta=8, theta0=0.0, width=W.TWO_PI, dr=5.0, precision=W.PREC_C128)
    u0 = W.random_field(8, 36, seed=7)
    got = O.march(O.setup(rd, g, 50.0), u0, 0, 16)
    u = u0
    for row, j0, j1 in ((0, 0, 5), (1, 5, 11), (2, 11, 16)):
        seg = O.setup(dataclasses.replace(base, ssp_c=tuple(rows[row])), g, 50.0)
        u = O.march(seg, u, j0, j1 - j0)
    assert np.array_equal(got, u)
    # and the three profiles really differ in their effect
    alone = O.march(O.setup(dataclasses.replace(base, ssp_c=tuple(rows[0])), g, 50.0), u0, 0, 16)
    assert O.rel_l2(alone, got) > 1e-3


def test_water_rows_with_depth_rows():
    """Water rows and depth rows together: the step j -> j+1 takes the depth
    interpolated at r_{j+1} and the profile in force there, each as when
    alone."""
    e = W.random_ssp_range_env(33, nr=4, row_dr=25.0, depth_rows=4)
    g = W.Grid(nz=44, ntheta=10, theta0=0.0, width=W.TWO_PI, dr=6.0, precision=W.PREC_C128)
    st = O.setup(e, g, 55.0)
    u = u0 = W.random_field(10, 44, seed=8)
    for j in range(14):
        r = st.r(j + 1)
        row = min(int(r // 25.0), 3)
        depth_rows = np.asarray(e.bathy_depth).reshape(e.bathy_nr, -1)
        # a range-independent setup with this step's profile and depth
        dcol = st.depth_at(r)
        sj = O.setup(dataclasses.replace(e, ssp_c=tuple(st.ssp_rows[row]), ssp_nr=0, bathy_nr=0,
                                         bathy_depth=tuple(depth_rows[0])), g, 55.0)
        sj.water, sj.rho, sj.q, sj.xl, sj.xd, sj.xu = sj.medium(dcol)
        u = O.step(sj, u, j)
    assert np.array_equal(O.march(st, u0, 0, 14), u)

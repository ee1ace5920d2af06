"""The azimuth solve of Eq. (6)/(8) by the factorisation the HIP azimuth pass
uses, written out in NumPy on the CPU (no GPU, no product code).

[I - s D_theta] is circulant (periodic) or Toeplitz (sector) with constant
coefficients and factors as c (1 - rho S)(1 - rho S^-1), c = s / rho,
s rho^2 - (1 + 2s) rho + s = 0, |rho| < 1.  Two ways to use it:

  direct:  u = (rho/s) (1 - rho S^-1)^-1 (1 - rho S)^-1 v
  defect:  u = v + e,  e = rho (1 - rho S^-1)^-1 (1 - rho S)^-1 D_theta v

Both are exact in exact arithmetic.  On a field rough in azimuth the highest
modes leave the solve 1 + 4 sigma times smaller than they enter it, so the
defect form, whose two terms are each as large as v, cancels about
log10(4 sigma) digits, while the direct form does not.  These tests check
the direct form against dense LAPACK solves and show the defect form's loss
on the rough sector input of the GPU parity suite (sigma_0 = 204).
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _rho_and_scale(sigma):
    s = 1j * sigma
    den = 1.0 + 2.0 * s + np.sqrt(1.0 + 4.0 * s)
    return 2.0 * s / den, 2.0 / den          # rho, rho / s


def _two_recurrences(t, rho, periodic):
    """x = (1 - rho S^-1)^-1 (1 - rho S)^-1 t along axis 0, cyclic wraps
    closed by 1 / (1 - rho^N) (the rank-one correction of each cyclic
    bidiagonal factor)."""
    n = t.shape[0]
    e = np.zeros_like(t[0])
    for m in range(n):
        e = rho * e + t[m]
    y = np.empty_like(t)
    prev = e / (1.0 - rho ** n) if periodic else np.zeros_like(e)
    for m in range(n):
        prev = t[m] + rho * prev
        y[m] = prev
    e = np.zeros_like(t[0])
    for m in range(n - 1, -1, -1):
        e = rho * e + y[m]
    nxt = e / (1.0 - rho ** n) if periodic else np.zeros_like(e)
    x = np.empty_like(t)
    for m in range(n - 1, -1, -1):
        nxt = y[m] + rho * nxt
        x[m] = nxt
    if not periodic:
        # sector: c (1 - rho L)(1 - rho U) = B - s rho e_0 e_0^T; the
        # Sherman-Morrison correction of that first row
        mm = np.arange(n)[:, None]
        kc = rho ** 2 * x[0] / (1.0 - rho ** (2 * n + 2))
        x = x - kc[None, :] * (rho ** mm - rho ** (2 * n - mm))
    return x


def azimuth_solve(v, sigma, periodic, form):
    rho, cs = _rho_and_scale(sigma)
    if form == "direct":
        return cs * _two_recurrences(v, rho, periodic)
    if periodic:
        t = np.roll(v, 1, 0) - 2.0 * v + np.roll(v, -1, 0)
    else:
        t = -2.0 * v
        t[1:] += v[:-1]
        t[:-1] += v[1:]
    return v + rho * _two_recurrences(t, rho, periodic)


def _dense(n, sigma, periodic):
    s = 1j * sigma
    a = (1.0 + 2.0 * s) * np.eye(n, dtype=complex) - s * (np.eye(n, k=1) + np.eye(n, k=-1))
    if periodic:
        a[0, -1] -= s
        a[-1, 0] -= s
    return a


@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("n", [1, 3, 7, 64, 90])
@pytest.mark.parametrize("sigma", [1e-6, 0.3, 40.0, 613.0])
def test_direct_factorised_solve_matches_dense(periodic, n, sigma):
    if periodic and n < 3:
        return
    rng = np.random.default_rng(n)
    v = rng.standard_normal((n, 5)) + 1j * rng.standard_normal((n, 5))
    ref = np.linalg.solve(_dense(n, sigma, periodic), v)
    got = azimuth_solve(v, sigma, periodic, "direct")
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-13


def test_defect_form_loses_digits_on_a_rough_sector_field_and_the_direct_form_does_not():
    """The rough sector case of the GPU parity suite (90 degrees, 64
    azimuths, 50 Hz, dr = 10 m), 4 steps from white noise: depth pass as the
    oracle's, then each azimuth form; the oracle's Thomas solve agrees with
    dense solves to ~1e-15 on these systems."""
    env = W.wedge_env(zmax=2400.0)
    grid = W.Grid(nz=192, ntheta=64, theta0=2.0, width=math.radians(90.0), dr=10.0,
                  precision=W.PREC_C128)
    st = O.setup(env, grid, 50.0)
    assert abs(st.s(0)) > 200.0
    u0 = W.random_field(64, 192, seed=sum(map(ord, "sector_90")) % 1000)
    ref, ud, ue = u0.copy(), u0.copy(), u0.copy()
    for j in range(4):
        s = st.s(j)

        def depth(u):
            xl, xd, xu = st.x_at(j)
            rhs = O.x_apply(st, O.y_apply(st, u, s), st.beta_p, (xl, xd, xu))
            return O.thomas(st.beta_m * xl, 1.0 + st.beta_m * xd, st.beta_m * xu, rhs)

        ref = O.step(st, ref, j)
        ud = azimuth_solve(depth(ud), s.imag, False, "direct")
        ue = azimuth_solve(depth(ue), s.imag, False, "defect")
    assert O.rel_l2(ud, ref) < 5e-14
    assert O.rel_l2(ue, ref) > 5e-13

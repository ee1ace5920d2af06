"""The cyclic-reduction form of the azimuth solve (Eq. (6)/(8)) that the
PCR azimuth kernel runs, emulated in NumPy complex128 and checked against
dense LAPACK solves of [I - s D_theta] u = v: periodic lines, and sectors
through the odd extension of period 2 Ntheta + 2 (zero ghost azimuths),
over the range of sigma the configs reach (1e-5 far from the source to
613 at the first step of the worst sector request)."""
import numpy as np
import pytest


def dense_solve(v, sigma, periodic):
    n = v.shape[0]
    s = 1j * sigma
    A = np.eye(n, dtype=complex) * (1 + 2 * s)
    for m in range(n):
        for mm in (m - 1, m + 1):
            if periodic:
                A[m, mm % n] -= s
            elif 0 <= mm < n:
                A[m, mm] -= s
    return np.linalg.solve(A, v)


def pcr_solve(v, sigma, periodic):
    """v: (ntheta, ndepth).  Returns (u, levels)."""
    nt = v.shape[0]
    s = 1j * sigma
    b, a = 1 + 2 * s, -s
    V = v.astype(complex).copy()
    P = nt if periodic else 2 * nt + 2

    def at(i):
        if periodic or i < nt:
            return V[i]
        if i == nt or i == P - 1:
            return np.zeros_like(V[0])
        return -V[2 * nt - i]

    dist, levels = 1 % P, 0
    while abs(a) ** 2 > 2.0 ** -120 * abs(b) ** 2:
        k = -a / b
        new = np.empty_like(V)
        for m in range(nt):
            lo, hi = m - dist, m + dist
            lo += P if lo < 0 else 0
            hi -= P if hi >= P else 0
            new[m] = V[m] + k * (at(lo) + at(hi))
        V = new
        b = b + 2 * k * a
        a = k * a
        dist = (2 * dist) % P
        levels += 1
        assert levels < 64
    return V / b, levels


@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("nt", [1, 2, 3, 7, 16, 32, 33, 64, 100])
@pytest.mark.parametrize("sigma", [1e-5, 0.03, 1.0, 40.0, 613.0])
def test_pcr_equals_dense_solve(periodic, nt, sigma):
    if periodic and nt < 3:
        pytest.skip("a periodic line has at least 3 azimuths")
    rng = np.random.default_rng(nt * 7 + int(sigma * 10))
    v = rng.standard_normal((nt, 3)) + 1j * rng.standard_normal((nt, 3))
    u, levels = pcr_solve(v, sigma, periodic)
    ref = np.stack([dense_solve(v[:, c], sigma, periodic) for c in range(3)], axis=1)
    # two backward-stable FP64 solves differ by about cond * eps, and
    # cond(I - s D_theta) <= 1 + 4 sigma
    assert np.linalg.norm(u - ref) <= 4 * (1 + 4 * sigma) * 2.0 ** -52 * np.linalg.norm(ref)
    # the coupling decays quadratically: few levels far from the source
    assert levels <= {1e-5: 3, 0.03: 5, 1.0: 8, 40.0: 11, 613.0: 14}[sigma]


def test_pcr_sector_is_the_odd_restriction_of_the_extended_circle():
    """A sector line with zero ghosts equals the full line of period
    2 Ntheta + 2 with the data odd about the ghosts (the reading the kernel
    uses for sectors): checked with a dense periodic solve of the extension."""
    nt, sigma = 9, 7.5
    rng = np.random.default_rng(3)
    v = rng.standard_normal(nt) + 1j * rng.standard_normal(nt)
    ext = np.concatenate([v, [0], -v[::-1], [0]])
    u_ext = dense_solve(ext, sigma, True)
    assert np.allclose(u_ext[:nt], dense_solve(v, sigma, False), rtol=0, atol=1e-14)
    assert abs(u_ext[nt]) < 1e-14 and abs(u_ext[-1]) < 1e-14


def test_planted_mistakes_fail():
    """A wrong coefficient update or a lost sign in the mirror must fail."""
    nt, sigma = 12, 20.0
    rng = np.random.default_rng(5)
    v = rng.standard_normal((nt, 1)) + 1j * rng.standard_normal((nt, 1))
    ref = dense_solve(v[:, 0], sigma, False)[:, None]
    good, _ = pcr_solve(v, sigma, False)
    assert np.linalg.norm(good - ref) < 1e-12 * np.linalg.norm(ref)
    # mirror without the sign flip (even instead of odd extension: a Neumann edge)
    nt_ = nt
    P = 2 * nt_ + 2
    s = 1j * sigma
    b, a = 1 + 2 * s, -s
    V = v.astype(complex).copy()
    dist = 1
    while abs(a) ** 2 > 2.0 ** -120 * abs(b) ** 2:
        k = -a / b

        def at(i):
            if i < nt_:
                return V[i]
            if i == nt_ or i == P - 1:
                return np.zeros_like(V[0])
            return V[2 * nt_ - i]
        V = np.stack([V[m] + k * (at((m - dist) % P) + at((m + dist) % P)) for m in range(nt_)])
        b, a = b + 2 * k * a, k * a
        dist = (2 * dist) % P
    assert np.linalg.norm(V / b - ref) > 1e-3 * np.linalg.norm(ref)

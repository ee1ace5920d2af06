"""Closed-form solution of the split Crank-Nicolson march for a separable
problem (azimuth-independent constant n^2, uniform density, periodic azimuth):
X = q I + h D2 has sine eigenvectors and D_theta has Fourier modes, so each
mode is multiplied per step by G_k H_q(j) with
  G_k = (1 + beta_+ lambda_k) / (1 + beta_- lambda_k),
  H_q(j) = (1 + s_j mu_q) / (1 - s_j mu_q).
Independent of any finite-difference sweep; used to pin the oracle and the
HIP path."""
import math

import numpy as np

import oracle as O
import workloads as W


def modal_march(st, u0, nsteps, floor, coupled=True):
    """Separable problem (theta-independent constant q, uniform density):
    X = q I + h D2 with sine eigenvectors, D_theta with Fourier modes.
    coupled=False: the N x 2D march (Y = 0), every H_q = 1; then the azimuth
    transform is the identity and any azimuth grid (sector too) qualifies."""
    nz, nth = st.nz, st.nth
    l = np.arange(1, nz + 1)
    k = np.arange(1, nz + 1)
    if floor == W.FLOOR_RIGID:
        ang = (k - 0.5) * math.pi / nz
    else:
        ang = k * math.pi / (nz + 1)
    phi = np.sin(np.outer(l, ang))                  # phi[l, k]
    c0 = st.env.c0
    n2 = (c0 / st.env.ssp_c[0]) ** 2 * (1 + 1j * O.ETA * st.env.atten_w) ** 2
    k0 = 2 * math.pi * st.f / c0
    h = 1.0 / (k0 * st.dz) ** 2
    lam = (n2 - 1.0) - 4.0 * h * np.sin(ang / 2) ** 2
    kap = k0 * st.dr
    G = (1 + (1 + 1j * kap) / 4 * lam) / (1 + (1 - 1j * kap) / 4 * lam)
    qq = np.arange(nth)
    mu = -4.0 * np.sin(math.pi * qq / nth) ** 2
    cq = np.fft.fft(u0, axis=0) / nth               # cq[q, l]
    ck = np.linalg.solve(phi, cq.T)                 # ck[k, q]
    fac = np.ones(nth, dtype=complex)
    for j in range(nsteps if coupled else 0):
        r = st.r0 + (j + 1) * st.dr
        s = 1j * st.dr / (4 * k0 * r * r * (2 * math.pi / nth) ** 2)
        fac *= (1 + s * mu) / (1 - s * mu)
    ck = ck * (G[:, None] ** nsteps) * fac[None, :]
    uq = phi @ ck                                    # uq[l, q]
    return (np.fft.ifft(uq.T, axis=0) * nth)



"""Complex128 oracle of the split Crank-Nicolson range march (Eq. (4)).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Plain NumPy, complex128 throughout, no blocking, fusion or reordering beyond
what the equations state.  Every function names the passage it follows.  The
paper leaves the discretisation of X and Y, the boundary conditions, the
starter and the medium model unstated; the readings used here are listed in the
repository's design notes (A1-A21) and are repeated briefly where they apply.

Parity status: every function here is pinned by tests under `tests/`
(closed-form modal march, energy identity, dense solves, FFT circulant solve,
flux-continuity of the density-weighted operator, azimuth independence,
rotation equivariance, residual).  The full-size wedge fields (config 2/4/5
environments) are not pinned by any value the paper prints - the paper prints
none - only through those checks on small analogues of the same code.
"""
from __future__ import annotations

import math

import numpy as np

FLOOR_PRESSURE_RELEASE = 0
FLOOR_RIGID = 1
MODE_NX2D = 1

#: dB-per-wavelength to imaginary wavenumber fraction: k = k_r (1 + i*ETA*a)
#: with a in dB/lambda, because a = 20*log10(e) * k_i * lambda.
ETA = 1.0 / (40.0 * math.pi * math.log10(math.e))

__all__ = [
    "ETA", "Setup", "setup", "is_periodic", "interp_ssp", "interp_bathy",
    "thomas", "periodic_thomas_sm", "apply_tridiag", "d_theta", "y_apply", "x_apply",
    "step", "march", "starter", "tl", "pressure", "rel_l2",
]


def is_periodic(width: float) -> bool:
    """A grid whose azimuth width is the full circle is periodic (Fig. 1
    shows one sector; a full 360-degree grid closes on itself)."""
    return width >= 2.0 * math.pi * (1.0 - 1e-12)


def interp_ssp(z: np.ndarray, zs, cs) -> np.ndarray:
    """Piecewise-linear sound speed c(z), constant beyond the sample ends."""
    zs = np.asarray(zs, dtype=np.float64)
    cs = np.asarray(cs, dtype=np.float64)
    if zs.size == 1:
        return np.full_like(z, cs[0])
    return np.interp(z, zs, cs)


def interp_bathy(theta: np.ndarray, ths, ds) -> np.ndarray:
    """Water depth D(theta): periodic piecewise-linear through the samples."""
    ths = np.asarray(ths, dtype=np.float64)
    ds = np.asarray(ds, dtype=np.float64)
    if ths.size == 1:
        return np.full_like(theta, ds[0])
    t = ths[0] + np.mod(theta - ths[0], 2.0 * math.pi)
    xp = np.concatenate([ths, [ths[0] + 2.0 * math.pi]])
    fp = np.concatenate([ds, [ds[0]]])
    return np.interp(t, xp, fp)


class Setup:
    """Grid, medium and depth-operator coefficients of one problem.

    Depth operator X (reading A1, A7, A9): for column m and depth node l,
        (X u)_l = q_l u_l + h [Lm_l u_{l-1} - (Lm_l + Lp_l) u_l + Lp_l u_{l+1}]
    with q = n^2 - 1, h = (k0 dz)^-2, density weights
        Lm_l = 2 rho_l / (rho_{l-1} + rho_l),  Lp_l = 2 rho_l / (rho_l + rho_{l+1}),
    surface u_0 = 0, pressure-release floor u_{Nz+1} = 0 or rigid floor
    u_{Nz+1} = u_{Nz-1}.  Stored as three diagonals xl, xd, xu of shape
    (Ntheta, Nz): row l of column m is xl*u_{l-1} + xd*u_l + xu*u_{l+1}.
    """

    def __init__(self, env, grid, f_hz: float):
        self.env, self.grid, self.f = env, grid, float(f_hz)
        nz, nth = int(grid.nz), int(grid.ntheta)
        self.nz, self.nth = nz, nth
        self.k0 = 2.0 * math.pi * self.f / env.c0
        # N x 2D ("weak 3D", Sec. 1): no coupling between azimuths, Y = 0
        self.nx2d = int(getattr(grid, "mode", 0)) == MODE_NX2D
        # depth nodes z_l = l dz, l = 1..Nz (reading A9)
        if env.floor == FLOOR_RIGID:
            self.dz = env.zmax / nz
        else:
            self.dz = env.zmax / (nz + 1)
        self.z = self.dz * np.arange(1, nz + 1, dtype=np.float64)
        # azimuth nodes (reading A10)
        self.periodic = is_periodic(grid.width)
        if self.periodic:
            self.dth = 2.0 * math.pi / nth
            self.theta = grid.theta0 + self.dth * np.arange(nth)
        else:
            self.dth = grid.width / (nth + 1)
            self.theta = grid.theta0 - 0.5 * grid.width + self.dth * np.arange(1, nth + 1)
        self.dr = float(grid.dr)
        self.r0 = float(grid.r0)
        # water depth per azimuth column: D(theta_m), or with range nodes
        # (reading A22) D(r_i, theta_m) at r_i = bathy_r0 + i bathy_dr, each
        # row periodic piecewise linear in theta, linear in r between rows and
        # constant beyond the first and last row
        nr = int(getattr(env, "bathy_nr", 0))
        self.range_dependent = nr >= 2
        nb = len(env.bathy_theta)
        if self.range_dependent:
            rows = np.asarray(env.bathy_depth, dtype=np.float64).reshape(nr, nb)
            self.bathy_r = env.bathy_r0 + env.bathy_dr * np.arange(nr, dtype=np.float64)
            self.dcol = np.stack([interp_bathy(self.theta, env.bathy_theta, rows[i])
                                  for i in range(nr)], axis=1)          # (Ntheta, nr)
        # water sound speed: one profile, or (reading A25) profiles c(r_i, z)
        # on range rows r_i = ssp_r0 + i ssp_dr, each holding from its range
        # until the next row's (stair-step in range; the first row also
        # before it)
        nsr = int(getattr(env, "ssp_nr", 0))
        nsz = len(env.ssp_z)
        self.ssp_rows = np.asarray(env.ssp_c, dtype=np.float64).reshape(max(nsr, 1), nsz)
        self.ssp_range_dependent = nsr >= 2
        if self.ssp_range_dependent:
            self.ssp_r = env.ssp_r0 + env.ssp_dr * np.arange(nsr, dtype=np.float64)
        self.any_range = self.range_dependent or self.ssp_range_dependent
        # the medium at r_0 (the only one when nothing depends on range)
        self.water, self.rho, self.q, self.xl, self.xd, self.xu = self.medium(
            self.depth_at(self.r0), self.ssp_row_at(self.r0))
        self._xcache = {}
        # Eq. (4): delta = i k0 dr; 1 + (1/4 +- delta/4) X = I + beta_pm X
        self.beta_p = (1.0 + 1j * self.k0 * self.dr) / 4.0
        self.beta_m = (1.0 - 1j * self.k0 * self.dr) / 4.0

    def medium(self, depth: np.ndarray, ssp_row: int = 0):
        """Medium and depth operator for water depths D_m of the columns and
        the water profile of range row `ssp_row` (readings A7, A8, A9, A25):
        water iff z_l <= D_m.  Returns water, rho, q = n^2 - 1 and the
        diagonals xl, xd, xu of X, each (Ntheta, Nz)."""
        env = self.env
        water = self.z[None, :] <= depth[:, None]
        cw = interp_ssp(self.z, env.ssp_z, self.ssp_rows[ssp_row])
        c = np.where(water, cw[None, :], env.c_b)
        rho = np.where(water, env.rho_w, env.rho_b).astype(np.float64)
        att = np.where(water, env.atten_w, env.atten_b)
        n2 = (env.c0 / c) ** 2 * (1.0 + 1j * ETA * att) ** 2
        q = n2 - 1.0
        # density weights with ghost densities rho_0 = rho_1, rho_{Nz+1} = rho_Nz
        rpad = np.concatenate([rho[:, :1], rho, rho[:, -1:]], axis=1)
        lm = 2.0 * rpad[:, 1:-1] / (rpad[:, :-2] + rpad[:, 1:-1])
        lp = 2.0 * rpad[:, 1:-1] / (rpad[:, 1:-1] + rpad[:, 2:])
        self.h = 1.0 / (self.k0 * self.dz) ** 2
        h = self.h
        xl = (h * lm).astype(np.complex128)
        xu = (h * lp).astype(np.complex128)
        xd = q - h * (lm + lp)
        xl[:, 0] = 0.0                      # surface: u_0 = 0
        if env.floor == FLOOR_RIGID:        # u_{Nz+1} = u_{Nz-1}
            xl[:, -1] = xl[:, -1] + xu[:, -1]
        xu[:, -1] = 0.0
        return water, rho, q, xl, xd, xu

    def depth_at(self, r: float) -> np.ndarray:
        """Water depth of every column at range r (reading A22): linear
        interpolation between the range rows (the library routine), constant
        beyond the first and last row; D(theta_m) when there are no rows."""
        if not self.range_dependent:
            return interp_bathy(self.theta, self.env.bathy_theta, self.env.bathy_depth)
        return np.array([np.interp(r, self.bathy_r, self.dcol[m]) for m in range(self.nth)])

    def ssp_row_at(self, r: float) -> int:
        """Water profile row in force at range r (reading A25): the last row
        whose range is <= r (a library search over the row ranges), row 0
        before the first."""
        if not self.ssp_range_dependent:
            return 0
        return max(int(np.searchsorted(self.ssp_r, r, side="right")) - 1, 0)

    def x_at(self, j: int):
        """Diagonals (xl, xd, xu) of X for the step j -> j+1: the medium at
        r_{j+1} on both sides of Eq. (4) (reading A3: Fig. 2 advances r, then
        updates both matrices)."""
        if not self.any_range:
            return self.xl, self.xd, self.xu
        if j not in self._xcache:
            if len(self._xcache) > 64:
                self._xcache.clear()
            r = self.r(j + 1)
            self._xcache[j] = self.medium(self.depth_at(r), self.ssp_row_at(r))[3:]
        return self._xcache[j]

    def r(self, j: int) -> float:
        """Range of step j: r_j = r0 + j dr (Fig. 2: r starts at 0 and grows
        by dr each step)."""
        return self.r0 + j * self.dr

    def s(self, j: int) -> complex:
        """Azimuth coefficient of the step j -> j+1: (delta/4) Y = s_j D_theta
        with Y = (k0 r)^-2 d^2/dtheta^2 discretised by the 3-point second
        difference, evaluated at r_{j+1} on both sides of Eq. (4) (reading A3:
        Fig. 2 advances r before the matrices are updated).  Zero in the
        N x 2D mode, where Y is dropped."""
        if self.nx2d:
            return 0.0 + 0.0j
        r = self.r(j + 1)
        return 1j * self.dr / (4.0 * self.k0 * r * r * self.dth * self.dth)


def setup(env, grid, f_hz: float) -> Setup:
    return Setup(env, grid, f_hz)


# ------------------------------------------------------------------ solvers
def thomas(a: np.ndarray, b: np.ndarray, c: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Solve tridiagonal systems along the LAST axis without pivoting
    (reading A17): row i is a_i x_{i-1} + b_i x_i + c_i x_{i+1} = d_i, with
    a_0 and c_{n-1} ignored.  Leading axes are independent systems.
    Forward elimination then back substitution (the Thomas algorithm)."""
    n = d.shape[-1]
    a, b, c, d = np.broadcast_arrays(a, b, c, d)
    cp = np.empty(d.shape, dtype=np.complex128)
    dp = np.empty(d.shape, dtype=np.complex128)
    piv = b[..., 0]
    cp[..., 0] = c[..., 0] / piv
    dp[..., 0] = d[..., 0] / piv
    for i in range(1, n):
        piv = b[..., i] - a[..., i] * cp[..., i - 1]
        cp[..., i] = c[..., i] / piv
        dp[..., i] = (d[..., i] - a[..., i] * dp[..., i - 1]) / piv
    x = np.empty(d.shape, dtype=np.complex128)
    x[..., n - 1] = dp[..., n - 1]
    for i in range(n - 2, -1, -1):
        x[..., i] = dp[..., i] - cp[..., i] * x[..., i + 1]
    return x


def periodic_thomas_sm(a, b, c, d: np.ndarray) -> np.ndarray:
    """Solve cyclic tridiagonal systems along the LAST axis: row i is
    a_i x_{i-1} + b_i x_i + c_i x_{i+1} = d_i with indices mod n, so
    a_0 multiplies x_{n-1} and c_{n-1} multiplies x_0.

    Sherman-Morrison: M = T + u v^T with u = (g, 0..0, c_{n-1}) and
    v = (1, 0..0, a_0/g), g = -b_0, where T is tridiagonal with
    b_0 -> b_0 - g and b_{n-1} -> b_{n-1} - c_{n-1} a_0 / g.  Then
    x = y - z (v.y)/(1 + v.z) with T y = d and T z = u."""
    a, b, c, d = np.broadcast_arrays(a, b, c, d)
    a = a.astype(np.complex128)
    b = b.astype(np.complex128).copy()
    c = c.astype(np.complex128)
    n = d.shape[-1]
    if n < 3:
        raise ValueError("cyclic system needs n >= 3")
    alpha = c[..., n - 1]        # corner multiplying x_0 in row n-1
    beta = a[..., 0]             # corner multiplying x_{n-1} in row 0
    g = -b[..., 0]
    b[..., 0] = b[..., 0] - g
    b[..., n - 1] = b[..., n - 1] - alpha * beta / g
    y = thomas(a, b, c, d)
    u = np.zeros(d.shape, dtype=np.complex128)
    u[..., 0] = g
    u[..., n - 1] = alpha
    z = thomas(a, b, c, u)
    vy = y[..., 0] + beta * y[..., n - 1] / g
    vz = z[..., 0] + beta * z[..., n - 1] / g
    return y - z * (vy / (1.0 + vz))[..., None]


def apply_tridiag(lo, di, up, x: np.ndarray) -> np.ndarray:
    """y_i = lo_i x_{i-1} + di_i x_i + up_i x_{i+1} along the last axis, with
    x_{-1} = x_n = 0 (boundary terms are already folded into the diagonals)."""
    y = di * x
    y[..., 1:] += lo[..., 1:] * x[..., :-1]
    y[..., :-1] += up[..., :-1] * x[..., 1:]
    return y


# ------------------------------------------------------------------ operators
def d_theta(st: Setup, u: np.ndarray) -> np.ndarray:
    """3-point second difference in azimuth (axis 0 of the (Ntheta, Nz)
    field): periodic for the full circle, zero ghost azimuths for a sector."""
    if st.periodic:
        return np.roll(u, 1, axis=0) - 2.0 * u + np.roll(u, -1, axis=0)
    out = -2.0 * u
    out[1:] += u[:-1]
    out[:-1] += u[1:]
    return out


def y_apply(st: Setup, u: np.ndarray, s: complex, sign: float = 1.0) -> np.ndarray:
    """(I + sign * s_j D_theta) u  -- the azimuth factor of Eq. (4)."""
    return u + sign * s * d_theta(st, u)


def x_apply(st: Setup, w: np.ndarray, beta: complex, x=None) -> np.ndarray:
    """(I + beta X) w, X applied down every azimuth column (Eq. (4)); X is
    the medium's at r_0 unless the diagonals x = (xl, xd, xu) are given."""
    xl, xd, xu = (st.xl, st.xd, st.xu) if x is None else x
    return w + beta * apply_tridiag(xl, xd, xu, w)


def step(st: Setup, u: np.ndarray, j: int) -> np.ndarray:
    """One range step u^j -> u^{j+1} of Eq. (4) by the two-step procedure:
      RHS = [I + beta_+ X][I + s_j D] u^j          (Eq. (4), right side;
                                                    reading A4: Y first)
      [I + beta_- X] v = RHS                         (Eq. (5)/(7), per azimuth)
      [I - s_j D] u^{j+1} = v                        (Eq. (6)/(8), per depth)"""
    s = st.s(j)
    xl, xd, xu = st.x_at(j)
    w = y_apply(st, u, s, +1.0)
    rhs = x_apply(st, w, st.beta_p, (xl, xd, xu))
    v = thomas(st.beta_m * xl, 1.0 + st.beta_m * xd, st.beta_m * xu, rhs)
    if st.nx2d:
        return v                     # [I - 0 D] u^{j+1} = v
    # azimuth systems: one per depth, unknowns along theta -> move theta last
    vt = v.T
    nth = st.nth
    lo = np.full(nth, -s, dtype=np.complex128)
    di = np.full(nth, 1.0 + 2.0 * s, dtype=np.complex128)
    up = np.full(nth, -s, dtype=np.complex128)
    if st.periodic:
        ut = periodic_thomas_sm(lo, di, up, vt)
    else:
        ut = thomas(lo, di, up, vt)
    return np.ascontiguousarray(ut.T)


def march(st: Setup, u0: np.ndarray, j0: int, nsteps: int, callback=None) -> np.ndarray:
    """Advance u^{j0} by nsteps range steps (the range loop of Fig. 2).  If given,
    callback(j, u) is called after every step with the new step index."""
    u = np.asarray(u0, dtype=np.complex128).copy()
    for k in range(nsteps):
        u = step(st, u, j0 + k)
        if callback is not None:
            callback(j0 + k + 1, u)
    return u


def starter(st: Setup, zs: float) -> np.ndarray:
    """Gaussian starter with a surface image (reading A11; the paper says only
    the initial field of Fig. 2):
        u0(z) = sqrt(k0) [exp(-k0^2 (z - zs)^2 / 2) - exp(-k0^2 (z + zs)^2 / 2)]
    identical on every azimuth."""
    k0, z = st.k0, st.z
    col = math.sqrt(k0) * (np.exp(-0.5 * k0 * k0 * (z - zs) ** 2)
                           - np.exp(-0.5 * k0 * k0 * (z + zs) ** 2))
    return np.repeat(col[None, :].astype(np.complex128), st.nth, axis=0)


def tl(st: Setup, u: np.ndarray, j: int) -> np.ndarray:
    """Transmission loss of the envelope, -20 log10|u| + 10 log10 r_j (the
    Tappert factor's amplitude ~ r^-1/2, Sec. 2.1; additive constant dropped)."""
    with np.errstate(divide="ignore"):
        return -20.0 * np.log10(np.abs(u)) + 10.0 * math.log10(st.r(j))


def pressure(st: Setup, u: np.ndarray, j: int) -> np.ndarray:
    """Complex pressure of step j from the envelope: p = u H0^(1)(k0 r_j), the
    outgoing Hankel factor that the PE ansatz splits off (Sec. 2.1).  The
    Hankel function is the library routine (SciPy); r_j must be positive."""
    from scipy.special import hankel1
    r = st.r(j)
    if not r > 0.0:
        raise ValueError("the pressure needs r_j > 0")
    return u * hankel1(0, st.k0 * r)


def rel_l2(x: np.ndarray, ref: np.ndarray) -> float:
    """Relative L2 error over the whole field (reading A19)."""
    return float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel()))

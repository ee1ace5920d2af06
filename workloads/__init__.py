"""Seeded synthetic inputs for the 3D wide-angle PE range march.

This module describes *inputs only*: environments (sound-speed samples,
bathymetry samples, bottom half-space constants), grids, frequency lists,
request traces and random fields.  It holds none of the method's arithmetic
(no operators, no solves, no starter field); both the CPU oracle and the HIP
path receive the same objects from here and each evaluates them with its own
code.

The paper's own test environments are not available (its input files are not
part of the text; Fig. 5's environment is unspecified), so every environment
below is synthetic.  The shapes follow the paper's workload class: a
single-frequency 3D march (Sec. 4.1) and a multi-frequency wide-band batch
(Sec. 3.2.3, Sec. 4.2.3), plus a served request stream.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

FLOOR_PRESSURE_RELEASE = 0
FLOOR_RIGID = 1
PREC_C64 = 0
PREC_C128 = 1
#: coupling between azimuths: full 3D (Eq. (4)) or N x 2D (Y = 0, Sec. 1)
MODE_3D = 0
MODE_NX2D = 1
TWO_PI = 2.0 * math.pi
AZ_CHUNKED = 0   # azimuth solver of the GPU path: chunked recurrences + wavefront scan
AZ_PCR = 1       # parallel cyclic reduction in LDS


@dataclass(frozen=True)
class Env:
    """Ocean environment (units: m, m/s, g/cm^3, dB per wavelength).

    ssp_z/ssp_c: water sound speed, piecewise-linear in z, constant beyond the
    ends.  bathy_theta/bathy_depth: water depth D(theta), periodic
    piecewise-linear in theta (one sample means a flat bottom).  Below D the
    medium is a homogeneous fluid half-space (c_b, rho_b, atten_b).  zmax is the
    computational floor and `floor` its boundary condition.  Range-dependent
    depth: bathy_nr >= 2 rows at ranges bathy_r0 + i*bathy_dr, bathy_depth
    then holding bathy_nr rows of len(bathy_theta) samples (row-major); D is
    linear in r between rows and constant beyond the first and last.
    Range-dependent water: ssp_nr >= 2 profiles at ranges ssp_r0 + i*ssp_dr,
    ssp_c then holding ssp_nr rows of len(ssp_z) speeds (row-major); each
    row holds from its range until the next row's (stair-step), row 0 also
    before it.
    """
    c0: float
    ssp_z: tuple
    ssp_c: tuple
    rho_w: float
    atten_w: float
    c_b: float
    rho_b: float
    atten_b: float
    bathy_theta: tuple
    bathy_depth: tuple
    zmax: float
    floor: int
    bathy_nr: int = 0
    bathy_r0: float = 0.0
    bathy_dr: float = 0.0
    ssp_nr: int = 0
    ssp_r0: float = 0.0
    ssp_dr: float = 0.0


@dataclass(frozen=True)
class Grid:
    """Computational grid.  width == 2*pi means the full circle (periodic in
    azimuth); a smaller width is a sector centred on theta0 with zero field on
    the two edge azimuths.  The march starts at range r0.  mode MODE_NX2D
    drops the azimuth operator (Y = 0): N independent 2D marches.
    depth_lanes / azimuth_lanes / azimuth_solver: kernel shape and azimuth
    solver of the GPU path (0: its own choice, the chunked solver; tuning
    knobs that change nothing but rounding)."""
    nz: int
    ntheta: int
    theta0: float
    width: float
    dr: float
    r0: float = 0.0
    precision: int = PREC_C64
    mode: int = MODE_3D
    depth_lanes: int = 0
    azimuth_lanes: int = 0
    azimuth_solver: int = 0


@dataclass(frozen=True)
class Problem:
    env: Env
    grid: Grid
    f_hz: float
    zs: float
    nsteps: int
    name: str = ""

    @property
    def points(self) -> int:
        return self.grid.nz * self.grid.ntheta


def _ceil_to(x: float, m: int) -> int:
    return int(m * math.ceil(x / m))


def _clamp(x, lo, hi):
    return max(lo, min(hi, x))


# ---------------------------------------------------------------- environments
def isovelocity_env(depth: float = 200.0, c: float = 1500.0, rho: float = 1.0,
                    atten: float = 0.0, floor: int = FLOOR_RIGID,
                    c0: float = 1500.0) -> Env:
    """Homogeneous water column filling the whole computational depth."""
    return Env(c0=c0, ssp_z=(0.0,), ssp_c=(c,), rho_w=rho, atten_w=atten,
               c_b=c, rho_b=rho, atten_b=atten,
               bathy_theta=(0.0,), bathy_depth=(1.0e9,),
               zmax=depth, floor=floor)


def munk_samples(zmax: float = 3000.0, dz: float = 10.0, c_min: float = 1490.0,
                 z_axis: float = 1000.0, scale: float = 1300.0,
                 eps: float = 0.00737):
    """Canonical Munk profile shape, moved to the requested axis depth and
    minimum speed, sampled every dz metres (an input table, interpolated
    piecewise-linearly by each consumer)."""
    z = np.arange(0.0, zmax + 0.5 * dz, dz)
    eta = 2.0 * (z - z_axis) / scale
    c = c_min * (1.0 + eps * (eta - 1.0 + np.exp(-eta)))
    return tuple(float(v) for v in z), tuple(float(v) for v in c)


def wedge_env(zmax: float = 3000.0, d_max: float = 2000.0, d_min: float = 200.0,
              c_b: float = 1700.0, rho_b: float = 1.5, atten_b: float = 0.5,
              floor: int = FLOOR_PRESSURE_RELEASE, ssp_dz: float = 10.0) -> Env:
    """Munk-like water over a fluid bottom whose depth slopes linearly along
    azimuth from d_max at theta=0 to d_min at theta=+-pi (periodic wedge)."""
    z, c = munk_samples(zmax=zmax, dz=ssp_dz)
    return Env(c0=1500.0, ssp_z=z, ssp_c=c, rho_w=1.0, atten_w=0.0,
               c_b=c_b, rho_b=rho_b, atten_b=atten_b,
               bathy_theta=(-math.pi, 0.0), bathy_depth=(d_min, d_max),
               zmax=zmax, floor=floor)


def slope_env(d0: float = 400.0, slope_deg: float = 3.0, d_min: float = 30.0,
              d_max: float = 2500.0, zmax: float = 3000.0, rmax: float = 60000.0,
              row_dr: float = 250.0, nb: int = 72, c_b: float = 1700.0,
              rho_b: float = 1.5, atten_b: float = 0.5,
              floor: int = FLOOR_PRESSURE_RELEASE, ssp_dz: float = 10.0) -> Env:
    """Munk-like water over a planar sloping fluid bottom seen from a source
    where the depth is d0: D = d0 - y tan(slope) with y = r sin(theta) the
    cross-slope coordinate (upslope towards theta = pi/2), clipped to
    [d_min, d_max].  Range- and azimuth-dependent: sampled on range rows every
    row_dr metres out to rmax and nb azimuths."""
    z, c = munk_samples(zmax=zmax, dz=ssp_dz)
    th = -math.pi + (2.0 * math.pi / nb) * np.arange(nb)
    nr = int(math.ceil(rmax / row_dr)) + 1
    r = row_dr * np.arange(nr)
    d = np.clip(d0 - np.outer(r, np.sin(th)) * math.tan(math.radians(slope_deg)), d_min, d_max)
    return Env(c0=1500.0, ssp_z=z, ssp_c=c, rho_w=1.0, atten_w=0.0,
               c_b=c_b, rho_b=rho_b, atten_b=atten_b,
               bathy_theta=tuple(map(float, th)), bathy_depth=tuple(map(float, d.ravel())),
               zmax=zmax, floor=floor, bathy_nr=nr, bathy_r0=0.0, bathy_dr=row_dr)


def flat_layered_env(depth: float = 120.0, zmax: float = 200.0,
                     c_w: float = 1510.0, c_b: float = 1650.0,
                     rho_b: float = 1.8, atten_b: float = 0.3,
                     floor: int = FLOOR_PRESSURE_RELEASE) -> Env:
    """Azimuth-independent water layer over a fluid half-space."""
    return Env(c0=1500.0, ssp_z=(0.0, zmax), ssp_c=(c_w, c_w + 8.0),
               rho_w=1.0, atten_w=0.0, c_b=c_b, rho_b=rho_b, atten_b=atten_b,
               bathy_theta=(0.0,), bathy_depth=(depth,), zmax=zmax,
               floor=floor)


# ---------------------------------------------------------------- configurations
def config1() -> Problem:
    """25 Hz, isovelocity 1500 m/s, 200 m rigid floor, Nz=64, Ntheta=32
    (periodic), dr=5 m, 200 steps, source at 50 m, complex128."""
    env = isovelocity_env(depth=200.0, floor=FLOOR_RIGID)
    grid = Grid(nz=64, ntheta=32, theta0=0.0, width=TWO_PI, dr=5.0,
                precision=PREC_C128)
    return Problem(env, grid, 25.0, 50.0, 200, "config1")


def config2(nsteps: int = 5000, precision: int = PREC_C64) -> Problem:
    """100 Hz, Munk-like profile, periodic wedge 2000->200 m, fluid bottom
    (1700 m/s, 1.5, 0.5 dB/lambda), zmax 3000 m pressure-release floor,
    Nz=2048, Ntheta=512, dr=10 m, source at 100 m."""
    env = wedge_env()
    grid = Grid(nz=2048, ntheta=512, theta0=0.0, width=TWO_PI, dr=10.0,
                precision=precision)
    return Problem(env, grid, 100.0, 100.0, nsteps, "config2")


def config2_slope(nsteps: int = 1000, precision: int = PREC_C64) -> Problem:
    """The config-2 grid (Nz=2048, Ntheta=512, dr=10 m, 100 Hz, source at
    100 m, zmax 3000 m) over the range- and azimuth-dependent sloping bottom
    of slope_env (a true 3D cross-slope wedge)."""
    grid = Grid(nz=2048, ntheta=512, theta0=0.0, width=TWO_PI, dr=10.0,
                precision=precision)
    return Problem(slope_env(), grid, 100.0, 100.0, nsteps, "config2_slope")


def config4_problems(nsteps: int = 1000, nfreq: int = 64,
                     precision: int = PREC_C64) -> List[Problem]:
    """Wide-band batch: nfreq frequencies log-spaced over 20-500 Hz in the
    config-2 environment.  Nz gives dz = lambda/8 over 3000 m (multiple of 64,
    clamped to 128..4096), Ntheta grows as sqrt(f) (multiple of 64, clamped to
    256..1024), dr = 1000/f clamped to 2..25 m."""
    env = wedge_env()
    out = []
    for f in np.geomspace(20.0, 500.0, nfreq):
        f = float(f)
        nz = _clamp(_ceil_to(8.0 * f * env.zmax / env.c0, 64), 128, 4096)
        nth = _clamp(_ceil_to(256.0 * math.sqrt(f / 20.0), 64), 256, 1024)
        dr = _clamp(1000.0 / f, 2.0, 25.0)
        grid = Grid(nz=nz, ntheta=nth, theta0=0.0, width=TWO_PI, dr=dr,
                    precision=precision)
        out.append(Problem(env, grid, f, 100.0, nsteps, f"f{f:.2f}"))
    return out


@dataclass(frozen=True)
class Request:
    rid: int
    arrival_s: float
    problem: Problem


def config5_trace(n: int = 2000, rate_hz: float = 200.0, seed: int = 0,
                  zmax: float = 2400.0) -> List[Request]:
    """Served stream: Poisson arrivals; f ~ U(20,400) Hz, zs ~ U(10,500) m,
    sector width in {30, 90, 360} degrees, centre ~ U(0, 2pi), maximum range
    ~ U(2, 20) km.  dz ~ lambda/4 over zmax, Ntheta grows with sqrt(f) and
    with the sector width, dr ~ lambda."""
    rng = np.random.default_rng(seed)
    env = wedge_env(zmax=zmax)
    t = 0.0
    out = []
    for i in range(n):
        t += float(rng.exponential(1.0 / rate_hz))
        f = float(rng.uniform(20.0, 400.0))
        zs = float(rng.uniform(10.0, 500.0))
        wdeg = float(rng.choice([30.0, 90.0, 360.0]))
        th0 = float(rng.uniform(0.0, TWO_PI))
        rmax = float(rng.uniform(2000.0, 20000.0))
        nz = _clamp(_ceil_to(6.4 * f, 64), 128, 4096)
        nth360 = _clamp(_ceil_to(128.0 * math.sqrt(f / 20.0), 32), 128, 512)
        if wdeg >= 360.0:
            nth, width = nth360, TWO_PI
        else:
            nth, width = max(32, _ceil_to(nth360 * wdeg / 360.0, 32)), math.radians(wdeg)
        dr = _clamp(1500.0 / f, 2.0, 75.0)
        steps = int(math.ceil(rmax / dr))
        grid = Grid(nz=nz, ntheta=nth, theta0=th0, width=width, dr=dr,
                    precision=PREC_C64)
        out.append(Request(i, t, Problem(env, grid, f, zs, steps, f"req{i}")))
    return out


def random_field(ntheta: int, nz: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Seeded complex Gaussian field of shape (ntheta, nz) (depth contiguous)."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((ntheta, nz))
    im = rng.standard_normal((ntheta, nz))
    return (re + 1j * im).astype(dtype)


def random_env(seed: int, zmax: float = 300.0, lossless: bool = False,
               floor: int = FLOOR_PRESSURE_RELEASE, nbathy: int = 5) -> Env:
    """Seeded random environment: a few SSP samples, a random periodic
    bathymetry inside (0.2..0.9)*zmax, random bottom constants."""
    rng = np.random.default_rng(seed)
    zs = np.sort(rng.uniform(0.0, zmax, 4))
    cs = rng.uniform(1480.0, 1540.0, 4)
    th = np.sort(rng.uniform(-math.pi, math.pi, nbathy))
    d = rng.uniform(0.2 * zmax, 0.9 * zmax, nbathy)
    return Env(c0=1500.0, ssp_z=tuple(map(float, zs)), ssp_c=tuple(map(float, cs)),
               rho_w=float(rng.uniform(0.9, 1.1)),
               atten_w=0.0 if lossless else float(rng.uniform(0.0, 0.05)),
               c_b=float(rng.uniform(1550.0, 1900.0)),
               rho_b=float(rng.uniform(1.2, 2.2)),
               atten_b=0.0 if lossless else float(rng.uniform(0.1, 1.0)),
               bathy_theta=tuple(map(float, th)), bathy_depth=tuple(map(float, d)),
               zmax=zmax, floor=floor)


def random_range_env(seed: int, zmax: float = 300.0, nr: int = 6, row_dr: float = 20.0,
                     r0: float = 0.0, floor: int = FLOOR_PRESSURE_RELEASE, nbathy: int = 5) -> Env:
    """random_env with nr random depth rows (inside (0.05..0.98)*zmax, so
    columns gain and lose water nodes from step to step) at ranges
    r0 + i*row_dr."""
    base = random_env(seed, zmax=zmax, floor=floor, nbathy=nbathy)
    rng = np.random.default_rng(seed + 7919)
    d = rng.uniform(0.05 * zmax, 0.98 * zmax, (nr, nbathy))
    return replace(base, bathy_depth=tuple(map(float, d.ravel())), bathy_nr=nr,
                   bathy_r0=float(r0), bathy_dr=float(row_dr))


def random_ssp_range_env(seed: int, zmax: float = 300.0, nr: int = 5, row_dr: float = 30.0,
                         r0: float = 0.0, depth_rows: int = 0,
                         floor: int = FLOOR_PRESSURE_RELEASE, nbathy: int = 5) -> Env:
    """random_env (or random_range_env with depth_rows rows) with nr random
    water profiles on the same sample depths (1470..1560 m/s) at ranges
    r0 + i*row_dr."""
    if depth_rows >= 2:
        base = random_range_env(seed, zmax=zmax, nr=depth_rows, row_dr=row_dr * 0.7, r0=r0,
                                floor=floor, nbathy=nbathy)
    else:
        base = random_env(seed, zmax=zmax, floor=floor, nbathy=nbathy)
    rng = np.random.default_rng(seed + 104729)
    c = rng.uniform(1470.0, 1560.0, (nr, len(base.ssp_z)))
    return replace(base, ssp_c=tuple(map(float, c.ravel())), ssp_nr=nr, ssp_r0=float(r0),
                   ssp_dr=float(row_dr))


def front_env(rmax: float = 60000.0, row_dr: float = 1000.0, axis0: float = 1000.0,
              axis1: float = 600.0, c_min0: float = 1490.0, c_min1: float = 1500.0,
              zmax: float = 3000.0, ssp_dz: float = 10.0) -> Env:
    """The wedge of wedge_env under a range-dependent Munk-like water column:
    the sound channel's axis rises from axis0 to axis1 and its minimum speed
    goes from c_min0 to c_min1 linearly over rmax (an ocean front), given as
    profiles every row_dr metres (stair-step in range between them)."""
    base = wedge_env(zmax=zmax, ssp_dz=ssp_dz)
    nr = int(math.ceil(rmax / row_dr)) + 1
    rows = []
    for i in range(nr):
        t = min(i * row_dr / rmax, 1.0)
        z, c = munk_samples(zmax=zmax, dz=ssp_dz, c_min=c_min0 + t * (c_min1 - c_min0),
                            z_axis=axis0 + t * (axis1 - axis0))
        rows.extend(c)
    return replace(base, ssp_c=tuple(map(float, rows)), ssp_nr=nr, ssp_r0=0.0, ssp_dr=float(row_dr))


def config2_front(nsteps: int = 1000, precision: int = PREC_C64) -> Problem:
    """The config-2 grid over the wedge under the range-dependent water of
    front_env (a profile every 1 km)."""
    grid = Grid(nz=2048, ntheta=512, theta0=0.0, width=TWO_PI, dr=10.0,
                precision=precision)
    return Problem(front_env(), grid, 100.0, 100.0, nsteps, "config2_front")


def with_grid(p: Problem, **kw) -> Problem:
    return replace(p, grid=replace(p.grid, **kw))

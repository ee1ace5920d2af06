"""Python binding of libpe3d.so (include/pe3d.h): argument marshalling only.

Every step of the march runs in the HIP library.  There is no fallback: if the
shared library is missing this module raises at import.  PyTorch is used only
to hold device fields and to name the current HIP stream.

The module-level functions carry the C names (pe3d_create, pe3d_march, ...)
and return/raise on the C status codes; `Pe3d` is a small owning wrapper.
"""
from __future__ import annotations

import ctypes as ct
import math
import os
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpe3d.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_1711_00005_amd.build_lib` "
        "(the PE march has no CPU fallback)")

# torch first: its wheel carries a HIP runtime of its own, and with the
# library (linked against the system's runtime) loaded before it, torch's
# device initialisation finds no GPU.  Loaded after torch, the library shares
# the process's runtime with the tensors it is handed.
import torch  # noqa: E402,F401

_lib = ct.CDLL(LIB_PATH)

PE3D_OK = 0
PE3D_EINVAL = -1
PE3D_ENOMEM = -2
PE3D_EDEVICE = -3
PE3D_EUNSUPPORTED = -4
PE3D_ESTATE = -5
PE3D_FLOOR_PRESSURE_RELEASE = 0
PE3D_FLOOR_RIGID = 1
PE3D_C64 = 0
PE3D_C128 = 1
PE3D_MODE_3D = 0
PE3D_MODE_NX2D = 1
PE3D_STATIC_SCRATCH_BYTES = 32 << 20
PE3D_AZIMUTH_CHUNKED = 0
PE3D_AZIMUTH_PCR = 1
PE3D_BATCH_LAUNCHES = 0
PE3D_BATCH_PERSISTENT = 1

EXPORTED = ("pe3d_create", "pe3d_march", "pe3d_destroy", "pe3d_footprint", "pe3d_get_step",
            "pe3d_set_step", "pe3d_starter", "pe3d_march_batch", "pe3d_tl", "pe3d_pressure", "pe3d_get_info",
            "pe3d_host_tables", "pe3d_profile_enable", "pe3d_profile_read", "pe3d_strerror",
            "pe3d_set_batch_schedule", "pe3d_march_static", "pe3d_release_pooled_memory",
            "pe3d_set_batch_kernel", "pe3d_batch_wait_timeouts", "pe3d_persist_schedule")


class pe3d_env(ct.Structure):
    _fields_ = [("c0", ct.c_double), ("n_ssp", ct.c_int32),
                ("ssp_z", ct.POINTER(ct.c_double)), ("ssp_c", ct.POINTER(ct.c_double)),
                ("rho_w", ct.c_double), ("atten_w", ct.c_double),
                ("c_b", ct.c_double), ("rho_b", ct.c_double), ("atten_b", ct.c_double),
                ("n_bathy", ct.c_int32),
                ("bathy_theta", ct.POINTER(ct.c_double)), ("bathy_depth", ct.POINTER(ct.c_double)),
                ("n_bathy_r", ct.c_int32), ("bathy_r0", ct.c_double), ("bathy_dr", ct.c_double),
                ("zmax", ct.c_double), ("floor", ct.c_int32),
                ("n_ssp_r", ct.c_int32), ("ssp_r0", ct.c_double), ("ssp_dr", ct.c_double)]


class pe3d_grid(ct.Structure):
    _fields_ = [("nz", ct.c_int32), ("ntheta", ct.c_int32), ("theta0", ct.c_double),
                ("width", ct.c_double), ("dr", ct.c_double), ("r0", ct.c_double),
                ("precision", ct.c_int32), ("mode", ct.c_int32),
                ("depth_lanes", ct.c_int32), ("azimuth_lanes", ct.c_int32),
                ("azimuth_solver", ct.c_int32)]


class pe3d_freq(ct.Structure):
    _fields_ = [("f_hz", ct.c_double)]


class pe3d_info(ct.Structure):
    _fields_ = [("nz", ct.c_int32), ("ntheta", ct.c_int32), ("periodic", ct.c_int32),
                ("precision", ct.c_int32), ("mode", ct.c_int32), ("k0", ct.c_double), ("dz", ct.c_double),
                ("dtheta", ct.c_double), ("dr", ct.c_double), ("r0", ct.c_double),
                ("pass_a_lanes", ct.c_int32), ("pass_a_chunk", ct.c_int32),
                ("pass_b_chunks", ct.c_int32), ("pass_b_depths", ct.c_int32),
                ("device_bytes", ct.c_size_t)]


class pe3d_kernel_stat(ct.Structure):
    _fields_ = [("name", ct.c_char * 48), ("launches", ct.c_int32), ("total_ms", ct.c_double),
                ("algo_bytes", ct.c_double)]


_H = ct.c_void_p
_lib.pe3d_create.argtypes = [ct.POINTER(pe3d_env), ct.POINTER(pe3d_grid), ct.POINTER(pe3d_freq),
                             ct.POINTER(_H)]
_lib.pe3d_march.argtypes = [_H, ct.c_int32, ct.c_void_p, ct.c_void_p]
_lib.pe3d_march_static.argtypes = [_H, ct.c_int32, ct.c_void_p, ct.c_void_p]
_lib.pe3d_destroy.argtypes = [_H]
_lib.pe3d_footprint.argtypes = [ct.POINTER(pe3d_env), ct.POINTER(pe3d_grid),
                                ct.POINTER(pe3d_freq), ct.POINTER(ct.c_size_t)]
_lib.pe3d_get_step.argtypes = [_H, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double)]
_lib.pe3d_set_step.argtypes = [_H, ct.c_int64]
_lib.pe3d_starter.argtypes = [_H, ct.c_double, ct.c_void_p, ct.c_void_p]
_lib.pe3d_march_batch.argtypes = [ct.POINTER(_H), ct.c_int32, ct.POINTER(ct.c_int32),
                                  ct.POINTER(ct.c_void_p), ct.c_int32, ct.c_void_p]
_lib.pe3d_tl.argtypes = [_H, ct.c_void_p, ct.c_void_p, ct.c_void_p]
_lib.pe3d_pressure.argtypes = [_H, ct.c_void_p, ct.c_void_p, ct.c_void_p]
_lib.pe3d_get_info.argtypes = [_H, ct.POINTER(pe3d_info)]
_lib.pe3d_host_tables.argtypes = [ct.POINTER(pe3d_env), ct.POINTER(pe3d_grid), ct.POINTER(pe3d_freq),
                                  ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p]
_lib.pe3d_profile_enable.argtypes = [ct.c_int32]
_lib.pe3d_profile_read.argtypes = [ct.POINTER(pe3d_kernel_stat), ct.c_int32, ct.POINTER(ct.c_int32)]
_lib.pe3d_strerror.argtypes = [ct.c_int]
_lib.pe3d_set_batch_schedule.argtypes = [ct.c_int32, ct.c_int64]
_lib.pe3d_release_pooled_memory.argtypes = [ct.POINTER(ct.c_size_t)]
_lib.pe3d_set_batch_kernel.argtypes = [ct.c_int32, ct.c_double]
_lib.pe3d_batch_wait_timeouts.argtypes = [ct.POINTER(ct.c_int64)]
_I32P = ct.POINTER(ct.c_int32)
_lib.pe3d_persist_schedule.argtypes = [ct.c_int32, _I32P, _I32P, _I32P, _I32P, _I32P, _I32P, _I32P, _I32P,
                                       ct.c_int64, ct.POINTER(ct.c_int64)]
for _n in EXPORTED:
    getattr(_lib, _n).restype = ct.c_int
_lib.pe3d_strerror.restype = ct.c_char_p


class Pe3dError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {pe3d_strerror(status)} ({status})")


def _check(st: int, where: str) -> None:
    if st != PE3D_OK:
        raise Pe3dError(st, where)


def pe3d_strerror(status: int) -> str:
    return _lib.pe3d_strerror(int(status)).decode()


def _darr(vals):
    vals = [float(v) for v in vals]
    return (ct.c_double * max(1, len(vals)))(*vals)


def make_env(env):
    """ctypes pe3d_env from any object with the Env attributes; returns the
    struct and the arrays it points to (keep both alive across the call)."""
    # the C side reads ssp_c and bathy_depth as (rows x samples) arrays
    nsr = max(int(getattr(env, "ssp_nr", 0)), 1)
    nbr = max(int(getattr(env, "bathy_nr", 0)), 1)
    if len(env.ssp_c) != nsr * len(env.ssp_z):
        raise ValueError(f"ssp_c holds {len(env.ssp_c)} speeds, expected {nsr} x {len(env.ssp_z)}")
    if len(env.bathy_depth) != nbr * len(env.bathy_theta):
        raise ValueError(f"bathy_depth holds {len(env.bathy_depth)} depths, expected {nbr} x "
                         f"{len(env.bathy_theta)}")
    keep = [_darr(env.ssp_z), _darr(env.ssp_c), _darr(env.bathy_theta), _darr(env.bathy_depth)]
    s = pe3d_env(c0=env.c0, n_ssp=len(env.ssp_z), ssp_z=keep[0], ssp_c=keep[1],
                 rho_w=env.rho_w, atten_w=env.atten_w, c_b=env.c_b, rho_b=env.rho_b,
                 atten_b=env.atten_b, n_bathy=len(env.bathy_theta), bathy_theta=keep[2],
                 bathy_depth=keep[3], n_bathy_r=int(getattr(env, "bathy_nr", 0)),
                 bathy_r0=float(getattr(env, "bathy_r0", 0.0)), bathy_dr=float(getattr(env, "bathy_dr", 0.0)),
                 zmax=env.zmax, floor=int(env.floor), n_ssp_r=int(getattr(env, "ssp_nr", 0)),
                 ssp_r0=float(getattr(env, "ssp_r0", 0.0)), ssp_dr=float(getattr(env, "ssp_dr", 0.0)))
    return s, keep


def make_grid(grid):
    return pe3d_grid(nz=int(grid.nz), ntheta=int(grid.ntheta), theta0=float(grid.theta0),
                     width=float(grid.width), dr=float(grid.dr), r0=float(getattr(grid, "r0", 0.0)),
                     precision=int(getattr(grid, "precision", PE3D_C64)),
                     mode=int(getattr(grid, "mode", PE3D_MODE_3D)),
                     depth_lanes=int(getattr(grid, "depth_lanes", 0)),
                     azimuth_lanes=int(getattr(grid, "azimuth_lanes", 0)),
                     azimuth_solver=int(getattr(grid, "azimuth_solver", 0)))


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _field_ptr(u, nz: int, nth: int, prec: int) -> int:
    import torch
    want = torch.complex128 if prec == PE3D_C128 else torch.complex64
    if not (isinstance(u, torch.Tensor) and u.is_cuda and u.dtype == want
            and u.is_contiguous() and tuple(u.shape) == (nth, nz)):
        raise ValueError(f"field must be a contiguous CUDA {want} tensor of shape ({nth}, {nz})")
    return u.data_ptr()


# ----------------------------------------------------------------------- C calls
def pe3d_footprint(env, grid, f_hz: float) -> int:
    e, keep = make_env(env)
    g = make_grid(grid)
    out = ct.c_size_t(0)
    _check(_lib.pe3d_footprint(ct.byref(e), ct.byref(g), ct.byref(pe3d_freq(f_hz)), ct.byref(out)),
           "pe3d_footprint")
    return int(out.value)


def pe3d_create(env, grid, f_hz: float) -> int:
    e, keep = make_env(env)
    g = make_grid(grid)
    h = _H()
    _check(_lib.pe3d_create(ct.byref(e), ct.byref(g), ct.byref(pe3d_freq(f_hz)), ct.byref(h)),
           "pe3d_create")
    return h.value


def pe3d_create_status(env, grid, f_hz: float) -> int:
    """Status of pe3d_create only (the handle, if any, is destroyed)."""
    e, keep = make_env(env)
    g = make_grid(grid)
    h = _H()
    st = _lib.pe3d_create(ct.byref(e), ct.byref(g), ct.byref(pe3d_freq(f_hz)), ct.byref(h))
    if st == PE3D_OK:
        _lib.pe3d_destroy(h)
    return st


def pe3d_host_tables(env, grid, f_hz: float):
    """FP64 host tables (host only): dict of numpy arrays qw, pw, pb (complex,
    nz), kcol (int, ntheta), blk (complex, ntheta x 12)."""
    import numpy as np
    e, keep = make_env(env)
    g = make_grid(grid)
    nz, nth = int(grid.nz), int(grid.ntheta)
    qw = np.zeros(2 * nz)
    pw = np.zeros(2 * nz)
    pb = np.zeros(2 * nz)
    kc = np.zeros(nth, dtype=np.int32)
    blk = np.zeros(24 * nth)
    _check(_lib.pe3d_host_tables(ct.byref(e), ct.byref(g), ct.byref(pe3d_freq(f_hz)),
                                 qw.ctypes.data, pw.ctypes.data, pb.ctypes.data, kc.ctypes.data,
                                 blk.ctypes.data), "pe3d_host_tables")
    c = lambda a: a[0::2] + 1j * a[1::2]
    return dict(qw=c(qw), pw=c(pw), pb=c(pb), kcol=kc.astype(int), blk=c(blk).reshape(nth, 12))


def pe3d_destroy(h) -> None:
    _check(_lib.pe3d_destroy(h), "pe3d_destroy")


def pe3d_march(h, nsteps: int, u_ptr: int, stream_ptr) -> None:
    _check(_lib.pe3d_march(h, int(nsteps), ct.c_void_p(u_ptr), ct.c_void_p(stream_ptr)), "pe3d_march")


def pe3d_march_static(h, nsteps: int, u_ptr: int, stream_ptr) -> None:
    _check(_lib.pe3d_march_static(h, int(nsteps), ct.c_void_p(u_ptr), ct.c_void_p(stream_ptr)),
           "pe3d_march_static")


def pe3d_starter(h, zs: float, u_ptr: int, stream_ptr) -> None:
    _check(_lib.pe3d_starter(h, float(zs), ct.c_void_p(u_ptr), ct.c_void_p(stream_ptr)),
           "pe3d_starter")


def pe3d_get_step(h):
    j = ct.c_int64(0)
    r = ct.c_double(0.0)
    _check(_lib.pe3d_get_step(h, ct.byref(j), ct.byref(r)), "pe3d_get_step")
    return int(j.value), float(r.value)


def pe3d_set_step(h, j: int) -> None:
    _check(_lib.pe3d_set_step(h, int(j)), "pe3d_set_step")


def pe3d_get_info(h) -> pe3d_info:
    info = pe3d_info()
    _check(_lib.pe3d_get_info(h, ct.byref(info)), "pe3d_get_info")
    return info


def pe3d_pressure(h, u_ptr: int, p_ptr: int, stream_ptr) -> None:
    _check(_lib.pe3d_pressure(h, ct.c_void_p(u_ptr), ct.c_void_p(p_ptr), ct.c_void_p(stream_ptr)),
           "pe3d_pressure")


def pe3d_tl(h, u_ptr: int, tl_ptr: int, stream_ptr) -> None:
    _check(_lib.pe3d_tl(h, ct.c_void_p(u_ptr), ct.c_void_p(tl_ptr), ct.c_void_p(stream_ptr)), "pe3d_tl")


def pe3d_march_batch(handles: Sequence[int], nsteps: Sequence[int], u_ptrs: Sequence[int],
                     use_graph: int, stream_ptr) -> None:
    """use_graph: 0 direct launches, 1 graph (captured once, replayed), 2
    capture only (nothing runs)."""
    n = len(handles)
    hs = (_H * n)(*handles)
    ns = (ct.c_int32 * n)(*[int(s) for s in nsteps])
    us = (ct.c_void_p * n)(*u_ptrs)
    _check(_lib.pe3d_march_batch(hs, n, ns, us, int(use_graph), ct.c_void_p(stream_ptr)),
           "pe3d_march_batch")


def pe3d_set_batch_schedule(chains: int, group_bytes: int) -> None:
    _check(_lib.pe3d_set_batch_schedule(int(chains), int(group_bytes)), "pe3d_set_batch_schedule")


def pe3d_set_batch_kernel(kind: int, wait_limit_s: float = 1.0) -> None:
    _check(_lib.pe3d_set_batch_kernel(int(kind), float(wait_limit_s)), "pe3d_set_batch_kernel")


def pe3d_batch_wait_timeouts() -> int:
    """Waits of persistent batched marches that ran out since the last call
    (synchronous; call after synchronising the marches' streams)."""
    n = ct.c_int64(0)
    _check(_lib.pe3d_batch_wait_timeouts(ct.byref(n)), "pe3d_batch_wait_timeouts")
    return int(n.value)


def pe3d_persist_schedule(na, asub, nb, bsub, nsteps, chain, group):
    """The persistent kernel's task list for problems of these shapes (host
    only): a list of (problem, first tile, step, kind, tiles, need)."""
    n = len(na)
    arrs = [(ct.c_int32 * n)(*[int(x) for x in a]) for a in (na, asub, nb, bsub, nsteps, chain, group)]
    cnt = ct.c_int64(0)
    _check(_lib.pe3d_persist_schedule(n, *arrs, None, 0, ct.byref(cnt)), "pe3d_persist_schedule")
    out = (ct.c_int32 * (6 * max(cnt.value, 1)))()
    _check(_lib.pe3d_persist_schedule(n, *arrs, out, cnt.value, ct.byref(cnt)), "pe3d_persist_schedule")
    return [tuple(out[6 * t:6 * t + 6]) for t in range(cnt.value)]


def pe3d_release_pooled_memory() -> int:
    """Return the library's idle pooled device memory to the runtime; bytes freed."""
    n = ct.c_size_t(0)
    _check(_lib.pe3d_release_pooled_memory(ct.byref(n)), "pe3d_release_pooled_memory")
    return int(n.value)


def pe3d_profile_enable(on: bool) -> None:
    _check(_lib.pe3d_profile_enable(int(bool(on))), "pe3d_profile_enable")


def pe3d_profile_read():
    """Per-kernel aggregates since the last read: list of dicts with name,
    launches, total_ms, algo_bytes."""
    cap = 64
    arr = (pe3d_kernel_stat * cap)()
    n = ct.c_int32(0)
    _check(_lib.pe3d_profile_read(arr, cap, ct.byref(n)), "pe3d_profile_read")
    return [dict(name=arr[i].name.decode(), launches=int(arr[i].launches),
                 total_ms=float(arr[i].total_ms), algo_bytes=float(arr[i].algo_bytes))
            for i in range(min(n.value, cap))]


# ----------------------------------------------------------------------- wrapper
class Pe3d:
    """Owning handle of one march (one frequency, one grid)."""

    def __init__(self, env, grid, f_hz: float):
        self.env, self.grid, self.f_hz = env, grid, float(f_hz)
        self.nz, self.ntheta = int(grid.nz), int(grid.ntheta)
        self.precision = int(getattr(grid, "precision", PE3D_C64))
        self.h = pe3d_create(env, grid, f_hz)

    def close(self) -> None:
        if self.h:
            pe3d_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def dtype(self):
        import torch
        return torch.complex128 if self.precision == PE3D_C128 else torch.complex64

    def new_field(self):
        import torch
        return torch.zeros((self.ntheta, self.nz), dtype=self.dtype, device="cuda")

    def starter(self, zs: float, u=None, stream=None):
        if u is None:
            u = self.new_field()
        pe3d_starter(self.h, zs, _field_ptr(u, self.nz, self.ntheta, self.precision), _stream_ptr(stream))
        return u

    def march(self, nsteps: int, u, stream=None):
        pe3d_march(self.h, nsteps, _field_ptr(u, self.nz, self.ntheta, self.precision), _stream_ptr(stream))
        return u

    def march_static(self, nsteps: int, u, stream=None):
        """pe3d_march with the library's file-scope scratch field (allocates nothing)."""
        pe3d_march_static(self.h, nsteps, _field_ptr(u, self.nz, self.ntheta, self.precision),
                          _stream_ptr(stream))
        return u

    def tl(self, u, stream=None):
        import torch
        out = torch.empty((self.ntheta, self.nz), dtype=torch.float32, device=u.device)
        pe3d_tl(self.h, _field_ptr(u, self.nz, self.ntheta, self.precision), out.data_ptr(),
                _stream_ptr(stream))
        return out

    def pressure(self, u, stream=None):
        """p = u H0^(1)(k0 r_j) at the current step, as a new field."""
        import torch
        out = torch.empty_like(u)
        pe3d_pressure(self.h, _field_ptr(u, self.nz, self.ntheta, self.precision),
                      _field_ptr(out, self.nz, self.ntheta, self.precision), _stream_ptr(stream))
        return out

    @property
    def step(self) -> int:
        return pe3d_get_step(self.h)[0]

    @property
    def range_m(self) -> float:
        return pe3d_get_step(self.h)[1]

    def set_step(self, j: int) -> None:
        pe3d_set_step(self.h, j)

    def info(self) -> pe3d_info:
        return pe3d_get_info(self.h)


def march_batch(marches: Sequence[Pe3d], nsteps, fields, use_graph: bool = True, stream=None) -> None:
    if isinstance(nsteps, int):
        nsteps = [nsteps] * len(marches)
    ptrs = [_field_ptr(u, m.nz, m.ntheta, m.precision) for m, u in zip(marches, fields)]
    pe3d_march_batch([m.h for m in marches], nsteps, ptrs, 1 if use_graph else 0, _stream_ptr(stream))


def set_batch_schedule(chains: int = 2, group_bytes: int = 112 << 20) -> None:
    """Schedule of later batched plans: independent chains (concurrent streams
    on graph replay) of groups of at most group_bytes of field, each group
    marched through all of its steps before the next (0: one group per
    chain).  The defaults are the library's."""
    pe3d_set_batch_schedule(chains, group_bytes)


def set_batch_kernel(kind: int = PE3D_BATCH_LAUNCHES, wait_limit_s: float = 1.0) -> None:
    """Kernel of later batched plans: PE3D_BATCH_LAUNCHES (one launch per
    pass per step per group, the library's default) or PE3D_BATCH_PERSISTENT
    (one persistent kernel per call; each of its waits bounded by
    wait_limit_s)."""
    pe3d_set_batch_kernel(kind, wait_limit_s)


def prepare_batch(marches: Sequence[Pe3d], nsteps, fields, stream=None) -> None:
    """Build and capture the graph that march_batch(marches, nsteps, fields)
    replays, without running it (fields and steps unchanged)."""
    if isinstance(nsteps, int):
        nsteps = [nsteps] * len(marches)
    ptrs = [_field_ptr(u, m.nz, m.ntheta, m.precision) for m, u in zip(marches, fields)]
    pe3d_march_batch([m.h for m in marches], nsteps, ptrs, 2, _stream_ptr(stream))

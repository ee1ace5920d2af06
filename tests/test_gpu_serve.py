"""Served stream on the GPU: continuous batching gives the same result for a
request whether it is served alone or in a mix (bitwise: the batched kernels
run each problem independently), and matches the oracle."""
import math
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)


def trace(n, seed, max_steps):
    tr = W.config5_trace(n=n, rate_hz=400.0, seed=seed)
    out = []
    for r in tr:
        p = r.problem
        # smaller grids and ranges keep the test short; the mix still has
        # sectors and full circles of different sizes
        g = W.Grid(nz=min(p.grid.nz, 512), ntheta=min(p.grid.ntheta, 128), theta0=p.grid.theta0,
                   width=p.grid.width, dr=p.grid.dr)
        out.append(W.Request(r.rid, r.arrival_s,
                             W.Problem(p.env, g, p.f_hz, p.zs, min(p.nsteps, max_steps), p.name)))
    return out


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    return _t


def test_served_alone_equals_served_in_mix(torch):
    from paper_1711_00005_amd.serve import Pe3dBackend, Scheduler, report
    tr = trace(16, seed=1, max_steps=30)
    keep = [r.rid for r in tr]
    say("serve mix", len(tr))
    be = Pe3dBackend(keep_fields=keep)
    sch = Scheduler(be, budget_bytes=256 << 20, chunk_steps=7)
    recs = sch.run(tr)
    rep = report(recs)
    assert rep["done"] == len(tr)
    assert sch.max_resident > 1
    for r in tr[:5]:
        say("serve alone", r.rid)
        alone = Pe3dBackend(keep_fields=[r.rid])
        Scheduler(alone, budget_bytes=256 << 20, chunk_steps=5).run([W.Request(r.rid, 0.0, r.problem)])
        assert np.array_equal(alone.kept[r.rid], be.kept[r.rid]), r.rid
    # one request against the oracle (complex64 tolerance)
    small = min(tr, key=lambda r: r.problem.points * r.problem.nsteps)
    p = small.problem
    st = O.setup(p.env, p.grid, p.f_hz)
    ref = O.march(st, O.starter(st, p.zs), 0, p.nsteps)
    assert O.rel_l2(be.kept[small.rid].astype(np.complex128), ref) < 1e-5


def test_served_with_persistent_kernel_equals_launches(torch):
    """The same trace served with the persistent batch kernel (one launch per
    iteration) gives every request the field the launches give, bit for
    bit, and no wait runs out."""
    from paper_1711_00005_amd import pe3d as P
    from paper_1711_00005_amd.serve import Pe3dBackend, Scheduler, report
    tr = trace(12, seed=2, max_steps=25)
    keep = [r.rid for r in tr]
    kept = {}
    for kind in (P.PE3D_BATCH_LAUNCHES, P.PE3D_BATCH_PERSISTENT):
        say("serve kind", kind, len(tr))
        P.set_batch_kernel(kind)
        try:
            be = Pe3dBackend(keep_fields=keep)
            recs = Scheduler(be, budget_bytes=256 << 20, chunk_steps=6).run(tr)
        finally:
            P.set_batch_kernel(P.PE3D_BATCH_LAUNCHES)
        assert report(recs)["done"] == len(tr)
        kept[kind] = be.kept
    torch.cuda.synchronize()
    assert P.pe3d_batch_wait_timeouts() == 0
    for r in tr:
        assert np.array_equal(kept[P.PE3D_BATCH_LAUNCHES][r.rid], kept[P.PE3D_BATCH_PERSISTENT][r.rid]), r.rid

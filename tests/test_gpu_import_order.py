"""The binding can be imported before torch: the HIP runtime of the process
is then still usable by torch and by the library (a fresh interpreter, so
that no earlier import decides the order)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import paper_1711_00005_amd.pe3d as P
import workloads as W
import torch
m = P.Pe3d(W.wedge_env(), W.Grid(nz=64, ntheta=8, theta0=0.0, width=W.TWO_PI, dr=10.0), 50.0)
u = m.starter(100.0)
m.march(3, u)
torch.cuda.synchronize()
assert torch.isfinite(torch.view_as_real(u)).all() and float(u.abs().max()) > 0
m.close()
print("import order ok", flush=True)
"""


@pytest.mark.gpu
def test_package_imported_before_torch():
    print("[gpu] import order: fresh interpreter", flush=True)
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, capture_output=True, text=True, timeout=110)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "import order ok" in r.stdout

"""Build libpe3d.so (HIP kernels for gfx950 + host runtime) in-tree with hipcc.

Usage: python -m paper_1711_00005_amd.build_lib   (or call build()).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libpe3d.so")
BUILD_DIR = os.path.join(PKG, "_build")

ARCH = os.environ.get("PE3D_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", f"-I{INCLUDE}", f"-I{CSRC}"]
# no packed FP32 instructions in device code
DEVICE_ONLY = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build libpe3d.so")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("command failed: " + " ".join(cmd))
    return r


def build(verbose: bool = False) -> str:
    """Compile every source and link libpe3d.so; returns its path."""
    hipcc = _hipcc()
    os.makedirs(BUILD_DIR, exist_ok=True)
    k_obj = os.path.join(BUILD_DIR, "pe3d_kernels.o")
    h_obj = os.path.join(BUILD_DIR, "pe3d_host.o")
    cmds = [
        [hipcc, "-c", "-x", "hip", f"--offload-arch={ARCH}", *COMMON, *DEVICE_ONLY,
         os.path.join(CSRC, "pe3d_kernels.hip"), "-o", k_obj],
        [hipcc, "-c", *COMMON, os.path.join(CSRC, "pe3d_host.cpp"), "-o", h_obj],
        [hipcc, "-shared", f"--offload-arch={ARCH}", "-fPIC", k_obj, h_obj, "-o", LIB + ".tmp"],
    ]
    for c in cmds:
        if verbose:
            print(" ".join(c), flush=True)
        _run(c)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

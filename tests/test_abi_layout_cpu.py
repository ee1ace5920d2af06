"""The ctypes structures of the Python binding have the C header's layout:
a C program built with gcc against include/pe3d.h prints every struct's size
and every field's offset, and the binding's ctypes definitions must agree
(a mismatch would pass wrong values through the C ABI without any error)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = ("pe3d_env", "pe3d_grid", "pe3d_freq", "pe3d_info", "pe3d_kernel_stat")


@pytest.fixture(scope="module")
def P():
    import paper_1711_00005_amd.pe3d as _P
    return _P


def _c_layout(P, tmp_path):
    gcc = shutil.which("gcc") or shutil.which("cc")
    if gcc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pe3d.h"', "int main(void) {"]
    for name in STRUCTS:
        cls = getattr(P, name)
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines.append('  printf("macro PE3D_STATIC_SCRATCH_BYTES %zu\\n", (size_t)PE3D_STATIC_SCRATCH_BYTES);')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}


def test_ctypes_structs_match_the_header(P, tmp_path):
    c = _c_layout(P, tmp_path)
    import ctypes as ct
    for name in STRUCTS:
        cls = getattr(P, name)
        assert c[(name, "size")] == ct.sizeof(cls), name
        for field, _ in cls._fields_:
            assert c[(name, field)] == getattr(cls, field).offset, (name, field)


def test_static_scratch_limit_matches_the_header(P, tmp_path):
    c = _c_layout(P, tmp_path)
    assert c[("macro", "PE3D_STATIC_SCRATCH_BYTES")] == P.PE3D_STATIC_SCRATCH_BYTES

"""CPU complex128 oracle for the 3D wide-angle PE range march.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy implementation of what the HIP path computes, used to check it.  Only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import it;
the product path never does.  It shares no code with the HIP library and
imports nothing from the product package.
"""
from .pe3d_oracle import *  # noqa: F401,F403

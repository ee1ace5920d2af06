"""Write tests/golden/config2_oracle_samples.npz: the complex128 oracle's
config-2 march (100 Hz, Munk-like profile, periodic wedge, fluid bottom,
Nz=2048, Ntheta=512, dr=10 m, Gaussian starter at 100 m) sampled at the
checkpoints used by the GPU parity tests.  Calls only `oracle` and the seeded
input generators; nothing here comes from the HIP path.

Stored per checkpoint j: the field on every 4th azimuth and every 16th depth
node, and the full-field L2 norm.  Run: python tests/golden/make_config2_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

CHECKPOINTS = (1, 10, 100, 250, 500)
TH_STRIDE, Z_STRIDE = 4, 16


def main():
    p = W.config2(nsteps=max(CHECKPOINTS))
    st = O.setup(p.env, p.grid, p.f_hz)
    u = O.starter(st, p.zs)
    out = {"checkpoints": np.array(CHECKPOINTS), "th_stride": TH_STRIDE, "z_stride": Z_STRIDE}
    t0 = time.time()

    def cb(j, v):
        if j in CHECKPOINTS:
            out[f"u{j}"] = v[::TH_STRIDE, ::Z_STRIDE].copy()
            out[f"norm{j}"] = np.linalg.norm(v)
            print(f"step {j} norm {out[f'norm{j}']:.6e} t={time.time() - t0:.1f}s", flush=True)

    O.march(st, u, 0, max(CHECKPOINTS), callback=cb)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config2_oracle_samples.npz")
    np.savez_compressed(path, **out)
    print("wrote", path)


if __name__ == "__main__":
    main()

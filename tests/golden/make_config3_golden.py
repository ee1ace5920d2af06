"""Write tests/golden/config3_oracle_samples.npz: the complex128 oracle's
config-2 march (100 Hz, Munk-like profile, periodic wedge, fluid bottom,
Nz=2048, Ntheta=512, dr=10 m, Gaussian starter at 100 m) to 5000 range steps
(50 km), sampled every 500 steps, for the long-range precision study of the
complex64 and FP64 GPU marches.  Calls only `oracle` and the seeded input
generators; nothing here comes from the HIP path.

Stored per checkpoint j: the field on every 4th azimuth and every 16th depth
node, the full-field L2 norm and the full-field peak |u| (the transmission-loss
comparison uses nodes within 60 dB of it).  One core, about 40 minutes.
Run: python tests/golden/make_config3_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

CHECKPOINTS = tuple(range(500, 5001, 500))
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
            out[f"peak{j}"] = np.abs(v).max()
            print(f"step {j} norm {out[f'norm{j}']:.6e} t={time.time() - t0:.1f}s", flush=True)

    O.march(st, u, 0, max(CHECKPOINTS), callback=cb)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config3_oracle_samples.npz")
    np.savez_compressed(path, **out)
    print("wrote", path)


if __name__ == "__main__":
    main()

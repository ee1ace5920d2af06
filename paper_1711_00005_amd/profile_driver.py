"""Fixed workload for hardware-counter profiling of the march kernels.

Runs the 64-frequency batch (the bench workload) for a few range steps with
direct launches (no graph), each launch over the whole batch (one chain, one
group: the launches whose durations bench.py times with events), then one plain device copy of a known size (a
calibration kernel for the memory-traffic counters).  Usage:
  rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_1711_00005_amd.profile_driver [steps]
"""
import os
import sys


def main():
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch
    import workloads as W
    from paper_1711_00005_amd import pe3d as P
    steps = int(sys.argv[1]) if len(sys.argv) > 1 else 2
    probs = W.config4_problems(nsteps=steps)
    ms = [P.Pe3d(p.env, p.grid, p.f_hz) for p in probs]
    us = [m.starter(p.zs) for m, p in zip(ms, probs)]
    P.set_batch_schedule(1, 0)
    P.march_batch(ms, 1, us, use_graph=False)   # first-step kernels of a call
    P.march_batch(ms, steps, us, use_graph=False)
    torch.cuda.synchronize()
    # calibration: copy of exactly 512 MiB (read 512 MiB, write 512 MiB)
    a = torch.empty(64 << 20, dtype=torch.complex64, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print("profile_driver done: steps", steps, "copy bytes", a.numel() * 8, flush=True)


if __name__ == "__main__":
    main()

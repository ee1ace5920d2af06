#!/usr/bin/env python3
"""Benchmark of the 3D wide-angle PE range march on one MI355X.

Default workload: the wide-band batch of 64 frequencies (20-500 Hz, dz =
lambda/8, Ntheta growing with sqrt(f), Munk-like profile over a periodic
wedge, 107.6 M grid points, 861 MB of complex64 field) advanced together by
the batched march (one launch per pass per range step for all 64 problems,
replayed from a captured hipGraph).  One bench "step" is one range step of
every problem: pass A + pass B over the whole batch.

Printed (one JSON line): throughput in grid-point * range-steps / s; the
dominant kernel's achieved HBM bandwidth from HIP events (algorithmic bytes =
the field read once and written once per pass); the same calls with the
other batch kernel (one persistent kernel per call, or the launches); the
plain per-frequency march (one problem at a time, per-step launches) on the
same batch and the ratio;
a parity sample against the complex128 oracle; the oracle's own CPU
throughput on a bounded sample.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

METRIC = "grid-point·range-steps/s (batched vs plain) at ≤1e-5 rel L2; p50/p99 latency"
UNIT = "grid-point·range-steps/s"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed range steps of the whole batch")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--chunk", type=int, default=100, help="range steps per batched call (one graph)")
    ap.add_argument("--chains", type=int, default=2,
                    help="batch schedule: independent chains replayed on concurrent streams")
    ap.add_argument("--group-mib", type=int, default=112,
                    help="batch schedule: field MiB of one group, marched through a whole call in turn (0: one group)")
    ap.add_argument("--batch-kernel", choices=["launches", "persistent"], default="launches",
                    help="batched march: one launch per pass per step per group, or one persistent "
                         "kernel per call")
    ap.add_argument("--no-persist-report", action="store_true",
                    help="do not also time the other batch kernel on the same batch (same calls)")
    ap.add_argument("--workload", choices=["config4", "config2"], default="config4")
    ap.add_argument("--nfreq", type=int, default=64)
    ap.add_argument("--precision", choices=["c64", "c128"], default="c64",
                    help="field storage (arithmetic is FP64 in both)")
    ap.add_argument("--plain-steps", type=int, default=10)
    ap.add_argument("--profile-steps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--precision-study", action="store_true",
                    help="also march config 2 to 5000 steps in complex64 and complex128 and compare "
                         "with the stored oracle samples every 500 steps")
    ap.add_argument("--nx2d-report", action="store_true",
                    help="also compare the N x 2D (Y = 0) mode with the 3D march on the config-2 wedge")
    ap.add_argument("--range-report", action="store_true",
                    help="also time the config-2 grid over the range-dependent sloping bottom")
    ap.add_argument("--tune", action="store_true",
                    help="choose every problem's kernel lanes by timing its shape alone (tune.py) first")
    ap.add_argument("--no-tune-azimuth", action="store_true",
                    help="skip the in-batch choice of the azimuth solver (chunked or cyclic reduction) "
                         "per Ntheta class")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests of the served stream (the first n of the 2000-request trace)")
    ap.add_argument("--serve-range-scale", type=float, default=1.0,
                    help="multiply every served request's range (and steps) by this factor")
    ap.add_argument("--serve-chunk", type=int, default=40,
                    help="range steps every resident request advances per served iteration")
    ap.add_argument("--serve-backlog-chunk", type=int, default=100,
                    help="range steps per served iteration while requests wait for admission")
    ap.add_argument("--serve-graph", action="store_true",
                    help="replay every served iteration as a captured HIP graph")
    ap.add_argument("--serve-batch-kernel", choices=["launches", "persistent"], default=None,
                    help="batch kernel of the served stream (default: --batch-kernel)")
    ap.add_argument("--serve-budget-gib", type=float, default=1.0,
                    help="HBM admission budget of the served stream (fields + tables of resident requests)")
    return ap.parse_args()


def problems_for(args):
    prec = W.PREC_C128 if args.precision == "c128" else W.PREC_C64
    store = "complex128" if prec == W.PREC_C128 else "complex64"
    if args.workload == "config4":
        return W.config4_problems(nsteps=args.steps, nfreq=args.nfreq, precision=prec), (
            f"config4: {args.nfreq} frequencies log-spaced 20-500 Hz, dz=lambda/8 (Nz 320-4096), "
            "Ntheta 256-1024, Munk-like profile over a periodic 2000-200 m wedge, fluid bottom "
            f"1700 m/s rho 1.5 0.5 dB/lambda, {store} field, FP64 arithmetic, batched")
    p = W.config2(nsteps=args.steps, precision=prec)
    return [p], ("config2: 100 Hz, Nz=2048, Ntheta=512, Munk-like profile over a periodic wedge, "
                 f"{store} field, FP64 arithmetic")


def measured_traffic(kernel_name, first_frac):
    """HBM bytes per launch of a kernel from the committed counter summary,
    in a launch mix with a fraction first_frac of first steps of a call, or
    None if the kernel source changed since the counters were taken."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "config4_batch_hbm_traffic.md")
    src = os.path.join(ROOT, "paper_1711_00005_amd", "csrc", "pe3d_kernels.hip")
    try:
        txt = open(prof).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    rec = dict(l.split()[0:2] for l in txt.splitlines() if l.startswith("kernel_sha256"))
    if rec.get("kernel_sha256") != sha:
        return None
    rec = {}
    for l in txt.splitlines():
        f = l.split()
        if len(f) == 4 and f[0] == "traffic_bytes" and kernel_name == f[1]:
            rec[f[2]] = int(f[3])
    if "steady" not in rec:
        return None
    return int(round((1.0 - first_frac) * rec["steady"] + first_frac * rec.get("first", rec["steady"])))


def march_steps(P, ms, us, nsteps, chunk, use_graph):
    done = 0
    while done < nsteps:
        k = min(chunk, nsteps - done)
        P.march_batch(ms, k, us, use_graph=use_graph)
        done += k


def _oracle_one_step(p):
    import oracle as O
    t0 = time.perf_counter()
    st = O.setup(p.env, p.grid, p.f_hz)
    u0 = O.starter(st, p.zs)
    u1 = O.step(st, u0, 0)
    return u1, time.perf_counter() - t0


def cpu_baseline(probs, sample_every: int):
    """The oracle (complex128 NumPy) on a bounded sample: one range step of
    every `sample_every`-th problem from its starter, one process per
    problem over the host cores this process may use (at most 16), as the
    paper spreads frequencies over MPI ranks.  Runs before the GPU is
    touched (the worker processes are forked)."""
    import multiprocessing as mp
    sample = probs[::sample_every]
    pts = sum(p.points for p in sample)
    cores = max(1, min(len(sample), len(os.sched_getaffinity(0)), 16))
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        t0 = time.perf_counter()
        res = pool.map(_oracle_one_step, sample, chunksize=1)
        dt = time.perf_counter() - t0
    outs = [r[0] for r in res]
    busy = sum(r[1] for r in res)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=pts / dt, unit=UNIT, cores=cores, cpu_model=model, kind="oracle",
                sample=f"1 range step of {len(sample)} of the {len(probs)} problems "
                       f"(every {sample_every}th, {pts} points) from the starter, one process "
                       f"per problem on {cores} cores",
                single_core_value=pts / busy), sample, outs


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); every problem of the "
              "batch is independent, so N GPUs would each run their own share with no exchange.",
              file=sys.stderr)
        sys.exit(2)
    probs, workload = problems_for(args)
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle), before the GPU is initialised")
        every = 4 if len(probs) >= 16 else 1
        cpu = cpu_baseline(probs, every)
        log(f"oracle {cpu[0]['value']:.3e} pt*steps/s on {cpu[0]['cores']} cores")

    import torch
    from paper_1711_00005_amd import pe3d as P

    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    torch.cuda.set_device(0)
    npts = sum(p.points for p in probs)
    log(f"workload: {len(probs)} problems, {npts} points")
    tuned = None
    if args.tune:
        from paper_1711_00005_amd import tune as T
        t0 = time.perf_counter()
        cache = {}
        for i, p in enumerate(probs):
            key = (p.grid.nz, p.grid.ntheta, p.grid.precision)
            if key not in cache:
                cache[key] = T.tune(p.env, p.grid, p.f_hz)[0]
            g = cache[key]
            probs[i] = dataclasses.replace(p, grid=dataclasses.replace(
                p.grid, depth_lanes=g.depth_lanes, azimuth_lanes=g.azimuth_lanes))
        tuned = dict(shapes=len(cache), seconds=round(time.perf_counter() - t0, 2))
        log(f"tuned {len(cache)} shapes in {tuned['seconds']} s")
    variants = None
    if not args.no_tune_azimuth:
        # azimuth solver per Ntheta class, measured inside batched launches
        # near the source and half-way through the march
        from paper_1711_00005_amd import tune as T
        t0 = time.perf_counter()
        tuned_probs, variants = T.tune_batch_azimuth(probs, far=max(1, probs[0].nsteps // 2) if len(probs) == 1
                                                     else 500)
        chosen = [c["chosen"] for c in variants["classes"].values()]
        # the per-class choice is kept only if the whole batch is faster with it
        P.set_batch_schedule(args.chains, args.group_mib << 20)
        probs, variants["whole_batch"] = T.keep_if_faster(probs, tuned_probs)
        variants.update(seconds=round(time.perf_counter() - t0, 2),
                        summary=f"{chosen.count('chunked')} classes chunked, {chosen.count('pcr')} cyclic reduction; "
                                f"kept: {variants['whole_batch']['kept']}")
        log(f"azimuth solver: {variants['summary']} ({variants['seconds']} s)")
    ms = [P.Pe3d(p.env, p.grid, p.f_hz) for p in probs]
    us = [m.starter(p.zs) for m, p in zip(ms, probs)]
    torch.cuda.synchronize()
    use_graph = not args.no_graph
    P.set_batch_schedule(args.chains, args.group_mib << 20)
    kinds = {"launches": P.PE3D_BATCH_LAUNCHES, "persistent": P.PE3D_BATCH_PERSISTENT}
    P.set_batch_kernel(kinds[args.batch_kernel])

    # ---- warmup; the graphs of the call sizes of the timed region are
    #      captured (not run) beforehand, so no capture falls inside it
    log("warmup")
    if use_graph:
        for k in {min(args.chunk, args.steps), args.steps % args.chunk}:
            if k:
                P.prepare_batch(ms, k, us)
    if args.warmup:
        march_steps(P, ms, us, args.warmup, args.chunk, use_graph)
    torch.cuda.synchronize()

    # ---- timed region
    log("timed")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    march_steps(P, ms, us, args.steps, args.chunk, use_graph)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    elapsed = max(wall, gpu_ms / 1e3)
    value = npts * args.steps / elapsed
    log(f"batched: {value:.4e} pt*steps/s, {1e3 * elapsed / args.steps:.3f} ms/step")

    # ---- per-kernel durations (same workload, direct launches bracketed by HIP
    #      events).  Each launch covers the whole batch here (one chain, one
    #      group): the kernels' own bandwidth, without the launch tails that
    #      the timed schedule overlaps across its chains.
    log("profile")
    P.set_batch_schedule(1, 0)
    P.pe3d_profile_enable(True)
    march_steps(P, ms, us, args.profile_steps, args.chunk, False)
    torch.cuda.synchronize()
    P.set_batch_schedule(args.chains, args.group_mib << 20)
    # first steps of a call in the replayed mix (they also read the neighbour columns)
    first_frac = -(-args.profile_steps // args.chunk) / args.profile_steps
    stats = P.pe3d_profile_read()
    P.pe3d_profile_enable(False)
    prof_ms = sum(s["total_ms"] for s in stats)
    kernels = []
    for s in stats:
        avg = s["total_ms"] / s["launches"]
        gbs = (s["algo_bytes"] / s["launches"]) / (avg * 1e-3) / 1e9
        kernels.append(dict(name=s["name"], launches=s["launches"], avg_ms=round(avg, 5),
                            algo_bytes_per_launch=s["algo_bytes"] / s["launches"],
                            achieved_gbs=round(gbs, 1)))
    dom = max(stats, key=lambda s: s["total_ms"])
    dom_avg = dom["total_ms"] / dom["launches"]
    dom_gbs = (dom["algo_bytes"] / dom["launches"]) / (dom_avg * 1e-3) / 1e9
    step_bytes = (64.0 if args.precision == "c128" else 32.0) * npts  # both passes, read + write
    roofline = dict(bound="hbm", achieved=round(dom_gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(dom_gbs / HBM_PEAK_GBS, 4),
                    traffic=measured_traffic(dom["name"], first_frac),
                    traffic_unit="bytes per launch",
                    algo_bytes_per_launch=dom["algo_bytes"] / dom["launches"], kernel=dom["name"],
                    step_achieved=round(step_bytes * args.steps / elapsed / 1e9, 1),
                    step_frac=round(step_bytes * args.steps / elapsed / 1e9 / HBM_PEAK_GBS, 4),
                    kernels=kernels, profiled_ms_per_step=round(prof_ms / args.profile_steps, 4),
                    profiled_schedule="whole batch per launch, direct launches on one stream",
                    timed_schedule=f"{args.chains} chains on concurrent streams, groups of <= "
                                   f"{args.group_mib} MiB of field marched through each call in turn")

    out = {"metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "storage": "complex128" if args.precision == "c128" else "complex64", "data": "synthetic",
           "config": {"workload": workload, "problems": len(probs), "grid_points": npts,
                      "graph": use_graph, "chunk_steps": args.chunk, "chains": args.chains,
                      "group_mib": args.group_mib, "batch_kernel": args.batch_kernel, "tuned_lanes": tuned,
                      "azimuth_solver_variants": variants},
           "roofline": roofline}

    # ---- the other batch kernel on the same batch, same calls
    if not args.no_persist_report:
        other = "persistent" if args.batch_kernel == "launches" else "launches"
        log(f"batch kernel {other}")
        P.set_batch_kernel(kinds[other])
        if use_graph:
            for k in {min(args.chunk, args.steps), args.steps % args.chunk}:
                if k:
                    P.prepare_batch(ms, k, us)
        march_steps(P, ms, us, args.chunk, args.chunk, use_graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record()
        march_steps(P, ms, us, args.steps, args.chunk, use_graph)
        ev1.record()
        torch.cuda.synchronize()
        el = max(time.perf_counter() - t0, ev0.elapsed_time(ev1) / 1e3)
        ov = npts * args.steps / el
        out["batch_kernels"] = {args.batch_kernel: dict(value=value, ms_per_step=1e3 * elapsed / args.steps),
                                other: dict(value=ov, ms_per_step=1e3 * el / args.steps),
                                "wait_timeouts": P.pe3d_batch_wait_timeouts()}
        log(f"{other}: {ov:.4e} pt*steps/s, {1e3 * el / args.steps:.3f} ms/step")
        P.set_batch_kernel(kinds[args.batch_kernel])

    # ---- plain per-frequency march on the same batch
    if not args.no_plain and len(probs) > 1:
        log("plain")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for m, u in zip(ms, us):
            m.march(args.plain_steps, u)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        pv = npts * args.plain_steps / tp
        out["plain"] = dict(value=pv, steps=args.plain_steps, ms_per_step=1e3 * tp / args.plain_steps,
                            how="each problem alone, one launch per pass per step, no graph")
        out["batched_over_plain"] = value / pv
        log(f"plain: {pv:.4e} pt*steps/s -> batched/plain = {value / pv:.2f}")

    # ---- oracle baseline and parity sample
    if cpu is not None:
        cb, sample, outs = cpu
        out["cpu_baseline"] = cb
        errs = []
        for p, ref in zip(sample, outs):
            m = P.Pe3d(p.env, p.grid, p.f_hz)
            u = m.starter(p.zs)
            m.march(1, u)
            torch.cuda.synchronize()
            got = u.cpu().numpy().astype(np.complex128)
            errs.append(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
            m.close()
        out["parity_sample"] = dict(max_rel_l2=max(errs), problems=len(errs), steps=1,
                                    reference="complex128 oracle")
        log(f"oracle {cb['value']:.3e} pt*steps/s; parity max rel L2 {max(errs):.2e}")

    for m in ms:
        m.close()
    del us

    # ---- served stream (Poisson arrivals at 200/s, continuous batching)
    if not args.no_serve:
        from paper_1711_00005_amd.serve import Pe3dBackend, Scheduler, report
        tr = W.config5_trace(n=args.serve_requests, rate_hz=200.0, seed=0)
        tr = [W.Request(r.rid, r.arrival_s, W.Problem(r.problem.env, r.problem.grid, r.problem.f_hz,
                                                      r.problem.zs,
                                                      max(1, int(math.ceil(r.problem.nsteps * args.serve_range_scale))),
                                                      r.problem.name)) for r in tr]
        log(f"serve: {len(tr)} requests")
        budget = int(args.serve_budget_gib * (1 << 30))
        skind = args.serve_batch_kernel or args.batch_kernel
        P.set_batch_kernel(kinds[skind])
        sch = Scheduler(Pe3dBackend(use_graph=args.serve_graph), budget, args.serve_chunk,
                        backlog_chunk_steps=args.serve_backlog_chunk)
        t0 = time.perf_counter()
        recs = sch.run(tr)
        rep = report(recs, time.perf_counter() - t0)
        rep["wait_timeouts"] = P.pe3d_batch_wait_timeouts()
        rep.update(rate_hz=200.0, budget_bytes=budget, chunk_steps=args.serve_chunk,
                   backlog_chunk_steps=sch.Kb, backlog_iterations=sch.backlog_iterations,
                   graph=args.serve_graph, batch_kernel=skind, max_resident=sch.max_resident,
                   range_scale=args.serve_range_scale,
                   trace="config5 seed 0: f~U(20,400) Hz, zs~U(10,500) m, width in {30,90,360} deg, "
                         "range~U(2,20) km scaled by range_scale, Nz=clamp(ceil64(6.4 f),128,4096), "
                         "Ntheta by sqrt(f) and width, dr=clamp(1500/f,2,75) m")
        out["serving"] = rep
        log(f"serve: p50 {rep['p50_latency_s']:.3f} s, p99 {rep['p99_latency_s']:.3f} s, "
            f"{rep['throughput_pt_steps_per_s']:.3e} pt*steps/s served of "
            f"{rep['offered_pt_steps_per_s']:.3e} offered, makespan {rep['makespan_s']:.2f} s")
    if args.precision_study:
        out["precision_study"] = precision_study(P)
    if args.nx2d_report:
        out["nx2d_report"] = nx2d_report(P)
    if args.range_report:
        out["range_report"] = range_report(P)
    print(json.dumps(out), flush=True)


def precision_study(P):
    """Config 2 (Nz 2048, Ntheta 512, 100 Hz) marched to 5000 steps (50 km) in
    complex64 (FP64 arithmetic) and complex128 on the GPU; at every 500 steps
    the field on the stored sample nodes (every 4th azimuth, 16th depth) is
    compared with the complex128 oracle: relative L2 over the samples, and
    the TL difference |20 log10(|u_gpu| / |u_orc|)| (RMS and max, dB) over
    the samples within 60 dB of the oracle's full-field peak."""
    import torch
    path = os.path.join(ROOT, "tests", "golden", "config3_oracle_samples.npz")
    if not os.path.exists(path):
        log("precision study: no stored oracle samples")
        return None
    g = np.load(path)
    cps = [int(c) for c in g["checkpoints"]]
    ts, zs = int(g["th_stride"]), int(g["z_stride"])
    res = dict(workload="config2 to 5000 steps (50 km)", checkpoints=cps,
               reference="complex128 oracle, sampled every 4th azimuth and 16th depth")
    for prec, name in ((W.PREC_C64, "complex64"), (W.PREC_C128, "complex128")):
        p = W.config2(nsteps=max(cps), precision=prec)
        m = P.Pe3d(p.env, p.grid, p.f_hz)
        u = m.starter(p.zs)
        rel, tl_rms, tl_max = [], [], []
        j = 0
        t0 = time.perf_counter()
        for c in cps:
            m.march(c - j, u)
            j = c
            torch.cuda.synchronize()
            us = u.cpu().numpy().astype(np.complex128)[::ts, ::zs]
            ref = g[f"u{c}"]
            rel.append(float(np.linalg.norm(us - ref) / np.linalg.norm(ref)))
            keep = np.abs(ref) >= 1e-3 * float(g[f"peak{c}"])
            d = np.abs(20.0 * np.log10(np.abs(us[keep]) / np.abs(ref[keep])))
            tl_rms.append(float(np.sqrt(np.mean(d * d))))
            tl_max.append(float(d.max()))
        res[name] = dict(rel_l2=rel, tl_rms_db=tl_rms, tl_max_db=tl_max,
                         seconds=round(time.perf_counter() - t0, 3))
        log(f"precision {name}: rel L2 {['%.2e' % x for x in rel]}")
        m.close()
    return res


def nx2d_report(P, nsteps=2000, every=500):
    """The config-2 wedge (Nz 2048, Ntheta 512, 100 Hz, complex64) marched
    nsteps in the full 3D mode and in the N x 2D mode (Y = 0) from the same
    starter: GPU time per step of each (plain march, HIP events), and at every
    `every` steps the TL difference 20 log10(|u_2d| / |u_3d|) in dB (RMS, max
    and the fraction of nodes beyond 3 dB) over the nodes within 60 dB of the
    3D field's peak, the 3D field taken as the reference."""
    import torch
    base = W.config2(nsteps=nsteps, precision=W.PREC_C64)
    res = dict(workload=f"config2 wedge, {nsteps} steps ({nsteps * base.grid.dr / 1000:.0f} km), complex64",
               checkpoints=list(range(every, nsteps + 1, every)))
    ms, us = {}, {}
    for name, mode in (("3d", W.MODE_3D), ("nx2d", W.MODE_NX2D)):
        g = dataclasses.replace(base.grid, mode=mode)
        ms[name] = P.Pe3d(base.env, g, base.f_hz)
        us[name] = ms[name].starter(base.zs)
    for name in ms:  # warm-up (module load, first launches), then rewind
        v = us[name].clone()
        ms[name].march(5, v)
        ms[name].set_step(0)
    torch.cuda.synchronize()
    ms_per_step = {k: 0.0 for k in ms}
    rms, mx, frac3 = [], [], []
    for j in range(0, nsteps, every):
        for name in ms:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ms[name].march(every, us[name])
            e1.record()
            torch.cuda.synchronize()
            ms_per_step[name] += e0.elapsed_time(e1) / nsteps
        a3 = us["3d"].abs().double().cpu().numpy()
        a2 = us["nx2d"].abs().double().cpu().numpy()
        keep = a3 >= 1e-3 * a3.max()
        d = 20.0 * np.log10(np.maximum(a2[keep], 1e-300) / a3[keep])
        rms.append(float(np.sqrt(np.mean(d * d))))
        mx.append(float(np.abs(d).max()))
        frac3.append(float(np.mean(np.abs(d) > 3.0)))
    res.update(ms_per_step={k: round(v, 5) for k, v in ms_per_step.items()},
               speedup_nx2d=round(ms_per_step["3d"] / ms_per_step["nx2d"], 3),
               tl_diff_rms_db=rms, tl_diff_max_db=mx, frac_beyond_3db=frac3)
    log(f"nx2d vs 3d: {ms_per_step}, TL diff RMS {['%.2f' % x for x in rms]} dB")
    for m in ms.values():
        m.close()
    return res


def range_report(P, nsteps=1000):
    """GPU time per step of the config-2 grid (Nz 2048, Ntheta 512, 100 Hz,
    complex64, plain march, HIP events over nsteps after a warm-up) over the
    range-independent wedge, over the range- and azimuth-dependent sloping
    bottom (per-step water-node update + the same two passes) and under the
    range-dependent water of an ocean front (a profile row every 1 km: the
    per-step row selection + the same two passes with that row's tables)."""
    import torch
    res = {}
    for name, p in (("wedge_range_independent", W.config2(nsteps=nsteps)),
                    ("slope_range_dependent", W.config2_slope(nsteps=nsteps)),
                    ("front_range_dependent_water", W.config2_front(nsteps=nsteps))):
        m = P.Pe3d(p.env, p.grid, p.f_hz)
        u = m.starter(p.zs)
        m.march(5, u.clone())
        m.set_step(0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        m.march(nsteps, u)
        e1.record()
        torch.cuda.synchronize()
        msps = e0.elapsed_time(e1) / nsteps
        res[name] = dict(ms_per_step=round(msps, 5),
                         pt_steps_per_s=p.points / (msps * 1e-3))
        if name == "wedge_range_independent":
            # the same lone problem through the batched march: calls of 100
            # steps, each replayed from a captured graph
            m.set_step(0)
            P.prepare_batch([m], 100, [u])
            torch.cuda.synchronize()
            e0.record()
            for _ in range(nsteps // 100):
                P.march_batch([m], 100, [u], use_graph=True)
            e1.record()
            torch.cuda.synchronize()
            g = e0.elapsed_time(e1) / (100 * (nsteps // 100))
            res["wedge_range_independent_graph"] = dict(ms_per_step=round(g, 5),
                                                        pt_steps_per_s=p.points / (g * 1e-3),
                                                        how="pe3d_march_batch of the one problem, "
                                                            "calls of 100 steps replayed from a graph")
            # and with the persistent batch kernel (one launch per call)
            P.set_batch_kernel(P.PE3D_BATCH_PERSISTENT)
            try:
                P.prepare_batch([m], 100, [u])
                P.march_batch([m], 100, [u], use_graph=True)
                torch.cuda.synchronize()
                e0.record()
                for _ in range(nsteps // 100):
                    P.march_batch([m], 100, [u], use_graph=True)
                e1.record()
                torch.cuda.synchronize()
            finally:
                P.set_batch_kernel(P.PE3D_BATCH_LAUNCHES)
            g = e0.elapsed_time(e1) / (100 * (nsteps // 100))
            res["wedge_range_independent_persistent"] = dict(ms_per_step=round(g, 5),
                                                             pt_steps_per_s=p.points / (g * 1e-3),
                                                             how="pe3d_march_batch of the one problem with "
                                                                 "the persistent kernel, calls of 100 steps "
                                                                 "replayed from a graph")
        m.close()
    res.update(workload="config2 grid: periodic wedge vs slope_env (d0 400 m, 3 deg plane slope "
                        "clipped to 30-2500 m, rows every 250 m) vs front_env (the wedge under a Munk "
                        "profile whose axis rises 1000 -> 600 m and minimum speed 1490 -> 1500 m/s "
                        "over 60 km, a row every 1 km), complex64, plain march",
               slowdown_range_dependent=round(res["slope_range_dependent"]["ms_per_step"]
                                              / res["wedge_range_independent"]["ms_per_step"], 3),
               slowdown_range_dependent_water=round(res["front_range_dependent_water"]["ms_per_step"]
                                                    / res["wedge_range_independent"]["ms_per_step"], 3))
    log(f"range report: {res}")
    return res


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Throughput of the coupled LBM-DEM time step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload dilute|small|dense]

A step is one full coupled time step (Alg. 1 of the paper): moments, Du_f/Dt
and grad P, n_int interaction subcycles (added mass, drag, pressure and
gravity forces with interpolation and spreading, DEM contact + lubrication
substeps, rebinning and the volume-fraction update) and the fused GNS-LBM
stream-collide. Inputs are resident in HBM before timing starts.

Prints one JSON line: MLUPS (cells x steps / s / 1e6) of the whole job, the
HBM roofline of the dominant kernel (HIP events on the library's stream,
algorithmic bytes per launch), and the FP64 CPU oracle timed on a bounded
sample of the same workload on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def workload(name, seed):
    from paper_1711_00336_amd import inputs as I
    if name == "dilute":
        return I.case_dilute_periodic(seed, n=128, eps_p=0.05, d=0.8, precision="fp32dev")
    if name == "dilute64":
        return I.case_dilute_periodic(seed, n=128, eps_p=0.05, d=0.8, precision="fp64")
    if name == "small":
        return I.case_small_walled(seed)
    raise SystemExit(f"unknown workload {name}")


def kernel_bytes(case):
    """Algorithmic HBM bytes per launch of each timed kernel class.

    stream_collide: per cell 19 PDF reads + 19 PDF writes + solid fraction +
    3 force components, in the storage precision."""
    rs = 4 if case.params.precision == "fp32dev" else 8
    nc = case.params.n[0] * case.params.n[1] * case.params.n[2]
    return {"stream_collide": nc * (19 + 19 + 1 + 3) * rs}


def cpu_baseline(case, budget_s=20.0):
    """The FP64 oracle on a bounded sample: a 32^3 box of the same workload
    (same solid fraction, diameter, density ratio, tau, n_int, n_dem)."""
    from paper_1711_00336_amd import inputs as I
    from oracle import oracle as O
    if not os.path.exists(O._LIB):
        O.build(force=False)
    p = case.params
    if case.name.startswith("periodic"):
        eps = float(case.name.split("eps")[-1])
        d = float(case.particles.d[0])
        rr = float(case.particles.rho_p[0])
        sample = I.case_settling(0, 32, eps, d, rr, precision="fp64")
        sample.params = sample.params.copy(tau=p.tau, n_int=p.n_int, n_dem=p.n_dem, h_c=p.h_c)
        desc = f"32^3 periodic box, eps_p={eps}, d={d}, {sample.particles.n} spheres"
    else:
        sample = case
        desc = f"{case.name}"
    o = O.Oracle(sample.params, sample.particles)
    nc = sample.params.n[0] * sample.params.n[1] * sample.params.n[2]
    o.step(1)  # warm-up
    t0 = time.perf_counter()
    k = 0
    while True:
        o.step(1)
        k += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": nc * k / dt / 1e6, "unit": "MLUPS", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{desc}, FP64 oracle, {k} coupled steps in {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="dilute")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1 "
              "(the spatial decomposition across GPUs is a design, not part of this build)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1711_00336_amd import lbdem

    case = workload(args.workload, args.seed)
    print(f"[bench] workload {case.name}: cells {np.prod(case.params.n)}, particles {case.particles.n}",
          file=sys.stderr, flush=True)
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    dom = lbdem.Domain(case.params, stream=stream.cuda_stream)
    dom.add(case.particles)
    nc = dom.nc

    dom.lbdem_step(args.warmup)
    dom.lbdem_sync()
    torch.cuda.synchronize()
    print(f"[bench] warmup {args.warmup} steps done", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    dom.lbdem_step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    dom.lbdem_sync()
    print(f"[bench] timed {args.steps} steps in {dt:.3f} s", file=sys.stderr, flush=True)

    # per-kernel-class device time (HIP events on the library's stream)
    ksteps = max(5, min(args.steps, 50))
    dom.lbdem_set_timing(True)
    dom.lbdem_step(ksteps)
    dom.lbdem_sync()
    times = {}
    for name in lbdem.KCLASS:
        ms, n = dom.lbdem_kernel_time(name)
        times[name] = {"ms_per_step": ms / ksteps, "launches_per_step": n / ksteps,
                       "avg_launch_ms": (ms / n if n else 0.0)}
    dom.lbdem_set_timing(False)
    diag = dom.lbdem_diagnostics()
    dom.close()

    kb = kernel_bytes(case)
    sc = times["stream_collide"]
    achieved = kb["stream_collide"] / (sc["avg_launch_ms"] * 1e-3) / 1e9 if sc["avg_launch_ms"] > 0 else 0.0
    roofline = {"bound": "hbm", "kernel": "stream_collide", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None, "bytes_per_launch": kb["stream_collide"],
                "avg_launch_ms": round(sc["avg_launch_ms"], 5)}

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(case, args.cpu_budget)

    ms_per_step = dt / args.steps * 1e3
    out = {
        "metric": "MLUPS per coupled LBM-DEM step (whole job)",
        "value": round(nc * args.steps / dt / 1e6, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if case.params.precision == "fp32dev" else "f64",
        "data": "synthetic",
        "config": {"workload": case.name, "cells": int(nc), "particles": int(case.particles.n),
                   "n_int": case.params.n_int, "n_dem": case.params.n_dem,
                   "pdf_storage": "f32 deviation" if case.params.precision == "fp32dev" else "f64 deviation",
                   "particle_integration": "f64", "tau": case.params.tau},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": {k: {kk: round(vv, 5) for kk, vv in v.items()} for k, v in times.items()},
        "u_ps": diag["u_ps"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

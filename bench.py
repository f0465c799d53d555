"""Benchmark of the sDUGKS step on one MI355X.

Workload: lid-driven cavity, 256 x 256 tanh-stretched quads (stretching 1.5),
Re = 1000 (lid 0.1, nu = 1e-4), CFL 0.5, D2Q9, FP64, from rest.  A step is
one full time step of the scheme (every kernel of the hot path) with the
convergence residual evaluated every 1000 steps, as in the paper's cavity
case.  Prints one JSON line: MLUPS (cell updates per second / 1e6), the HBM
roofline of the step kernels, and the CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
RESIDUAL_INTERVAL = 1000
# Compulsory bytes per cell update of the fused FP64 step on quads, same-step
# macroscopic flux: f (72 B) and W (24 B) read and written once, plus the
# geometry read once (centroid 16, 1/V 8, four neighbours x (index 4 + two
# LSQ weights 16), two faces x (owner/neighbour 8 + l*n 16 + midpoint 16)).
ALG_BYTES_PER_CELL = 2 * (72 + 24) + 184


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=4000)
    p.add_argument("--warmup", type=int, default=200)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    return p.parse_args()


def cpu_baseline(mesh, bcs, kw, target_s):
    import oracle
    o = oracle.Oracle(mesh, bcs, **kw)
    t = time.perf_counter()
    o.step(5)
    per_step = (time.perf_counter() - t) / 5
    n = max(5, int(target_s / per_step))
    t = time.perf_counter()
    o.step(n)
    el = time.perf_counter() - t
    return {"value": o.n_cells * n / el / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"cavity 256x256 FP64, {n} steps from step 5 of a run from rest (single thread, gcc -O2)"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the multi-GPU design is described, not built.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import meshgen
    from paper_2007_07347_amd import sdugks

    torch.cuda.set_device(0)
    mesh, bcs = meshgen.cavity(256, beta=1.5, U=0.1)
    kw = dict(nu=0.1 / 1000, cfl=0.5)
    s = sdugks.Solver(mesh, bcs, **kw)
    nc = s.n_cells
    s.step(a.warmup)
    torch.cuda.synchronize()

    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    done = 0
    eps = None
    t0 = time.perf_counter()
    start.record()
    while done < a.steps:
        k = min(RESIDUAL_INTERVAL, a.steps - done)
        s.step(k)
        done += k
        if k == RESIDUAL_INTERVAL:
            eps = s.residual()            # synchronises, as a solve does every 1000 steps
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(end)
    mlups = nc * a.steps / (ms / 1e3) / 1e6

    # per-kernel durations with HIP events on the solver's stream
    kt = s.step_profiled(min(a.steps, 2000))
    step_ms = sum(kt.values())
    dominant = max(kt, key=kt.get)
    achieved = ALG_BYTES_PER_CELL * nc / (step_ms / 1e3) / 1e9
    roof = {"bound": "hbm", "kernel": "+".join(kt), "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "bytes_per_cell": ALG_BYTES_PER_CELL, "kernel_ms": {k: round(v, 5) for k, v in kt.items()},
            "dominant": dominant}
    out = {
        "metric": "MLUPS (D2Q9 cell-updates/s) & %HBM peak; p50/p99 time-to-steady under load",
        "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms / a.steps, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "lid-driven cavity 256x256 tanh(1.5) quads, Re 1000, CFL 0.5, D2Q9, FP64, "
                               "residual every 1000 steps",
                   "cells": nc, "dt": s.dt, "tau": s.tau, "residual_at_end": eps},
        "roofline": roof,
        "wall_s": round(wall, 3),
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(mesh, bcs, kw, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

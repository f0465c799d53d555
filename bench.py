"""Benchmark of the sDUGKS step on one MI355X.

Headline workload: lid-driven cavity, 256 x 256 tanh-stretched quads
(stretching 1.5), Re = 1000 (lid 0.1, nu = 1e-4), CFL 0.5, D2Q9, FP64, from
rest.  A step is one full time step of the scheme (the fused step kernel) with
the convergence residual evaluated every 1000 steps, as in the paper's cavity
case.  The tile schedule comes from the autotuner.

The one JSON line also carries: the same workload with FP32-deviation storage;
the batched form on 64 uneven cavities (edge log-uniform in [32, 512] cells,
Re uniform in [100, 5000], FP32 deviation storage) against stepping the same
instances one after another; the continuous-batching serving loop on a finite
seeded request trace with p50/p99 time-to-steady, against the per-case FP64
loop; steady drag, lift, stagnation pressure and recirculation length of the
circular cylinder at Re = 10, 20, 40 and its Strouhal number and mean drag at
Re = 60, 80, 100; throughput on the 200,000-triangle cylinder O-grid in both
storage forms; the original half-step DUGKS against the simplified scheme
(cost per step on the headline cavity, shear-wave accuracy, largest stable
CFL against Dt/tau); the share of the HBM peak on a 2048 x 2048 cavity whose
working set is far beyond the Infinity Cache; the HBM roofline of the step
kernel; and the CPU oracle timed on a bounded sample of the headline workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra | --sections a,b,...]
                    [--schedule T,B] [--batch-schedule T,B] [--cylinder-schedule T,B]
    python bench.py --copy-calibration MB     (plain device copy, for counter scaling, and copy,
                                               read and write bandwidth)
    python bench.py --large-only              (only the 2048 x 2048 cavity, for HBM counters)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
RESIDUAL_INTERVAL = 1000
# Compulsory bytes per cell update of the step on quads with the same-step
# macroscopic flux: f and W read and written once (FP64: 2 * (72 + 24);
# FP32 deviation: 2 * (36 + 24)) plus the geometry read once (centroid 16,
# 1/V 8, four neighbours x (index 4 + two LSQ weights 16), two faces x
# (owner/neighbour 8 + l*n 16 + midpoint 16) = 184).
ALG_BYTES = {"f64": 2 * (72 + 24) + 184, "fp32dev": 2 * (36 + 24) + 184}
# triangles: three faces per cell, 144 B of geometry per cell instead of 184
ALG_BYTES_TRI = {"f64": 2 * (72 + 24) + 144, "fp32dev": 2 * (36 + 24) + 144}
_CSRC = os.path.join(ROOT, "paper_2007_07347_amd", "csrc")
# the sources each step kernel is compiled from (its own file and the shared
# device helpers): the traffic counters of a kernel hold while these are unchanged
KERNEL_SOURCES = {
    "k_step_tiled": ("step_tiled.hip", "step_common.h"),
    "k_step_batch": ("step_tiled.hip", "step_common.h"),
    "k_step_cart": ("step_cart.hip", "step_common.h"),
    "k_step_batch_cart": ("step_cart.hip", "step_common.h"),
}
TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")
SECTIONS = ("cavity256", "converge", "serving", "cylinder200k", "original", "large",
            "converge_cylinder", "cylinder", "serving_narrow")
# Run only when named, so that the default run stays within a few minutes:
# the 200k cylinder to its stopping rule (about 2.7M steps, two minutes),
# the cylinder physics (Re 10 to 100) and the narrower serving trace
DEFAULT_SECTIONS = SECTIONS[:6]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=2000)
    p.add_argument("--warmup", type=int, default=40)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-extra", action="store_true", help="headline workload only")
    p.add_argument("--sections", default=",".join(DEFAULT_SECTIONS),
                   help="extra sections to run after the headline, comma-separated from " + ",".join(SECTIONS))
    p.add_argument("--schedule", default="", metavar="T,B|structured",
                   help="schedule of the 256 x 256 cavity forms instead of the autotuner's pick: the general step's "
                        "tile cells and threads per workgroup, or the structured step (for counter runs, where the "
                        "profiler distorts the autotuner's timings)")
    p.add_argument("--batch-schedule", default="", metavar="T,B|structured",
                   help="schedule of every member of the batched headline instead of the batch autotuner's pick")
    p.add_argument("--cylinder-schedule", default="", metavar="T,B",
                   help="schedule of both precisions on the 200,000-triangle cylinder instead of the autotuner's "
                        "picks (for profiled runs)")
    p.add_argument("--headline-precision", default="fp32dev", choices=("fp32dev", "fp32neq"),
                   help="FP32 storage form of the batched headline: FP32 face arithmetic (fp32dev) or FP64 "
                        "arithmetic (fp32neq)")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MB")
    p.add_argument("--large-only", action="store_true",
                   help="only the 2048 x 2048 cavity (working set above 2 GB), for HBM counters")
    return p.parse_args()


def code_hash(text):
    """sha1 (16 hex digits) of a C++ source with comments, blank lines and
    trailing blanks removed: edits to comments leave the compiled kernel, and
    so this hash, unchanged."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines()]
    return hashlib.sha1("\n".join(ln for ln in lines if ln).encode()).hexdigest()[:16]


def kernel_hash(kernel="k_step_tiled"):
    """code_hash of the sources of a step kernel, named with or without its
    template arguments ("k_step_batch_cart<1>" or "k_step_batch_cart")."""
    text = []
    for f in KERNEL_SOURCES[kernel.split("<")[0]]:
        with open(os.path.join(_CSRC, f)) as fh:
            text.append(fh.read())
    return code_hash("\n".join(text))


def measured_traffic(workload, schedule=None):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source and with this tile schedule; else None."""
    try:
        with open(TRAFFIC) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get(workload)
    if not e or e.get("kernel_code_sha1") != kernel_hash(e.get("kernel", "k_step_tiled")):
        return None
    if schedule is not None and e.get("schedule") not in (None, schedule):
        return None
    return e.get("bytes_per_launch")


def copy_calibration(mb):
    """Five plain device copies of mb MiB (the launches the counter scaling is
    taken from), then the HBM bandwidth that plain torch kernels reach on this
    device: copy, read-only sum (FP64, torch's faster reduction) and fill, 20
    launches each after one warm-up."""
    import torch
    n = mb * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()

    def tbs(f, nbytes, reps=20):
        f()
        ms = time_steps(lambda k: [f() for _ in range(k)], reps) / reps
        return round(nbytes / (ms / 1e3) / 1e12, 3)

    print(json.dumps({"copy_bytes_each_way": n * 4, "launches": 5,
                      "copy_TBs": tbs(lambda: b.copy_(a), 2 * n * 4),
                      "read_TBs": tbs(lambda: a.view(torch.float64).sum(), n * 4),
                      "write_TBs": tbs(lambda: b.fill_(1.0), n * 4)}), flush=True)


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def paper_cylinder():
    """The paper's own cylinder results from tests/golden/cylinder_present.txt:
    ({Re: (Cd, L/R)} steady, {Re: (Cd, L/R, St)} unsteady)."""
    steady, unsteady = {}, {}
    with open(os.path.join(ROOT, "tests", "golden", "cylinder_present.txt")) as fh:
        for line in fh:
            f = line.split("#", 1)[0].split()
            if f:
                vals = tuple(float(v) for v in f[2:] if v != "-")
                (steady if f[0] == "steady" else unsteady)[int(f[1])] = vals
    return steady, unsteady


def time_steps(step, n, stream=None):
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    step(n)
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b)


def headline(sdugks, autotune, meshgen, a, precision):
    import torch
    mesh, bcs = meshgen.cavity(256, beta=1.5, U=0.1)
    kw = dict(nu=0.1 / 1000, cfl=0.5, precision=precision)
    if a.schedule == "structured":
        sched = dict(autotune.STRUCTURED)
    elif a.schedule:
        t, b = (int(x) for x in a.schedule.split(","))
        sched = {"tile_cells": t, "block_threads": b, "structured": 1}
    else:
        sched, _ = autotune.autotune(mesh, bcs, steps=200, **kw)
    s = sdugks.Solver(mesh, bcs, **sched, **kw)
    nc = s.n_cells
    # an even warm-up long enough to capture both step graphs for the buffer
    # index the timed region starts from
    s.step(max(66, a.warmup + (a.warmup & 1)))
    torch.cuda.synchronize()
    done, eps = 0, None
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
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
    # per-launch HIP events on the solver's stream, same workload, after the timed region
    kt = s.step_profiled(min(a.steps, 2000))
    return s, mesh, bcs, kw, sched, nc, ms, wall, eps, kt


BATCH_WORKLOAD = ("64 lid-driven cavities, tanh(1.5) quads with edge log-uniform in [32, 512] (seed 2026), Re uniform "
                  "in [100, 5000], lid 0.1, CFL 0.5, D2Q9, FP32 deviation storage with FP64 macros, batched: one "
                  "graph-replayed fused launch per step over all members, every member's residual every 1000 steps")


def batch_problems(sdugks, meshgen, seed=2026, n_inst=64, precision=None):
    """The 64 uneven cavities of the batched workload: (mesh, bcs, kw) each."""
    import numpy as np
    rng = np.random.default_rng(seed)
    sizes = meshgen.log_uniform_int(rng, 32, 512, size=n_inst)
    res = rng.uniform(100.0, 5000.0, size=n_inst)
    prec = sdugks.FP32DEV if precision is None else precision
    return [(*meshgen.cavity(int(n), beta=1.5, U=0.1), dict(nu=0.1 / re, cfl=0.5, precision=prec))
            for n, re in zip(sizes, res)]


def batch_headline(sdugks, autotune, meshgen, a, seed=2026, n_inst=64):
    """The headline: 64 uneven cavities advanced by one batched launch per
    step (graph replays), the batched residual of every member every 1000
    steps.  Timed with HIP events on the batch's stream; the step kernel is
    the only kernel between residual checks, so its average launch duration
    is the timed region over the step count (the residual launches add well
    under 0.1 %).  Then the same members stepped one after another (the plain
    per-instance loop) for comparison."""
    import torch
    prec = sdugks.FP32NEQ if a.headline_precision == "fp32neq" else sdugks.FP32DEV
    problems = batch_problems(sdugks, meshgen, seed, n_inst, precision=prec)
    cells = int(sum(len(m["cell_ptr"]) - 1 for m, _, _ in problems))
    if a.batch_schedule == "structured":
        sched, table = dict(autotune.STRUCTURED), []
    elif a.batch_schedule:
        t, bt = (int(x) for x in a.batch_schedule.split(","))
        sched, table = {"tile_cells": t, "block_threads": bt, "structured": 1}, []
    else:
        sched, table = autotune.autotune_batch(problems)
    # the members live on the batch's stream, as in a serving process with one
    # stream for its batch: the batch then has no member streams to order after
    stream = torch.cuda.Stream()
    solvers = [sdugks.Solver(mesh, bcs, stream=stream, **sched, **kw) for mesh, bcs, kw in problems]
    ws = sum(s.workspace.numel() for s in solvers)
    b = sdugks.Batch(solvers, stream=stream)
    # the warm-up captures the batch's graphs (2 to 32 steps, all at the first call) and
    # replays the longest and the shortest, then the odd step
    warm = max(35, a.warmup)
    b.step(warm)
    b.residuals()
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    done, eps = 0, None
    t0 = time.perf_counter()
    start.record(stream)
    while done < a.steps:
        k = min(RESIDUAL_INTERVAL, a.steps - done)
        b.step(k)
        done += k
        if k == RESIDUAL_INTERVAL:
            eps = b.residuals()           # one launch pair and one synchronisation for all members
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(end)
    b.close()
    # the plain per-instance loop on the same members
    loop_steps = min(a.steps, 200, max(a.steps // 10, 20))
    for s in solvers:
        s.step(2)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(loop_steps):
        for s in solvers:
            s.step(1)
    torch.cuda.synchronize()
    ms_l = (time.perf_counter() - t1) * 1e3
    for s in solvers:
        s.close()
    return {"cells": cells, "ms": ms, "wall": wall, "eps": eps, "sched": sched, "table": table, "warm": warm,
            "working_set_MB": round(ws / 1e6, 1), "loop_steps": loop_steps, "loop_ms": ms_l}


# the serving workload's ranges: cavities 64^2 to 1024^2, cylinders 10k to 1M triangles
SERVING_TRACE = dict(n_requests=24, rate=20.0, couette_n=(8, 128), cavity_n=(64, 1024),
                     cylinder_cells=(10_000, 1_000_000), re_range=(10.0, 2000.0), cylinder_re=(10.0, 2000.0))
# a narrower trace (cavities to 256^2, cylinders to 100k triangles) on which more requests converge
SERVING_TRACE_NARROW = dict(SERVING_TRACE, cavity_n=(64, 256), cylinder_cells=(10_000, 100_000))


def serving(meshgen, seed=7, step_cap=100_000, trace_kw=None):
    """Continuous-batching serving loop on a finite seeded trace (Poisson
    arrivals at 20 per second; Couette 4 x N, N in [8, 128]; cavities N x N,
    N in [64, 1024]; cylinder O-grids of 10k to 1M triangles; Re in
    [10, 2000], Couette flow kept at Re <= 40; trace_kw narrows the ranges),
    FP32 deviation storage, a
    request whose residual stalls above the tolerance continued with FP64 arithmetic,
    instances built on a worker thread while the batch runs and every
    member's residual from one batched reduction per chunk; against the plain
    per-case FP64 loop on the same trace.  Accuracy: the velocity of each
    request served by both against the FP64 loop's (relative L2 and
    L-infinity over cells; equal step counts are not enforced, each run stops
    at its own check)."""
    import numpy as np
    from paper_2007_07347_amd import sdugks, serve
    tk = SERVING_TRACE if trace_kw is None else trace_kw
    trace = meshgen.serving_trace(seed=seed, **tk)
    rq = [serve.Request(r["rid"], r["arrival"], r["mesh"], r["bcs"], r["params"], r["kind"], r["n_cells"])
          for r in trace]
    budget = 8 << 30
    be = serve.GpuBackend()
    res_b, st_b = serve.Server(be, budget_bytes=budget, interval=1000, tol=1e-7, step_cap=step_cap,
                               keep_macros=True).run(rq)
    be.close()
    progress(f"serving: batched {st_b['converged']} converged, p50 {st_b['p50_time_to_steady_s']}")
    res_s, st_s = serve.SequentialServer(serve.GpuBackend(precision=sdugks.FP64), budget_bytes=budget, interval=1000,
                                         tol=1e-7, step_cap=step_cap, keep_macros=True).run(rq)
    r3 = lambda x: None if x is None else round(x, 3)  # noqa: E731
    acc = []
    for rb, rs, t in zip(res_b, res_s, trace):
        row = {"rid": rb.rid, "kind": rb.kind, "cells": rb.n_cells, "Re": round(t["re"], 1),
               "batched": rb.status, "fp64_loop": rs.status, "steps": [rb.steps, rs.steps]}
        if rb.macros is not None and rs.macros is not None:
            ub = np.concatenate([rb.macros[1], rb.macros[2]])
            us = np.concatenate([rs.macros[1], rs.macros[2]])
            row["velocity_rel_l2"] = float(f"{np.linalg.norm(ub - us) / np.linalg.norm(us):.3g}")
            row["velocity_rel_linf"] = float(f"{np.abs(ub - us).max() / np.abs(us).max():.3g}")
        acc.append(row)
    both = [r["velocity_rel_l2"] for r in acc if r["batched"] == r["fp64_loop"] == "converged"
            and "velocity_rel_l2" in r]
    cn, cc = tk["cavity_n"], tk["cylinder_cells"]
    return {"workload": f"{len(rq)} requests (Couette 4xN N in [8,128], cavity NxN N in [{cn[0]},{cn[1]}], cylinder "
                        f"O-grid {cc[0] // 1000}k-{cc[1] // 1000}k cells; Re 10-2000, Couette <= 40), Poisson 20/s, "
                        f"seed {seed}, residual 1e-7, cap {step_cap} steps, HBM budget 8 GiB",
            "cells": [t["n_cells"] for t in trace],
            "batched_fp32dev": {k: (r3(v) if isinstance(v, float) else v) for k, v in st_b.items()},
            "per_case_fp64_loop": {k: (r3(v) if isinstance(v, float) else v) for k, v in st_s.items()},
            "accuracy_vs_fp64_loop": {"max_velocity_rel_l2_converged_in_both": max(both) if both else None,
                                      "requests": acc}}


def cylinder_form(meshgen, n_theta=200, n_r=125, tol=1e-8):
    """Steady flow around a circular cylinder (O-grid, far field at 20
    diameters, 50,000 triangles, FP64) at Re = 10, 20, 40, each marched from
    the free stream until the velocity residual of successive checks (every
    2000 steps) is below tol: drag and lift coefficients from the wall
    momentum flux, stagnation pressure coefficient and recirculation length.
    The paper's table values (its own 75d x 50d domain and meshes) are given
    for context."""
    import math
    import numpy as np
    from paper_2007_07347_amd import cylinder, sdugks
    paper, paper_u = paper_cylinder()
    mesh, bcs = meshgen.cylinder_ogrid(n_theta, n_r, seed=0)
    rows = []
    for re in (10, 20, 40):
        t0 = time.perf_counter()
        s, r = cylinder.run_steady(sdugks, mesh, bcs, re, tol=tol, interval=2000, cfl=0.5)
        L = cylinder.recirculation_length(s, mesh, bcs, nu=0.1 / re, cfl=0.5, u0=0.1)
        th, cp = cylinder.pressure_coefficient(s, mesh, bcs)
        progress(f"cylinder Re {re}: {r['steps']} steps, C_d {r['Cd']:.4f}")
        rows.append({"Re": re, "steps": r["steps"], "residual": float(f"{r['residual']:.3g}"),
                     "Cd": round(float(r["Cd"]), 4), "Cl": float(f"{r['Cl']:.2g}"), "L_over_R": round(2.0 * L, 3),
                     "Cp_front": round(float(cp[np.argmin(np.abs(th - math.pi))]), 3),
                     "dt_over_tau": round(s.dt / s.tau, 4), "wall_s": round(time.perf_counter() - t0, 1),
                     "paper_Cd": paper[re][0], "paper_L_over_R": paper[re][1]})
        s.close()
    unsteady = []
    for re in (60, 80, 100):
        t0 = time.perf_counter()
        s, r = cylinder.run_shedding(sdugks, mesh, bcs, re, t_transient=1500.0, t_sample=500.0, cfl=0.5, kick=0.2)
        s.close()
        progress(f"cylinder Re {re}: St {r['St']:.4f}")
        unsteady.append({"Re": re, "St": round(r["St"], 4), "Cd_mean": round(r["Cd_mean"], 4),
                         "Cl_amp": round(r["Cl_amp"], 4), "steps": r["steps"], "wall_s": round(time.perf_counter() - t0, 1),
                         "St_fit": round(-3.3265 / re + 0.1816 + 1.6e-4 * re, 4),
                         "paper_Cd": paper_u[re][0], "paper_St": paper_u[re][2]})
    return {"workload": f"circular cylinder, O-grid {n_theta}x{n_r} split into {2 * n_theta * n_r} triangles, "
                        f"r 0.5..20, u_inf 0.1, FP64; steady cases to residual {tol:g}, unsteady cases "
                        f"1500 time units of transient (transverse kick 0.2 u_inf in the near wake) then 500 sampled",
            "steady": rows, "unsteady": unsteady}


def converge_done(pname, eps, steps, f64_done, f64_steps, tol, cap):
    """Stopping rule of the converge section for one form after a check: FP64
    stops at the tolerance or the cap; the FP32 deviation form at the
    tolerance or once FP64 has stopped and it has run as many steps; the FP32
    non-equilibrium form at the tolerance or at 1.5 times FP64's steps.  A
    non-finite residual stops any form."""
    if math.isnan(eps) or eps < tol:
        return True
    if pname == "f64":
        return steps >= cap
    return f64_done and steps >= f64_steps * (1.5 if pname == "fp32neq" else 1.0)


CONVERGE_CASES = ("cavity256_re1000", "cylinder200k_re40")


def converge_form(sdugks, meshgen, names=CONVERGE_CASES, tol=1e-8, interval=RESIDUAL_INTERVAL, cap=8_000_000):
    """The two stopping rules, run to the end (`names` chooses): the 256 x 256
    cavity at Re 1000 from rest and the 200,000-triangle cylinder at Re 40
    from the free stream, each in FP64 until the velocity residual (checked every 1000 steps) falls
    below 1e-8, with the two FP32 storage forms of the same case advanced
    alongside, each on a stream of its own.  The FP32 deviation form stops
    with FP64 (or earlier, at the tolerance); the FP32 non-equilibrium form,
    which has FP64 arithmetic, runs on to the tolerance itself, up to 1.5
    times FP64's steps.  Reported: steps, wall time, final residual and mass
    drift of each, whether it met the rule, and each FP32 form's velocity
    error (relative L2 and L-infinity over cells) against the converged FP64
    field; a form that stopped above the tolerance also gets its residual at
    the end (median of its last ten checks)."""
    import numpy as np
    import torch
    cases = {"cavity256_re1000": (lambda: meshgen.cavity(256, beta=1.5, U=0.1), dict(nu=1e-4, cfl=0.5, structured=2)),
             "cylinder200k_re40": (lambda: meshgen.cylinder_ogrid(400, 250, seed=0),
                                   dict(nu=0.1 / 40, cfl=0.5, u0=0.1, tile_cells=64, block_threads=256))}
    out = {"rule": f"velocity residual below {tol:g}, checked every {interval} steps; the FP32 deviation form "
                   "runs alongside FP64 for its steps, the FP32 non-equilibrium form on to the rule (cap 1.5x FP64)",
           "cases": {}}
    for name in names:
        build, kw = cases[name]
        mesh, bcs = build()
        runs = {}
        for prec, pname in ((sdugks.FP64, "f64"), (sdugks.FP32DEV, "fp32dev"), (sdugks.FP32NEQ, "fp32neq")):
            st = torch.cuda.Stream()
            s = sdugks.Solver(mesh, bcs, stream=st, precision=prec, **kw)
            runs[pname] = {"s": s, "m0": s.mass(), "steps": 0, "eps": math.inf, "hist": [], "done": False,
                           "t": None}
        t0 = time.perf_counter()
        last = t0
        while not all(r["done"] for r in runs.values()):
            for r in runs.values():
                if not r["done"]:
                    r["s"].step(interval)
            for pname, r in runs.items():
                if r["done"]:
                    continue
                r["steps"] += interval
                r["eps"] = r["s"].residual()
                r["hist"].append(r["eps"])
                f = runs["f64"]
                r["done"] = converge_done(pname, r["eps"], r["steps"], f["done"], f["steps"], tol, cap)
                if r["done"]:
                    r["t"] = time.perf_counter() - t0
            if time.perf_counter() - last > 15:
                last = time.perf_counter()
                progress(f"converge {name}: " + ", ".join(f"{p} {r['steps']} steps eps {r['eps']:.2e}"
                                                          for p, r in runs.items()))
        res = {}
        uv = {}
        for pname, r in runs.items():
            s = r["s"]
            rho, u, v = s.macros()
            uv[pname] = np.concatenate([u, v])
            res[pname] = {"steps": r["steps"], "residual": float(f"{r['eps']:.3g}"), "met_rule": bool(r["eps"] < tol),
                          "wall_s": round(r["t"], 1),
                          "mass_drift": float(f"{(s.mass() - r['m0']) / r['m0']:.4g}"),
                          "ms_per_step_alongside": round(r["t"] * 1e3 / r["steps"], 5)}
            s.close()
        for pname in ("fp32dev", "fp32neq"):
            d = uv[pname] - uv["f64"]
            res[pname]["velocity_rel_l2_vs_f64"] = float(f"{np.linalg.norm(d) / np.linalg.norm(uv['f64']):.3g}")
            res[pname]["velocity_rel_linf_vs_f64"] = float(f"{np.abs(d).max() / np.abs(uv['f64']).max():.3g}")
            if not res[pname]["met_rule"]:
                res[pname]["residual_floor"] = float(f"{np.median(runs[pname]['hist'][-10:]):.3g}")
        res["cells"] = len(mesh["cell_ptr"]) - 1
        out["cases"][name] = res
        progress(f"converge {name}: f64 {res['f64']['steps']} steps, fp32dev error "
                 f"{res['fp32dev']['velocity_rel_l2_vs_f64']}, fp32neq {res['fp32neq']['steps']} steps")
    return out


def _shear_wave_error(sdugks, meshgen, n, nu, scheme, cfl=0.5, amp=0.01, decay=0.5):
    """Decaying shear wave u = amp sin(2 pi y) e^(-nu k^2 t) on n x n
    periodic quads, run from its equilibrium state until the amplitude has
    fallen by e^-decay: relative L2 error of u at the centroids."""
    import numpy as np
    mesh, bcs = meshgen.periodic_box(n, n)
    g = sdugks.geometry(mesh, bcs, nu=nu, cfl=cfl)
    k = 2.0 * math.pi
    steps = max(1, round(decay / (nu * k * k) / g["dt"]))
    u0 = amp * np.sin(k * g["cy"])
    s = sdugks.Solver(mesh, bcs, nu=nu, cfl=cfl, scheme=scheme)
    s.set_macros(1.0, u0, 0.0)
    s.step(steps)
    _, u, v = s.macros()
    ratio = s.dt / s.tau
    s.close()
    exact = u0 * math.exp(-nu * k * k * steps * g["dt"])
    return float(np.sqrt(((u - exact) ** 2).sum() / (exact ** 2).sum())), steps, ratio


def _stays_bounded(sdugks, mesh, bcs, state, uref, ratio, cfl, dt1, scheme, steps=20000, extra=None):
    """True if the run keeps finite macros with speed <= 3 uref and density in
    [0.5, 2] over the given number of steps (checked every 2000)."""
    import numpy as np
    s = sdugks.Solver(mesh, bcs, tau=cfl * dt1 / ratio, cfl=cfl, scheme=scheme, **(extra or {}))
    if state is not None:
        s.set_macros(*state)
    ok, n = True, 0
    while ok and n < steps:
        s.step(2000)
        n += 2000
        rho, u, v = s.macros()
        sp = np.sqrt(u * u + v * v)
        ok = bool(np.isfinite(rho).all() and np.isfinite(sp).all() and sp.max() <= 3 * uref
                  and rho.min() >= 0.5 and rho.max() <= 2.0)
    s.close()
    return ok


def original_scheme_form(sdugks, meshgen, sched, steps=3000):
    """The original half-step DUGKS against the paper's simplified scheme,
    both in the same fused kernel: cost per step on the headline cavity (same
    tile schedule), accuracy on the decaying shear wave at two Dt/tau, and the
    largest CFL that stays bounded for 20,000 steps as a function of Dt/tau,
    on a cavity with walls and on periodic triangles."""
    import numpy as np
    import torch
    cost = {}
    mesh, bcs = meshgen.cavity(256, beta=1.5, U=0.1)
    for prec, pname in ((sdugks.FP64, "f64"), (sdugks.FP32DEV, "fp32dev")):
        for scheme, sname in ((sdugks.SCHEME_SIMPLIFIED, "simplified"), (sdugks.SCHEME_ORIGINAL, "original")):
            s = sdugks.Solver(mesh, bcs, nu=1e-4, cfl=0.5, precision=prec, scheme=scheme, **sched)
            s.step(300)
            torch.cuda.synchronize()
            ms = time_steps(s.step, steps)
            cost[f"{sname}_{pname}_mlups"] = round(s.n_cells * steps / (ms / 1e3) / 1e6, 1)
            s.close()
    accuracy = []
    for nu in (1e-2, 1e-3, 1e-4):
        for n in (32, 64, 128):
            row = {"n": n, "nu": nu}
            for scheme, sname in ((sdugks.SCHEME_SIMPLIFIED, "simplified"), (sdugks.SCHEME_ORIGINAL, "original")):
                err, nst, ratio = _shear_wave_error(sdugks, meshgen, n, nu, scheme)
                row[f"{sname}_err"] = float(f"{err:.4g}")
            row.update(steps=nst, dt_over_tau=round(ratio, 4))
            accuracy.append(row)
    ratios = (0.01, 0.03, 0.1, 0.3, 1.0, 10.0, 100.0)

    def tri_state():
        m, b = meshgen.jittered_periodic_triangles(32, seed=1)
        g = sdugks.geometry(m, b, nu=0.01)
        u = 0.05 * np.sin(2 * math.pi * g["cy"])
        return m, b, (1.0, u, 0.0), 0.05

    cases = {"cavity 64x64 tanh(1.5), walls, from rest": meshgen.cavity(64) + (None, 0.1),
             "periodic jittered triangles 32x32x2, shear wave": tri_state()}
    stability = []
    for cname, (m, b, state, uref) in cases.items():
        dt1 = sdugks.geometry(m, b, nu=0.01, cfl=1.0)["dt"]
        for scheme, sname in ((sdugks.SCHEME_SIMPLIFIED, "simplified"), (sdugks.SCHEME_ORIGINAL, "original")):
            row = {"case": cname, "scheme": sname, "max_cfl": []}
            for ratio in ratios:
                ok = lambda c: _stays_bounded(sdugks, m, b, state, uref, ratio, c, dt1, scheme)
                lo, hi = 0.25, 2.5
                if not ok(lo):
                    row["max_cfl"].append(f"<{lo}")
                    continue
                if ok(hi):
                    row["max_cfl"].append(f">={hi}")
                    continue
                for _ in range(5):
                    mid = 0.5 * (lo + hi)
                    lo, hi = (mid, hi) if ok(mid) else (lo, mid)
                row["max_cfl"].append(round(lo, 3))
            progress(f"stability {cname} {sname}: {row['max_cfl']}")
            stability.append(row)
    return {"cost": {"workload": "lid-driven cavity 256x256 tanh(1.5), Re 1000, CFL 0.5, headline tile schedule",
                     "steps": steps, **cost},
            "shear_wave_accuracy": {"workload": "periodic n x n quads, u = 0.01 sin(2 pi y), CFL 0.5, "
                                                "run until the amplitude has decayed by e^-0.5",
                                    "rows": accuracy},
            "stability": {"criterion": "finite, speed <= 3 u_ref, density in [0.5, 2] over 20000 steps; "
                                       "largest CFL by bisection in [0.25, 2.5]",
                          "dt_over_tau": list(ratios), "rows": stability}}


def cylinder200k_form(sdugks, autotune, meshgen, steps=2000, warmup=50, schedule=""):
    """Throughput on the 200,000-triangle cylinder O-grid (Re 40, far-field
    inflow 0.1) in FP32 deviation storage and in FP64, each on its autotuned
    schedule (or both on the given "T,B"), and the FP32 form's velocity
    deviation from FP64 after the same steps from rest."""
    import numpy as np
    import torch
    mesh, bcs = meshgen.cylinder_ogrid(400, 250, seed=0)
    out = {"workload": "circular cylinder, O-grid 400x250 split into 200,000 jittered triangles, r 0.5..20, "
                       f"Re 40, u_inf 0.1, CFL 0.5, {steps} steps after {warmup} from rest"}
    uv = {}
    for prec, pname in ((sdugks.FP32DEV, "fp32dev"), (sdugks.FP64, "f64")):
        kw = dict(nu=0.1 / 40, cfl=0.5, u0=0.1, precision=prec)
        if schedule:
            t, b = (int(x) for x in schedule.split(","))
            sched = {"tile_cells": t, "block_threads": b, "structured": 1}
        else:
            sched, _ = autotune.autotune(mesh, bcs, steps=100, **kw)
        s = sdugks.Solver(mesh, bcs, **sched, **kw)
        s.step(warmup)
        torch.cuda.synchronize()
        ms = time_steps(s.step, steps, s.stream) / steps
        nc = s.n_cells
        _, u, v = s.macros()
        uv[pname] = np.concatenate([u, v])
        s.close()
        alg = ALG_BYTES_TRI[pname] * nc / (ms / 1e3) / 1e9
        out[pname] = {"mlups": round(nc / (ms / 1e3) / 1e6, 1), "ms_per_step": round(ms, 5), "schedule": sched,
                      "alg_bytes_per_cell": ALG_BYTES_TRI[pname], "achieved_GBs": round(alg, 1),
                      "frac_of_hbm_peak": round(alg / HBM_PEAK_GBS, 4),
                      "traffic_bytes_per_launch": measured_traffic(f"cylinder200k_{pname}", sched)}
    d = uv["fp32dev"] - uv["f64"]
    out["fp32dev_velocity_rel_l2_vs_f64"] = float(np.linalg.norm(d) / np.linalg.norm(uv["f64"]))
    progress(f"cylinder 200k: fp32dev {out['fp32dev']['mlups']} / f64 {out['f64']['mlups']} MLUPS")
    return out


def large_form(sdugks, meshgen, n=2048, steps=100, warmup=20):
    """Lid-driven cavity on n x n tanh quads (n = 2048: 4.2M cells, device
    state above 2 GB, far beyond the 256 MB Infinity Cache), Re 1000, FP64 and
    FP32 deviation, on the general step's 64-cell tiles and on the structured
    step: MLUPS and the step's share of the HBM peak, from the algorithmic
    bytes and, while the committed counters match the kernel, from the
    measured HBM traffic.  The structured step reads no geometry tables, so
    its own compulsory bytes (the state, read and written once) are given too."""
    import torch
    mesh, bcs = meshgen.cavity(n, beta=1.5, U=0.1)
    out = {"workload": f"lid-driven cavity {n}x{n} tanh(1.5) quads, Re 1000, CFL 0.5, general step on tiles of "
                       f"64 cells and structured step, {steps} steps after {warmup}"}
    general = {"tile_cells": 64, "block_threads": 256, "structured": 1}
    forms = [(sdugks.FP64, "f64", general), (sdugks.FP32DEV, "fp32dev", general),
             (sdugks.FP64, "structured_f64", {"structured": 2}),
             (sdugks.FP32DEV, "structured_fp32dev", {"structured": 2})]
    for prec, name, sched in forms:
        pname = "f64" if prec == sdugks.FP64 else "fp32dev"
        kw = dict(nu=1e-4, cfl=0.5, precision=prec, **sched)
        s = sdugks.Solver(mesh, bcs, **kw)
        s.step(warmup)
        torch.cuda.synchronize()
        ms = time_steps(s.step, steps) / steps
        nc = s.n_cells
        s.close()
        alg = ALG_BYTES[pname] * nc / (ms / 1e3) / 1e9
        e = {"mlups": round(nc / (ms / 1e3) / 1e6, 1), "ms_per_step": round(ms, 5), "schedule": sched,
             "working_set_GB": round(sdugks.state_bytes(mesh, bcs, **kw) / 1e9, 2),
             "achieved_GBs": round(alg, 1), "frac_of_hbm_peak": round(alg / HBM_PEAK_GBS, 4)}
        if sched.get("structured") == 2:
            own = 2 * ((72 if prec == sdugks.FP64 else 36) + 24)
            e["kernel_own_bytes_per_cell"] = own
            e["frac_of_own_bytes"] = round(own * nc / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
        t = measured_traffic(f"cavity{n}_{name}", sched)
        if t is not None:
            e["traffic_bytes_per_launch"] = t
            e["measured_GBs"] = round(t / (ms / 1e3) / 1e9, 1)
            e["measured_frac_of_hbm_peak"] = round(t / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
        out[name] = e
        progress(f"large cavity {name}: {e['mlups']} MLUPS, {e['frac_of_hbm_peak']} of HBM peak (algorithmic)")
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(meshgen, target_s=15.0):
    """The FP64 oracle on the host: the headline workload (the 64 cavities,
    200 steps per instance) on all the threads the process may use, the same
    instances for a few steps on one thread, and the windows of the other
    configurations (Couette 4 x 32 for its full 5000 steps, the 256 x 256
    cavity and the 200,000-triangle cylinder for 1000 steps on all threads, a
    shorter window on one thread).  MLUPS = cells x steps / seconds of
    stepping (set-up excluded).  Threaded and single-thread runs give
    identical results (the oracle's loops are per cell and per face)."""
    import oracle
    from paper_2007_07347_amd import sdugks
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    used = oracle.set_threads(threads)

    def run(mesh, bcs, kw, steps):
        o = oracle.Oracle(mesh, bcs, **{k: v for k, v in kw.items() if k in ("nu", "cfl", "u0")})
        t = time.perf_counter()
        o.step(steps)
        el = time.perf_counter() - t
        return o.n_cells * steps, el

    def batch(steps):
        upd = el = 0.0
        for mesh, bcs, kw in batch_problems(sdugks, meshgen):
            u, e = run(mesh, bcs, kw, steps)
            upd += u
            el += e
        return upd, el

    mlups = lambda ue: round(ue[0] / ue[1] / 1e6, 3)  # noqa: E731
    head = batch(200)
    progress(f"cpu baseline: 64 cavities x 200 steps on {used} threads, {mlups(head)} MLUPS")
    cav = (*meshgen.cavity(256), dict(nu=1e-4, cfl=0.5))
    cyl = (*meshgen.cylinder_ogrid(400, 250, seed=0), dict(nu=0.1 / 40, cfl=0.5, u0=0.1))
    cou = (*meshgen.couette(4, 32, 0.1), dict(nu=0.01, cfl=0.5))
    windows = {"couette_4x32_5000_steps": mlups(run(*cou, 5000)),
               "cavity256_1000_steps": mlups(run(*cav, 1000)),
               "cylinder200k_1000_steps": mlups(run(*cyl, 1000))}
    oracle.set_threads(1)
    single = {"cavities64_5_steps_each": mlups(batch(5)), "cavity256_100_steps": mlups(run(*cav, 100)),
              "cylinder200k_30_steps": mlups(run(*cyl, 30))}
    return {"value": mlups(head), "unit": "MLUPS", "cores": used, "kind": "oracle",
            "sample": "the headline's 64 cavities (2,289,523 cells), 200 steps per instance from rest, FP64 oracle "
                      f"(gcc -O2, OpenMP over cells and faces) on {used} threads",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(), "threads": used,
            "windows_all_threads": windows, "single_thread": single}


def cavity256_form(sdugks, autotune, meshgen, a):
    """The single 256 x 256 cavity (Re 1000) in both storage forms: MLUPS and
    the step kernel's effective bandwidth (its 35 MB working set stays in the
    256 MB Infinity Cache, so this is not an HBM figure)."""
    out = {"workload": "lid-driven cavity 256x256 tanh(1.5) quads, Re 1000, CFL 0.5, D2Q9, residual every 1000 "
                       "steps; working set in the Infinity Cache, so bandwidths are effective, not HBM"}
    steps = max(a.steps, 2000)
    b = argparse.Namespace(**vars(a))
    b.steps = steps
    for prec, pname in ((sdugks.FP64, "f64"), (sdugks.FP32DEV, "fp32dev"), (sdugks.FP32NEQ, "fp32neq")):
        s, mesh, bcs, kw, sched, nc, ms, wall, eps, kt = headline(sdugks, autotune, meshgen, b, prec)
        k_ms = ms / steps
        ab = ALG_BYTES["fp32dev" if pname == "fp32neq" else pname]
        out[pname] = {"mlups": round(nc * steps / (ms / 1e3) / 1e6, 1), "ms_per_step": round(k_ms, 5),
                      "steps": steps, "schedule": sched, "alg_bytes_per_cell": ab,
                      "effective_GBs": round(ab * nc / (k_ms / 1e3) / 1e9, 1),
                      "kernel_ms_event_per_launch": round(max(kt.values()), 5),
                      "traffic_bytes_per_launch": measured_traffic(
                          f"cavity256_{pname}" + ("_structured" if sched.get("structured") == 2 else ""), sched),
                      "working_set_MB": round(sdugks.state_bytes(mesh, bcs, **kw, **sched) / 1e6, 1)}
        s.close()
        progress(f"cavity 256 {pname}: {out[pname]['mlups']} MLUPS")
    return out


def main():
    a = parse()
    unknown = {x for x in a.sections.split(",") if x} - set(SECTIONS)
    if unknown:
        print(f"unknown sections: {sorted(unknown)}; choose from {','.join(SECTIONS)}", file=sys.stderr)
        sys.exit(2)
    for opt, v in (("--schedule", a.schedule), ("--batch-schedule", a.batch_schedule),
                   ("--cylinder-schedule", a.cylinder_schedule)):
        if opt != "--cylinder-schedule" and v == "structured":
            continue
        if v and not (len(v.split(",")) == 2 and all(x.isdigit() for x in v.split(","))):
            print(f"{opt} takes two integers T,B (got {v!r})", file=sys.stderr)
            sys.exit(2)
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the multi-GPU design is described, not built.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if a.copy_calibration:
        copy_calibration(a.copy_calibration)
        return
    import meshgen
    from paper_2007_07347_amd import autotune, sdugks
    if a.large_only:
        print(json.dumps({"large": large_form(sdugks, meshgen)}), flush=True)
        return

    t_start = time.perf_counter()
    hb = batch_headline(sdugks, autotune, meshgen, a)
    cells, ms = hb["cells"], hb["ms"]
    mlups = cells * a.steps / (ms / 1e3) / 1e6
    progress(f"headline (64-cavity batch) {mlups:.1f} MLUPS")
    k_ms = ms / a.steps
    achieved = ALG_BYTES["fp32dev"] * cells / (k_ms / 1e3) / 1e9
    eps = hb["eps"]
    structured = hb["sched"].get("structured") == 2
    # the structured step reads no geometry tables: its own compulsory bytes are
    # the state alone, f and W read and written once (FP32 f: 2 x (36 + 24))
    own = 2 * (36 + 24)
    roof = {"bound": "hbm", "kernel": "k_step_batch_cart" if structured else "k_step_batch",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic("batch64_fp32dev" + ("" if structured else "_general"), hb["sched"]),
            "alg_bytes_per_cell": ALG_BYTES["fp32dev"], "cells_per_launch": cells, "kernel_ms": round(k_ms, 5),
            "working_set_MB": hb["working_set_MB"],
            "note": "working set above the 256 MB Infinity Cache; achieved = algorithmic bytes per cell (304 B: "
                    "the FP32 state read and written once plus the stored geometry of a general quad mesh) x cells "
                    "per launch / average launch duration (HIP events on the batch stream)"}
    if structured:
        roof["kernel_own_bytes_per_cell"] = own
        roof["frac_of_own_bytes"] = round(own * cells / (k_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    out = {
        "metric": "MLUPS (D2Q9 cell-updates/s) & %HBM peak; p50/p99 time-to-steady under load",
        "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms / a.steps, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": BATCH_WORKLOAD, "instances": 64, "cells": cells, "schedule": hb["sched"],
                   # untimed steps actually run before the timed ones: at least 35, so that
                   # every captured graph the timed steps use has been replayed once
                   "warmup_steps_run": hb["warm"],
                   "residual_at_end": None if eps is None else {"min": float(f"{min(eps):.3g}"),
                                                                "max": float(f"{max(eps):.3g}")}},
        "roofline": roof,
        "wall_s": round(hb["wall"], 3),
        "per_instance_loop": {"steps": hb["loop_steps"],
                              "mlups": round(cells * hb["loop_steps"] / (hb["loop_ms"] / 1e3) / 1e6, 1),
                              "ms_per_step": round(hb["loop_ms"] / hb["loop_steps"], 4)},
        "batch_autotune_ms_per_step": {autotune.label(r): (None if r["ms"] is None else round(r["ms"], 4))
                                       for r in hb["table"]},
    }
    sections = set() if a.no_extra else {x for x in a.sections.split(",") if x}
    section_s = {"headline": round(time.perf_counter() - t_start, 1)}

    def run(name, key, fn):
        # each section's wall time (set-up, autotuning and its own timed runs)
        t0 = time.perf_counter()
        out[key] = fn()
        section_s[name] = round(time.perf_counter() - t0, 1)
        progress(f"{name} done in {section_s[name]} s")
    if "cavity256" in sections:
        run("cavity256", "cavity256", lambda: cavity256_form(sdugks, autotune, meshgen, a))
    if "converge" in sections:
        run("converge", "converge", lambda: converge_form(sdugks, meshgen, names=CONVERGE_CASES[:1]))
    if "converge_cylinder" in sections:
        run("converge_cylinder", "converge_cylinder", lambda: converge_form(sdugks, meshgen, names=CONVERGE_CASES[1:]))
    if "serving" in sections:
        run("serving", "serving", lambda: serving(meshgen))
    if "serving_narrow" in sections:
        run("serving_narrow", "serving_narrow",
            lambda: serving(meshgen, step_cap=300_000, trace_kw=SERVING_TRACE_NARROW))
    if "cylinder" in sections:
        run("cylinder", "cylinder", lambda: cylinder_form(meshgen))
    if "original" in sections:
        run("original", "original_scheme", lambda: original_scheme_form(sdugks, meshgen, out.get("cavity256", {}).get(
            "f64", {}).get("schedule", {"tile_cells": 32, "block_threads": 128})))
    if "cylinder200k" in sections:
        run("cylinder200k", "cylinder200k",
            lambda: cylinder200k_form(sdugks, autotune, meshgen, schedule=a.cylinder_schedule))
    if "large" in sections:
        run("large", "large", lambda: large_form(sdugks, meshgen))
    if not a.no_cpu:
        run("cpu_baseline", "cpu_baseline", lambda: cpu_baseline(meshgen, a.cpu_seconds))
    out["section_wall_s"] = section_s
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

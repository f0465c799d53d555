"""Autotuner of the fused step's schedule: on tensor-product quad meshes the
structured step (fixed tiles, one lane per face) against the
general fused step; for the general step, the tile size (cells per
workgroup, which sets the halo overhead and the LDS per workgroup, hence how
many workgroups share a compute unit) and threads per workgroup (which sets
how many lanes serve each cell in every phase: four per cell, one per face
of a quad, in the face pass).

Each candidate is built with the library, warmed up, and timed with HIP
events over a fixed number of steps on the instance's own stream; the
fastest is returned and cached on disk per mesh signature, so a serving loop
or a batch tunes once per mesh class.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from . import sdugks

# (tile cells, threads) of the general step: a tile holds at most a quarter as
# many cells as threads
CANDIDATES = [(16, 64), (16, 128), (32, 128), (16, 256), (32, 256), (64, 256)]
STRUCTURED = {"structured": 2}


def label(sched):
    """Name of a schedule in timing tables: the lanes-per-face axis (one lane
    per face on the structured step, four lanes per cell, one per face slot,
    on the general step) and the general step's tile cells / threads."""
    if sched.get("structured") == 2:
        return "structured, 1 lane per face"
    return f"general {sched['tile_cells']}/{sched['block_threads']}, 4 lanes per cell"


def candidates_for(problems, candidates=None):
    """Schedules to try: the structured step when every mesh is a tensor
    product (it takes no tile parameters), then the general step's."""
    out = []
    if candidates is None:
        if all(sdugks.tiling(m, b, **{k: v for k, v in kw.items() if k != "precision"})["structured"]
               for m, b, kw in problems):
            out.append(dict(STRUCTURED))
        candidates = CANDIDATES
    out += [{"tile_cells": t, "block_threads": b, "structured": 1} for t, b in candidates]
    return out
CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")


def signature(mesh, precision):
    """Mesh class key: cell count, polygon degrees and a hash of the connectivity."""
    h = hashlib.sha1()
    h.update(np.ascontiguousarray(mesh["cell_ptr"]).tobytes())
    h.update(np.ascontiguousarray(mesh["cell_nodes"]).tobytes())
    return f"{len(mesh['cell_ptr']) - 1}-{precision}-{h.hexdigest()[:12]}"


def _load_cache(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store_cache(path, db):
    """Best effort: a read-only location only costs the re-tuning."""
    try:
        with open(path + ".tmp", "w") as fh:
            json.dump(db, fh, indent=1)
        os.replace(path + ".tmp", path)
    except OSError:
        pass


def time_candidate(mesh, bcs, sched, steps=200, warmup=20, **kw):
    import torch
    s = sdugks.Solver(mesh, bcs, **sched, **kw)
    s.step(warmup)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s.stream)
    s.step(steps)
    b.record(s.stream)
    b.synchronize()
    ms = a.elapsed_time(b) / steps
    s.close()
    return ms


def autotune(mesh, bcs, candidates=None, steps=200, cache=CACHE, refresh=False, **kw):
    """Return ({"tile_cells", "block_threads"}, table) for the fastest fused
    schedule of this mesh; table lists ms per step of every candidate."""
    key = signature(mesh, kw.get("precision", sdugks.FP64))
    db = _load_cache(cache) if cache else {}
    if not refresh and key in db:
        return db[key]["best"], db[key]["table"]
    table = []
    for sched in candidates_for([(mesh, bcs, kw)], candidates):
        try:
            ms = time_candidate(mesh, bcs, sched, steps=steps, **kw)
        except sdugks.SdugksError as e:        # e.g. a tile too small for the mesh degree
            table.append({**sched, "ms": None, "error": str(e)})
            continue
        table.append({**sched, "ms": ms})
    ok = [r for r in table if r["ms"] is not None]
    if not ok:
        raise RuntimeError("no candidate schedule fits: " + "; ".join(r["error"] for r in table))
    best = min(ok, key=lambda r: r["ms"])
    best = {k: v for k, v in best.items() if k not in ("ms", "error")}
    if cache:
        db[key] = {"best": best, "table": table}
        _store_cache(cache, db)
    return best, table


def batch_signature(problems):
    """Key of a set of batch members: each member's mesh class and parameters."""
    h = hashlib.sha1()
    for mesh, bcs, kw in problems:
        h.update(signature(mesh, kw.get("precision", sdugks.FP64)).encode())
        h.update(json.dumps(sorted((k, v) for k, v in kw.items() if k != "precision")).encode())
    return f"batch-{len(problems)}-{h.hexdigest()[:12]}"


def time_batch_candidate(problems, sched, steps=50, warmup=10):
    """ms per batched step of all problems, every member on this schedule."""
    import torch
    solvers = []
    try:
        for mesh, bcs, kw in problems:
            solvers.append(sdugks.Solver(mesh, bcs, **sched, **kw))
        b = sdugks.Batch(solvers)
        try:
            b.step(warmup)
            torch.cuda.synchronize()
            a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            b.step(steps)
            e.record()
            torch.cuda.synchronize()
            return a.elapsed_time(e) / steps
        finally:
            b.close()
    finally:
        for s in solvers:
            s.close()


def autotune_batch(problems, candidates=None, steps=50, cache=CACHE, refresh=False):
    """Schedule for a batch: problems is a list of (mesh, bcs, solver keyword
    arguments without the schedule); each candidate schedule is applied to
    every member and the batched step timed as a whole (one launch covers all
    members, so its schedule is one choice).  Returns ({"tile_cells",
    "block_threads"}, table), cached like autotune()."""
    key = batch_signature(problems)
    db = _load_cache(cache) if cache else {}
    if not refresh and key in db:
        return db[key]["best"], db[key]["table"]
    table = []
    for sched in candidates_for(problems, candidates):
        try:
            ms = time_batch_candidate(problems, sched, steps=steps)
        except sdugks.SdugksError as e:
            table.append({**sched, "ms": None, "error": str(e)})
            continue
        table.append({**sched, "ms": ms})
    ok = [r for r in table if r["ms"] is not None]
    if not ok:
        raise RuntimeError("no candidate schedule fits: " + "; ".join(r["error"] for r in table))
    best = min(ok, key=lambda r: r["ms"])
    best = {k: v for k, v in best.items() if k not in ("ms", "error")}
    if cache:
        db[key] = {"best": best, "table": table}
        _store_cache(cache, db)
    return best, table

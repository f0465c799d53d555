"""Serving loop: continuous batching of steady-state sDUGKS solves.

Requests (a mesh, its boundary table, the flow parameters) arrive over time.
The scheduler keeps a FIFO queue, admits the head of the queue as soon as a
slot is free and the request's device bytes fit the remaining HBM budget,
advances every admitted instance together (one batched launch per step,
replayed from a captured graph) in chunks of `interval` steps, then polls
each instance's velocity residual (the convergence test of the paper's
cavity case, checked every 1000 steps there) and retires instances that
converged, diverged (non-finite state) or hit their step cap.  Retirement
frees the slot and the memory, and the next queued request is admitted
before the next chunk: requests that arrive while others run join the
running batch.

Admission overlaps the GPU: when the backend offers create_async(), the
admitted request's instance (mesh build on the host, upload on a stream of
its own) is made on a worker thread while the batch keeps stepping, and joins
the batch at the first chunk boundary after it is ready.  When the batch
offers residuals(), every member's residual comes from one batched reduction
and one synchronisation per chunk.

An instance whose residual has stopped falling while still above the
tolerance (no 20 % gain over `stall_checks` checks) is handed to the
backend's optional escalate(): the GPU backend continues it from its current
state with the same FP32 storage and FP64 arithmetic (FP32NEQ), which has
no such floor (the floor comes from the FP32 arithmetic), when the new
instance fits the remaining budget.

A request whose instance cannot be sized or made (the library rejects its
mesh or parameters, or the memory runs out) is retired as "failed" with the
error's text, and any bytes it held return to the budget; the others are
served as before.
A failed escalation leaves the request in its first form.

Time-to-steady of a request = completion time - arrival time (queueing
included).  The backend interface keeps the policy testable without a GPU:

    backend.bytes(req) -> int                 device bytes the instance needs
    backend.create(req) -> instance           instance.step(n), .residual(),
                                              .macros(), .close(), .n_cells
    backend.create_async(req) -> future       optional: .done(), .result() -> instance
    backend.batch(instances) -> batch         batch.step(n), .set_members(list),
                                              .close(); optional .residuals() ->
                                              one residual per member, raising
                                              an error with .code == -4 and
                                              .residuals (NaN where not finite)
    backend.escalate(req, inst, room)         optional: (instance, bytes) that
        -> (instance, int) or None            continues inst, or None
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Any, Callable, List, Optional


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                  # seconds after the start of the trace
    mesh: Any
    bcs: Any
    params: dict
    kind: str = ""
    n_cells: int = 0


@dataclasses.dataclass
class Result:
    rid: int
    kind: str
    n_cells: int
    status: str                     # "converged", "not_converged", "diverged", "rejected", "failed"
    arrival: float
    admitted: float
    finished: float
    steps: int
    residual: float
    macros: Optional[tuple] = None
    error: str = ""                 # "failed": why the instance could not be made

    @property
    def time_to_steady(self):
        return self.finished - self.arrival


class Server:
    """Continuous-batching scheduler over a backend (see module docstring).

    budget_bytes: device memory the admitted instances may hold together.
    max_slots:    admitted instances at most.
    interval:     steps between residual checks (the paper checks every 1000).
    tol:          residual that counts as steady.
    step_cap:     steps after which an instance is retired as not converged.
    keep_macros:  copy (rho, u, v) out of each retired instance.
    stall_checks: checks without a 20 % fall of the residual after which a
                  request above the tolerance is escalated (0: never).
    """

    def __init__(self, backend, budget_bytes, max_slots=64, interval=1000, tol=1e-7, step_cap=200_000,
                 keep_macros=False, stall_checks=8, clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.interval = int(interval)
        self.tol = float(tol)
        self.step_cap = int(step_cap)
        self.keep_macros = keep_macros
        self.stall_checks = int(stall_checks)
        self.clock = clock
        self.sleep = sleep
        self.log: List[tuple] = []          # (time, event, rid, extra)

    def run(self, requests: List[Request]):
        """Serve a finite trace; returns (results in request order, stats)."""
        pending = sorted(requests, key=lambda r: r.arrival)
        queue: List[Request] = []
        staging = []                        # [req, future, bytes, admitted_at]: instances being made
        active = []                         # [req, instance, bytes, admitted_at, steps, best, stalled, escalated]
        results = {}
        used = 0
        batch = None
        members_changed = False
        cell_updates = 0
        make_async = getattr(self.backend, "create_async", None)
        t0 = self.clock()
        now = lambda: self.clock() - t0     # noqa: E731
        while pending or queue or active or staging:
            t = now()
            while pending and pending[0].arrival <= t:
                queue.append(pending.pop(0))
            # admission, FIFO: the head waits until it fits (no overtaking)
            while queue and len(active) + len(staging) < self.max_slots:
                req = queue[0]
                try:
                    need = self.backend.bytes(req)
                except Exception as e:          # the library refuses its mesh or parameters
                    queue.pop(0)
                    self._fail(results, req, now(), e)
                    continue
                if need > self.budget:
                    queue.pop(0)
                    results[req.rid] = Result(req.rid, req.kind, req.n_cells, "rejected", req.arrival, now(),
                                              now(), 0, math.inf)
                    self.log.append((now(), "reject", req.rid, need))
                    continue
                if used + need > self.budget:
                    break
                queue.pop(0)
                used += need
                self.log.append((now(), "admit", req.rid, need))
                if make_async is not None:
                    staging.append([req, make_async(req), need, now()])
                    continue
                try:
                    inst = self.backend.create(req)
                except Exception as e:          # this request only: its bytes return to the budget
                    used -= need
                    self._fail(results, req, now(), e)
                    continue
                active.append([req, inst, need, now(), 0, math.inf, 0, False])
                members_changed = True
            # instances made on the worker join at this chunk boundary; with
            # nothing running, wait for the first one instead of spinning
            if staging and not active:
                try:
                    staging[0][1].result()
                except Exception:               # handled with the others below
                    pass
            still = []
            for st in staging:
                if not st[1].done():
                    still.append(st)
                    continue
                try:
                    inst = st[1].result()
                except Exception as e:
                    used -= st[2]
                    self._fail(results, st[0], now(), e)
                    continue
                active.append([st[0], inst, st[2], st[3], 0, math.inf, 0, False])
                members_changed = True
            staging = still
            if not active:
                if pending:
                    self.sleep(max(0.0, min(pending[0].arrival - now(), 0.05)))
                continue
            if batch is None:
                batch = self.backend.batch([a[1] for a in active])
            elif members_changed:
                batch.set_members([a[1] for a in active])
            members_changed = False
            batch.step(self.interval)
            for a in active:
                a[4] += self.interval
                cell_updates += a[1].n_cells * self.interval
            # every residual, from one batched reduction when the batch has it
            eps_all = None
            if hasattr(batch, "residuals"):
                try:
                    eps_all = list(batch.residuals())
                except Exception as e:          # some member not finite: NaN marks it
                    if getattr(e, "code", None) != -4:
                        raise
                    eps_all = list(e.residuals)
            # poll every instance, then change the membership once, then free
            keep, retired = [], []
            can_escalate = self.stall_checks > 0 and hasattr(self.backend, "escalate")
            for k, a in enumerate(active):
                req, inst, need, t_adm, steps = a[:5]
                status = None
                if eps_all is not None:
                    eps = eps_all[k]
                    if math.isnan(eps):
                        status = "diverged"
                else:
                    try:
                        eps = inst.residual()
                    except Exception as e:      # non-finite state: only this request fails
                        if getattr(e, "code", None) != -4:
                            raise
                        eps, status = math.nan, "diverged"
                if status is None:
                    if eps <= self.tol:
                        status = "converged"
                    elif steps >= self.step_cap:
                        status = "not_converged"
                if status is None:
                    if eps < 0.8 * a[5]:
                        a[5], a[6] = eps, 0
                    else:
                        a[6] += 1
                    if can_escalate and not a[7] and a[6] >= self.stall_checks:
                        try:
                            got = self.backend.escalate(req, inst, self.budget - used + need)
                        except Exception as e:  # keep serving it in its first form
                            got = None
                            a[7] = True
                            self.log.append((now(), "escalate_failed", req.rid, str(e)))
                        if got is not None:
                            new, new_need = got
                            used += new_need - need
                            a[1], a[2], a[5], a[6], a[7] = new, new_need, math.inf, 0, True
                            retired.append(inst)
                            self.log.append((now(), "escalate", req.rid, steps))
                    keep.append(a)
                    continue
                macros = inst.macros() if (self.keep_macros and status != "diverged") else None
                results[req.rid] = Result(req.rid, req.kind, req.n_cells, status, req.arrival, t_adm, now(), steps,
                                          eps, macros)
                self.log.append((now(), status, req.rid, steps))
                used -= need
                retired.append(inst)
            if retired:
                # the batch drops the members before they are destroyed
                if keep:
                    batch.set_members([a[1] for a in keep])
                else:
                    batch.close()
                    batch = None
                for inst in retired:
                    inst.close()
            active = keep
        elapsed = now()
        out = [results[r.rid] for r in sorted(requests, key=lambda r: r.rid)]
        return out, summarize(out, elapsed, cell_updates)

    def _fail(self, results, req, t, e):
        results[req.rid] = Result(req.rid, req.kind, req.n_cells, "failed", req.arrival, t, t, 0, math.inf,
                                  error=str(e))
        self.log.append((t, "failed", req.rid, str(e)))


def summarize(results, elapsed, cell_updates):
    done = [r for r in results if r.status == "converged"]
    tts = sorted(r.time_to_steady for r in done)

    def pct(p):
        if not tts:
            return None
        k = min(len(tts) - 1, max(0, int(math.ceil(p / 100.0 * len(tts))) - 1))
        return tts[k]
    return {"requests": len(results), "converged": len(done),
            "not_converged": sum(r.status == "not_converged" for r in results),
            "diverged": sum(r.status == "diverged" for r in results),
            "rejected": sum(r.status == "rejected" for r in results),
            "failed": sum(r.status == "failed" for r in results),
            "p50_time_to_steady_s": pct(50), "p99_time_to_steady_s": pct(99),
            "makespan_s": elapsed, "cell_updates": cell_updates,
            "aggregate_mlups": cell_updates / elapsed / 1e6 if elapsed > 0 else None}


class SequentialServer(Server):
    """The plain per-case loop: one request at a time, in arrival order, no
    batching (the baseline the continuous batch is compared with)."""

    def run(self, requests: List[Request]):
        pending = sorted(requests, key=lambda r: r.arrival)
        results = {}
        cell_updates = 0
        t0 = self.clock()
        now = lambda: self.clock() - t0     # noqa: E731
        for req in pending:
            if req.arrival > now():
                self.sleep(req.arrival - now())
            try:
                need = self.backend.bytes(req)
            except Exception as e:
                self._fail(results, req, now(), e)
                continue
            if need > self.budget:
                results[req.rid] = Result(req.rid, req.kind, req.n_cells, "rejected", req.arrival, now(), now(), 0,
                                          math.inf)
                continue
            t_adm = now()
            try:
                inst = self.backend.create(req)
            except Exception as e:
                self._fail(results, req, now(), e)
                continue
            steps, status, eps = 0, None, math.inf
            while status is None:
                inst.step(self.interval)
                steps += self.interval
                cell_updates += inst.n_cells * self.interval
                try:
                    eps = inst.residual()
                except Exception as e:
                    if getattr(e, "code", None) == -4:
                        status, eps = "diverged", math.nan
                        break
                    raise
                if eps <= self.tol:
                    status = "converged"
                elif steps >= self.step_cap:
                    status = "not_converged"
            macros = inst.macros() if (self.keep_macros and status != "diverged") else None
            results[req.rid] = Result(req.rid, req.kind, req.n_cells, status, req.arrival, t_adm, now(), steps, eps,
                                      macros)
            inst.close()
        elapsed = now()
        out = [results[r.rid] for r in sorted(requests, key=lambda r: r.rid)]
        return out, summarize(out, elapsed, cell_updates)


class GpuBackend:
    """Backend on libsdugks: one solver per request (its device memory a torch
    tensor of sdugks_state_bytes), one batch for all admitted solvers; a
    stalled FP32DEV solver is continued by an FP32NEQ one (same storage,
    FP64 arithmetic).  create_async()
    builds a solver on a worker thread (the library's mesh build and upload
    release the interpreter lock) on a stream of its own, so that neither its
    host work nor its synchronous uploads wait for the running batch."""

    def __init__(self, precision=None, workers=2, **defaults):
        from . import sdugks
        self.sd = sdugks
        self.precision = sdugks.FP32DEV if precision is None else precision
        self.defaults = defaults
        self.workers = int(workers)
        self._pool = None
        self._bytes = {}

    def _kw(self, req):
        kw = dict(self.defaults)
        kw.update(req.params)
        kw.setdefault("precision", self.precision)
        return kw

    def bytes(self, req):
        # the host mesh build behind this is paid once per request
        key = (id(req), self.precision)
        if key not in self._bytes:
            self._bytes[key] = self.sd.state_bytes(req.mesh, req.bcs, **self._kw(req))
        return self._bytes[key]

    def create(self, req, stream=None):
        return self.sd.Solver(req.mesh, req.bcs, stream=stream, **self._kw(req))

    def _create_on_side_stream(self, req):
        import torch
        return self.create(req, stream=torch.cuda.Stream())

    def create_async(self, req):
        if self._pool is None:
            from concurrent.futures import ThreadPoolExecutor
            self._pool = ThreadPoolExecutor(max_workers=self.workers, thread_name_prefix="sdugks-admit")
        return self._pool.submit(self._create_on_side_stream, req)

    def batch(self, instances):
        return self.sd.Batch(instances)

    def escalate(self, req, inst, room):
        kw = self._kw(req)
        if kw["precision"] != self.sd.FP32DEV:
            return None
        kw["precision"] = self.sd.FP32NEQ
        need = self.sd.state_bytes(req.mesh, req.bcs, **kw)
        if need > room:
            return None
        new = self.sd.Solver(req.mesh, req.bcs, stream=getattr(inst, "stream", None), **kw)
        try:
            new.set_state(*inst.state())
        except Exception:
            new.close()
            raise
        return new, need

    def close(self):
        if self._pool is not None:
            self._pool.shutdown(wait=True)
            self._pool = None

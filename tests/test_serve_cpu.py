"""Serving scheduler on the CPU: admission by HBM budget and slots, FIFO
order, continuous batching, failure isolation, step caps, and results that
are the same alone and in the mix (oracle-backed instances)."""
import math

import numpy as np
import pytest

import meshgen
from paper_2007_07347_amd.serve import Request, SequentialServer, Server, summarize


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-4)


class FakeInst:
    """Converges after `need` steps; residual 1 before, 1e-9 after."""

    def __init__(self, req, clock, log):
        self.req, self.clock, self.log = req, clock, log
        self.n_cells = req.n_cells
        self.steps = 0
        self.closed = False

    def step(self, n):
        assert not self.closed
        self.steps += n

    def residual(self):
        assert not self.closed
        if self.req.params.get("poison"):
            e = RuntimeError("not finite")
            e.code = -4
            raise e
        return 1e-9 if self.steps >= self.req.params["need"] else 1.0

    def macros(self):
        return (self.req.rid, self.steps)

    def close(self):
        self.closed = True


class FakeBatch:
    def __init__(self, members, clock, log):
        self.members, self.clock, self.log = list(members), clock, log

    def set_members(self, members):
        self.members = list(members)

    def step(self, n):
        self.log.append(("batch", tuple(m.req.rid for m in self.members)))
        cells = 0
        for m in self.members:
            m.step(n)
            cells += m.n_cells
        self.clock.t += 1e-6 * n * (1 + cells / 1000.0)   # one launch per step

    def close(self):
        self.members = []


class FakeBackend:
    def __init__(self, clock, cost=None):
        self.clock, self.log, self.cost = clock, [], cost or (lambda r: r.n_cells * 100)
        self.live = {}

    def bytes(self, req):
        return self.cost(req)

    def create(self, req):
        inst = FakeInst(req, self.clock, self.log)
        self.live[req.rid] = inst
        return inst

    def batch(self, instances):
        return FakeBatch(instances, self.clock, self.log)


def reqs(specs):
    return [Request(rid=k, arrival=a, mesh=None, bcs=None, params=p, kind="fake", n_cells=n)
            for k, (a, n, p) in enumerate(specs)]


def run(server_cls, specs, **kw):
    clock = SimClock()
    be = FakeBackend(clock, kw.pop("cost", None))
    srv = server_cls(be, clock=clock, sleep=clock.sleep, **kw)
    res, stats = srv.run(reqs(specs))
    return res, stats, srv, be


def test_budget_and_slots_respected_fifo():
    specs = [(0.0, 100, {"need": 3000}), (0.0, 300, {"need": 1000}), (0.0, 100, {"need": 1000}),
             (0.0, 100, {"need": 2000}), (0.001, 400, {"need": 1000})]
    res, stats, srv, be = run(Server, specs, budget_bytes=50_000, max_slots=3, interval=1000)
    assert stats["converged"] == 5
    used, live, order = 0, 0, []
    sizes = {k: n * 100 for k, (a, n, p) in enumerate(specs)}
    for t, ev, rid, extra in srv.log:
        if ev == "admit":
            used += sizes[rid]
            live += 1
            order.append(rid)
        elif ev == "converged":
            used -= sizes[rid]
            live -= 1
        assert used <= 50_000 and live <= 3
    assert order == sorted(order)          # FIFO: nobody overtakes the head


def test_continuous_batching_joins_running_batch():
    specs = [(0.0, 10, {"need": 10_000}), (0.0005, 10, {"need": 1000})]
    res, stats, srv, be = run(Server, specs, budget_bytes=10**9, interval=1000)
    batches = [m for kind, m in be.log if kind == "batch"]
    assert (0, 1) in batches                 # the later request ran together with the first
    assert res[1].finished < res[0].finished


def test_oversized_request_rejected_others_served():
    specs = [(0.0, 100, {"need": 1000}), (0.0, 10**6, {"need": 1000}), (0.0, 100, {"need": 2000})]
    res, stats, srv, be = run(Server, specs, budget_bytes=10**6)
    assert [r.status for r in res] == ["converged", "rejected", "converged"]


def test_divergence_isolated_and_step_cap():
    specs = [(0.0, 10, {"need": 3000}), (0.0, 10, {"need": 2000, "poison": True}), (0.0, 10, {"need": 10**9})]
    res, stats, srv, be = run(Server, specs, budget_bytes=10**6, step_cap=5000, interval=1000)
    assert [r.status for r in res] == ["converged", "diverged", "not_converged"]
    assert res[0].steps == 3000 and res[2].steps == 5000
    assert all(inst.closed for inst in be.live.values())


def test_percentiles():
    from paper_2007_07347_amd.serve import Result
    rs = [Result(k, "x", 1, "converged", 0.0, 0.0, float(k + 1), 0, 0.0) for k in range(100)]
    s = summarize(rs, 100.0, 10**8)
    assert s["p50_time_to_steady_s"] == 50.0 and s["p99_time_to_steady_s"] == 99.0
    assert s["aggregate_mlups"] == pytest.approx(1.0)


def test_sequential_baseline_serves_in_arrival_order():
    specs = [(0.0, 10, {"need": 2000}), (0.0, 10, {"need": 1000})]
    res, stats, srv, be = run(SequentialServer, specs, budget_bytes=10**6)
    assert res[0].finished <= res[1].admitted


# ---- real physics on the CPU: oracle-backed instances
class OracleInst:
    def __init__(self, req, oracle_mod):
        self.o = oracle_mod.Oracle(req.mesh, req.bcs, **req.params)
        self.n_cells = self.o.n_cells

    def step(self, n):
        self.o.step(n)

    def residual(self):
        return self.o.residual()

    def macros(self):
        return self.o.macros()

    def close(self):
        pass


class OracleBatch:
    def __init__(self, members):
        self.members = list(members)

    def set_members(self, members):
        self.members = list(members)

    def step(self, n):
        for m in self.members:
            m.step(n)

    def close(self):
        self.members = []


class OracleBackend:
    def __init__(self, oracle_mod):
        self.oracle = oracle_mod

    def bytes(self, req):
        return req.n_cells * 400

    def create(self, req):
        return OracleInst(req, self.oracle)

    def batch(self, instances):
        return OracleBatch(instances)


def test_results_same_alone_and_in_the_mix(oracle_mod):
    trace = meshgen.serving_trace(seed=3, n_requests=5, couette_n=(4, 8), cavity_n=(6, 10),
                                  cylinder_cells=(100, 300), re_range=(5.0, 20.0), cylinder_re=(5.0, 10.0))
    rq = [Request(r["rid"], r["arrival"], r["mesh"], r["bcs"], r["params"], r["kind"], r["n_cells"]) for r in trace]
    clock = SimClock()
    srv = Server(OracleBackend(oracle_mod), budget_bytes=10**9, interval=200, tol=1e-6, step_cap=4000,
                 keep_macros=True, clock=clock, sleep=clock.sleep)
    res, stats = srv.run(rq)
    for r, q in zip(res, rq):
        o = oracle_mod.Oracle(q.mesh, q.bcs, **q.params)
        o.step(r.steps)
        for a, b in zip(r.macros, o.macros()):
            assert np.array_equal(a, b)
    assert stats["converged"] + stats["not_converged"] == 5


class PlateauInst(FakeInst):
    """Like the FP32 deviation form: the residual falls tenfold per 1000 steps
    down to a floor of 1e-6, above the tolerance."""

    def residual(self):
        assert not self.closed
        return max(1e-6, 10.0 ** (-self.steps / 1000.0))


class PreciseInst(FakeInst):
    """The FP64 continuation: converges 3000 steps after it takes over."""

    def __init__(self, req, clock, log, start):
        super().__init__(req, clock, log)
        self.start = self.steps = start

    def residual(self):
        assert not self.closed
        return 1e-9 if self.steps >= self.start + 3000 else 1e-6


class EscalatingBackend(FakeBackend):
    def __init__(self, clock):
        super().__init__(clock)
        self.escalated, self.old = [], []

    def create(self, req):
        inst = PlateauInst(req, self.clock, self.log)
        self.live[req.rid] = inst
        return inst

    def escalate(self, req, inst, room):
        need = 2 * self.bytes(req)
        if need > room:
            return None
        new = PreciseInst(req, self.clock, self.log, inst.steps)
        self.escalated.append((req.rid, inst.steps))
        self.old.append(inst)
        self.live[req.rid] = new
        return new, need


def _serve_escalating(budget, **kw):
    clock = SimClock()
    be = EscalatingBackend(clock)
    srv = Server(be, budget_bytes=budget, clock=clock, sleep=clock.sleep, interval=1000, tol=1e-7,
                 stall_checks=4, **kw)
    res, stats = srv.run(reqs([(0.0, 100, {}), (0.0, 100, {})]))
    return res, stats, srv, be


def test_stalled_request_escalated_and_converges():
    """The residual floors at step 6000; four checks later (step 10000) the
    request continues in the precise form and converges 3000 steps after."""
    res, stats, srv, be = _serve_escalating(budget=10**6, step_cap=50_000)
    assert [r.status for r in res] == ["converged", "converged"]
    assert [s for _, s in be.escalated] == [10_000, 10_000]
    assert [r.steps for r in res] == [13_000, 13_000]
    assert all(inst.closed for inst in be.old) and all(inst.closed for inst in be.live.values())
    assert sum(ev == "escalate" for _, ev, _, _ in srv.log) == 2


def test_escalation_needs_room_in_the_budget():
    """The precise form needs twice the bytes: with room for neither request
    to double, both run on to the step cap."""
    res, stats, srv, be = _serve_escalating(budget=25_000, step_cap=20_000)
    assert be.escalated == []
    assert [r.status for r in res] == ["not_converged", "not_converged"]


def test_batch_signature_separates_member_sets():
    import meshgen
    from paper_2007_07347_amd import autotune
    a = [(*meshgen.cavity(12), dict(nu=1e-3)), (*meshgen.cavity(16), dict(nu=1e-3))]
    b = [(*meshgen.cavity(12), dict(nu=1e-3)), (*meshgen.cavity(16), dict(nu=2e-3))]
    assert autotune.batch_signature(a) == autotune.batch_signature(list(a))
    assert autotune.batch_signature(a) != autotune.batch_signature(b)
    assert autotune.batch_signature(a) != autotune.batch_signature(a[:1])


# ---- admission on a worker and one batched residual per chunk
class SimFuture:
    """Ready once the simulated clock passes `ready_at`."""

    def __init__(self, clock, ready_at, value):
        self.clock, self.ready_at, self.value = clock, ready_at, value

    def done(self):
        return self.clock.t >= self.ready_at

    def result(self):
        if not self.done():                 # waiting costs the time left
            self.clock.t = self.ready_at
        return self.value


class ResidualBatch(FakeBatch):
    def residuals(self):
        out, bad = [], False
        for m in self.members:
            try:
                out.append(m.residual())
            except RuntimeError:
                out.append(math.nan)
                bad = True
        if bad:
            e = RuntimeError("not finite")
            e.code, e.residuals = -4, out
            raise e
        return out


class AsyncBackend(FakeBackend):
    """Instances take `make_s` simulated seconds to build on the worker."""

    def __init__(self, clock, make_s=0.01):
        super().__init__(clock)
        self.make_s, self.made_at = make_s, {}

    def create_async(self, req):
        inst = self.create(req)
        self.made_at[req.rid] = self.clock.t + self.make_s
        return SimFuture(self.clock, self.clock.t + self.make_s, inst)

    def batch(self, instances):
        return ResidualBatch(instances, self.clock, self.log)


def test_async_admission_overlaps_the_running_batch():
    """A request admitted while another runs is built on the worker; the
    batch keeps stepping meanwhile (chunks without it), and it joins at the
    first chunk boundary after it is ready.  Budget accounting includes the
    instances still being built; a poisoned member is isolated by the
    batched residual."""
    clock = SimClock()
    be = AsyncBackend(clock, make_s=0.01)
    specs = [(0.0, 10, {"need": 40_000}), (0.001, 10, {"need": 3000}), (0.001, 10, {"need": 5000, "poison": True}),
             (0.002, 10, {"need": 1000})]
    srv = Server(be, budget_bytes=3 * 1000, clock=clock, sleep=clock.sleep, interval=1000)
    res, stats = srv.run(reqs(specs))
    assert [r.status for r in res] == ["converged", "converged", "diverged", "converged"]
    batches = [m for kind, m in be.log if kind == "batch"]
    # request 0 ran alone while 1 and 2 were being built, then with them
    first_joint = next(k for k, m in enumerate(batches) if 1 in m)
    assert first_joint > 1 and all(m == (0,) for m in batches[:first_joint])
    t_admit = {rid: t for t, ev, rid, _ in srv.log if ev == "admit"}
    assert t_admit[3] >= min(res[1].finished, res[2].finished)   # 3 waited for budget, FIFO
    assert all(inst.closed for inst in be.live.values())


# ---- a request whose instance cannot be made fails alone
class FailingBackend(AsyncBackend):
    """create() raises for requests marked "bad" (as the library does for a
    mesh it rejects); create_async() hands the error over through the future."""

    def __init__(self, clock, use_async):
        super().__init__(clock)
        self.use_async = use_async
        if not use_async:
            self.create_async = None

    def bytes(self, req):
        if req.params.get("unsized"):
            e = ValueError(f"parameters of request {req.rid} rejected")
            e.code = -1
            raise e
        return super().bytes(req)

    def create(self, req):
        if req.params.get("bad"):
            e = ValueError(f"mesh of request {req.rid} rejected")
            e.code = -1
            raise e
        return super().create(req)

    def batch(self, instances):
        return FakeBatch(instances, self.clock, self.log)


class FailedFuture(SimFuture):
    def __init__(self, clock, ready_at, err):
        super().__init__(clock, ready_at, None)
        self.err = err

    def result(self):
        super().result()
        raise self.err


@pytest.mark.parametrize("use_async", [False, True])
def test_failed_creation_isolated_and_budget_returned(use_async):
    clock = SimClock()
    be = FailingBackend(clock, use_async)
    if use_async:
        def create_async(req):
            try:
                inst = be.create(req)
            except ValueError as e:
                return FailedFuture(clock, clock.t + 0.01, e)
            return SimFuture(clock, clock.t + 0.01, inst)
        be.create_async = create_async
    # the budget holds one request at a time: the failed one must give its bytes back
    specs = [(0.0, 10, {"need": 2000, "bad": True}), (0.0, 10, {"need": 2000}), (0.0, 10, {"need": 1000, "bad": True}),
             (0.0, 10, {"need": 1000}), (0.0, 10, {"need": 1000, "unsized": True}), (0.0, 10, {"need": 1000})]
    srv = Server(be, budget_bytes=1000, clock=clock, sleep=clock.sleep, interval=1000)
    res, stats = srv.run(reqs(specs))
    assert [r.status for r in res] == ["failed", "converged", "failed", "converged", "failed", "converged"]
    assert "rejected" in res[0].error and res[1].error == "" and "parameters" in res[4].error
    assert stats["failed"] == 3 and stats["converged"] == 3
    assert all(inst.closed for inst in be.live.values())


def test_failed_creation_in_the_sequential_loop():
    clock = SimClock()
    be = FailingBackend(clock, use_async=False)
    srv = SequentialServer(be, budget_bytes=10**6, clock=clock, sleep=clock.sleep, interval=1000)
    res, stats = srv.run(reqs([(0.0, 10, {"need": 1000, "bad": True}), (0.0, 10, {"need": 1000}),
                               (0.0, 10, {"need": 1000, "unsized": True})]))
    assert [r.status for r in res] == ["failed", "converged", "failed"]


def test_failed_escalation_keeps_the_first_form():
    """An escalation that raises leaves the request in its first form, not
    escalated again, and it runs on to the step cap."""
    clock = SimClock()
    be = EscalatingBackend(clock)

    def boom(req, inst, room):
        raise MemoryError("no room on the device")
    be.escalate = boom
    srv = Server(be, budget_bytes=10**6, clock=clock, sleep=clock.sleep, interval=1000, tol=1e-7,
                 stall_checks=4, step_cap=20_000)
    res, stats = srv.run(reqs([(0.0, 100, {})]))
    assert [r.status for r in res] == ["not_converged"]
    assert sum(ev == "escalate_failed" for _, ev, _, _ in srv.log) == 1
    assert all(inst.closed for inst in be.live.values())

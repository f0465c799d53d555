"""Serving loop on the GPU: requests admitted by HBM budget into one running
batch give, bit for bit, the result of the same request solved alone for the
same number of steps; a request whose FP32-deviation residual stalls above
the tolerance is continued with FP64 arithmetic (same FP32 storage) and
converges."""
import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone():
    import torch
    assert torch.cuda.is_available()
    from paper_2007_07347_amd import sdugks, serve
    trace = meshgen.serving_trace(seed=11, n_requests=8, rate=200.0, couette_n=(8, 16), cavity_n=(12, 24),
                                  cylinder_cells=(500, 2000), re_range=(10.0, 60.0), cylinder_re=(10.0, 20.0))
    rq = [serve.Request(r["rid"], r["arrival"], r["mesh"], r["bcs"], r["params"], r["kind"], r["n_cells"])
          for r in trace]
    backend = serve.GpuBackend()
    budget = sum(backend.bytes(q) for q in rq[:3])          # at most about three at a time
    srv = serve.Server(backend, budget_bytes=budget, interval=500, tol=1e-7, step_cap=6000, keep_macros=True,
                       stall_checks=0)
    res, stats = srv.run(rq)
    print(stats, flush=True)
    assert stats["requests"] == 8 and stats["rejected"] == 0
    admits = [e for e in srv.log if e[1] == "admit"]
    assert [e[2] for e in admits] == sorted(e[2] for e in admits)
    for r, q in zip(res, rq):
        s = sdugks.Solver(q.mesh, q.bcs, precision=sdugks.FP32DEV, **q.params)
        for _ in range(r.steps // 500):
            s.step(500)
        for a, b in zip(r.macros, s.macros()):
            assert np.array_equal(a, b)
        s.close()


def test_stalled_request_continues_with_fp64_arithmetic():
    """Cylinder at Re 20 on a coarse O-grid: the deviation form's residual
    floors above 1e-7, the server continues the request from its current state
    with FP64 arithmetic on the same FP32 storage, and it converges to the
    FP64 solution."""
    import torch
    assert torch.cuda.is_available()
    from paper_2007_07347_amd import sdugks, serve
    mesh, bcs = meshgen.cylinder_ogrid(64, 24, seed=1)
    params = dict(nu=0.1 / 20, cfl=0.5, u0=0.1)
    q = serve.Request(0, 0.0, mesh, bcs, params, "cylinder", 2 * 64 * 24)
    srv = serve.Server(serve.GpuBackend(), budget_bytes=1 << 30, interval=1000, tol=1e-7, step_cap=400_000,
                       keep_macros=True, stall_checks=8)
    (r,), stats = srv.run([q])
    print(r.status, r.steps, r.residual, [e for e in srv.log if e[1] == "escalate"], flush=True)
    assert r.status == "converged" and r.residual <= 1e-7
    assert [e[1] for e in srv.log].count("escalate") == 1
    ref = sdugks.Solver(mesh, bcs, precision=sdugks.FP64, **params)
    eps = 1.0
    while eps > 1e-8:
        ref.step(5000)
        eps = ref.residual()
    _, u, v = ref.macros()
    _, us, vs = r.macros
    l2 = np.sqrt(((us - u) ** 2 + (vs - v) ** 2).sum() / (u ** 2 + v ** 2).sum())
    print("velocity L2 against FP64 alone", l2, flush=True)
    assert l2 <= 1e-5
    ref.close()


def test_rejected_parameters_fail_alone():
    """Requests the library refuses (no viscosity; the structured step asked
    for on a triangle mesh) end as "failed" with the library's message, and
    the valid requests of the same trace are served bit for bit as alone."""
    import torch
    assert torch.cuda.is_available()
    from paper_2007_07347_amd import sdugks, serve
    good = [(meshgen.cavity(12), dict(nu=1e-3, cfl=0.5)), (meshgen.couette(4, 8), dict(nu=0.01, cfl=0.5))]
    bad = [(meshgen.cavity(12), dict(nu=-1.0, cfl=0.5)),
           (meshgen.cylinder_ogrid(24, 8, seed=1), dict(nu=2.5e-3, cfl=0.5, u0=0.1, structured=2))]
    specs = [good[0], bad[0], good[1], bad[1]]
    rq = [serve.Request(k, 0.0, m, b, p, "test", len(m["cell_ptr"]) - 1) for k, ((m, b), p) in enumerate(specs)]
    srv = serve.Server(serve.GpuBackend(), budget_bytes=1 << 30, interval=500, tol=1e-7, step_cap=2000,
                       keep_macros=True, stall_checks=0)
    res, stats = srv.run(rq)
    print([(r.status, r.error) for r in res], flush=True)
    assert [r.status != "failed" for r in res] == [True, False, True, False]
    assert "nu" in res[1].error and "structured" in res[3].error
    for r, q in zip(res, rq):
        if r.status == "failed":
            continue
        s = sdugks.Solver(q.mesh, q.bcs, precision=sdugks.FP32DEV, **q.params)
        for _ in range(r.steps // 500):
            s.step(500)
        for a, b in zip(r.macros, s.macros()):
            assert np.array_equal(a, b)
        s.close()

"""Serving loop on the GPU: requests admitted by HBM budget into one running
batch give, bit for bit, the result of the same request solved alone for the
same number of steps."""
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
    srv = serve.Server(backend, budget_bytes=budget, interval=500, tol=1e-7, step_cap=6000, keep_macros=True)
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

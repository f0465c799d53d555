"""The allocation-free residual entry point (sdugks_residuals_static) called
through the C ABI, against the batched residual of a batch object
(sdugks_batch_residual) on identically stepped twins: bitwise equal, on two
calls in a row, the second with fewer and smaller members."""
import ctypes as C

import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2007_07347_amd import sdugks
    return sdugks


def static_residuals(sd, solvers):
    arr = (C.c_void_p * len(solvers))(*[s.handle for s in solvers])
    eps = np.zeros(len(solvers))
    rc = sd._lib.sdugks_residuals_static(arr, len(solvers), eps.ctypes.data_as(C.c_void_p))
    return rc, eps


def test_static_residuals_equal_batch_residuals(sd):
    import torch
    print("no-alloc residuals: two calls, the second smaller", flush=True)
    stream = torch.cuda.Stream()
    cases = [(37, sd.FP64), (64, sd.FP32DEV), (21, sd.FP64), (90, sd.FP32DEV), (12, sd.FP64)]

    def make():
        return [sd.Solver(*meshgen.cavity(n), stream=stream, nu=1e-3, cfl=0.5, precision=p) for n, p in cases]

    A, B = make(), make()
    batch = sd.Batch(A, stream=stream)
    for s in B:
        s.step(25)
    batch.step(25)
    # first call: all five members (the first check after rest is +inf)
    for _ in range(2):
        ea = batch.residuals()
        rc, eb = static_residuals(sd, B)
        assert rc == sd.OK
        assert np.array_equal(ea, eb), (ea, eb)
        batch.step(30)
        for s in B:
            s.step(30)
    # second call: fewer, smaller members
    small = [0, 2, 4]
    batch.set_members([A[k] for k in small])
    batch.step(10)
    for k in small:
        B[k].step(10)
    ea = batch.residuals()
    rc, eb = static_residuals(sd, [B[k] for k in small])
    assert rc == sd.OK and np.isfinite(eb).all()
    assert np.array_equal(ea, eb), (ea, eb)
    # refusals: beyond the maximum, duplicates, mixed streams
    rc, _ = static_residuals(sd, [B[0]] * 1025)
    assert rc == sd.EINVAL and b"at most 1024" in sd._lib.sdugks_last_error()
    rc, _ = static_residuals(sd, [B[0], B[0]])
    assert rc == sd.EINVAL
    other = sd.Solver(*meshgen.cavity(9), nu=1e-3, cfl=0.5)
    rc, _ = static_residuals(sd, [B[1], other])
    assert rc == sd.EINVAL and b"one stream" in sd._lib.sdugks_last_error()
    other.close()
    batch.close()
    for s in A + B:
        s.close()

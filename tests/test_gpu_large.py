"""Parity at the large launch configuration: the 2048 x 2048 tanh cavity
(4.2M cells, working set above 0.8 GB) on both steps the bench times there
(the general step on 64-cell tiles and 256 threads, and the structured step
on its 16 x 14 or 16 x 7 tiles), against the oracle on sampled cells.

The oracle cannot step 4.2M cells in a test, but one step of a cell depends
only on the state of the cells within two faces of it (its own and its
neighbours' fbar+ and gradients, and the first ring's gradients read the
second ring).  So for each sampled cell the oracle steps a 7 x 7 window of
the same nodes around it, from the GPU's state, with the GPU's time step;
window sides inside the cavity are closed by a resting wall of an extra tag,
whose effect cannot reach the centre cell in one step.  The centre cell's
f and W must then agree with the GPU's to the parity bar."""
import numpy as np
import pytest

import meshgen

N = 2048
NU = 1e-4


@pytest.fixture(scope="module")
def sd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2007_07347_amd import sdugks
    return sdugks


def samples(n, seed=11, n_interior=6):
    rng = np.random.default_rng(seed)
    fixed = [(0, 0), (n - 1, 0), (0, n - 1), (n - 1, n - 1), (n // 2, 0), (0, n // 2), (n - 1, n // 2),
             (n // 2, n - 1), (1, 1), (n - 2, n - 2), (63, 64), (64, 63),
             (15, 14), (16, 13), (32, 7), (33, 6)]      # tile corners of both steps
    rand = [tuple(int(x) for x in rng.integers(2, n - 2, size=2)) for _ in range(n_interior)]
    return fixed + rand


def window(xs, i0, j0, r=3):
    """The sub-grid of cells within r cells of (i0, j0) in each direction:
    its mesh, its boundary conditions and the global ids of its cells."""
    n = len(xs) - 1
    il, ih = max(i0 - r, 0), min(i0 + r, n - 1)
    jl, jh = max(j0 - r, 0), min(j0 + r, n - 1)
    art = 2                                           # the window's own sides: a resting wall
    mesh = meshgen.structured(xs[il:ih + 2], xs[jl:jh + 2],
                              tag_bottom=0 if jl == 0 else art, tag_right=0 if ih == n - 1 else art,
                              tag_top=1 if jh == n - 1 else art, tag_left=0 if il == 0 else art)
    J, I = np.meshgrid(np.arange(jl, jh + 1), np.arange(il, ih + 1), indexing="ij")
    gid = (J * n + I).ravel()
    centre = int(np.flatnonzero(gid == j0 * n + i0)[0])
    return mesh, gid, centre


def test_window_step_equals_full_step(oracle_mod):
    """The locality the GPU test relies on, on the CPU with the oracle alone:
    on a 40 x 40 cavity from a generic state, one oracle step of a 7 x 7
    window gives its centre cell the same bits as one step of the whole
    mesh, at corners, walls, the lid and inside; a 3 x 3 window does not."""
    n = 40
    mesh, bcs = meshgen.cavity(n)
    xs = meshgen.tanh_nodes(n)
    o = oracle_mod.Oracle(mesh, bcs, nu=NU, cfl=0.5)
    f0, W0, _ = meshgen.random_state(o.n_cells, seed=17, amp=0.02)
    o.set_state(f0, W0)
    o.step(1)
    f1, W1, _ = o.state()
    cells = [s for s in samples(n, n_interior=10) if max(s) < n] + [(5, 6), (20, 1), (38, 20)]
    for i0, j0 in cells:
        wmesh, gid, c = window(xs, i0, j0)
        ow = oracle_mod.Oracle(wmesh, bcs + [meshgen.bc(meshgen.WALL)], nu=NU, dt=o.dt)
        ow.set_state(f0[gid], W0[gid])
        ow.step(1)
        fo, Wo, _ = ow.state()
        assert np.array_equal(fo[c], f1[gid[c]]) and np.array_equal(Wo[c], W1[gid[c]]), (i0, j0)
    wmesh, gid, c = window(xs, 20, 20, r=1)
    ow = oracle_mod.Oracle(wmesh, bcs + [meshgen.bc(meshgen.WALL)], nu=NU, dt=o.dt)
    ow.set_state(f0[gid], W0[gid])
    ow.step(1)
    assert np.abs(ow.state()[0][c] - f1[gid[c]]).max() > 1e-6


@pytest.mark.gpu
@pytest.mark.parametrize("step", ["general", "structured"])
@pytest.mark.parametrize("precision,bar", [("FP64", 1e-12), ("FP32DEV", 2e-6)])
def test_cavity_2048_sampled_cells(sd, oracle_mod, precision, bar, step):
    mesh, bcs = meshgen.cavity(N)
    xs = meshgen.tanh_nodes(N)
    sched = dict(tile_cells=64, block_threads=256) if step == "general" else dict(structured=2)
    g = sd.Solver(mesh, bcs, nu=NU, cfl=0.5, precision=getattr(sd, precision), **sched)
    assert g.n_cells == N * N
    f0, W0, _ = meshgen.random_state(g.n_cells, seed=17, amp=0.02)
    g.set_state(f0, W0)
    f0, W0, _ = g.state()                 # as stored (FP32 deviation form rounds f)
    g.step(1)
    f1, W1, _ = g.state()
    dt = g.dt
    g.close()
    worst = 0.0
    for i0, j0 in samples(N):
        wmesh, gid, c = window(xs, i0, j0)
        o = oracle_mod.Oracle(wmesh, bcs + [meshgen.bc(meshgen.WALL)], nu=NU, dt=dt)
        assert o.dt == dt
        o.set_state(f0[gid], W0[gid])
        o.step(1)
        fo, Wo, _ = o.state()
        ef = np.abs(f1[gid[c]] - fo[c]).max() / np.abs(fo[c]).max()
        ew = np.abs(W1[gid[c]] - Wo[c]).max() / np.abs(Wo[c]).max()
        worst = max(worst, ef, ew)
        assert ef <= bar and ew <= bar, ((i0, j0), ef, ew)
    print(precision, step, "worst sampled relative error", f"{worst:.2e}", flush=True)

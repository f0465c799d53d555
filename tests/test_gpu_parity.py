"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle,
element by element on the same seeded inputs.

Tolerance: FP64 results agree within 1e-12 relative, rel-Linf(x, y) =
max|x - y| / max|y| per field (f, rho, momentum (rho u, rho v) on one scale,
G).  The oracle rounds
every operation separately (no contraction) and sums in its own order; the
GPU contracts multiply-adds and sums in another order, so results differ at
the 1e-16 level per operation and stay many orders below the bar over the
windows used here (the scheme is dissipative).
"""
import math
import sys

import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def sd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2007_07347_amd import sdugks
    return sdugks


def rel_linf(x, y):
    d = np.abs(x - y).max()
    s = np.abs(y).max()
    return d / s if s > 0 else d


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare(gpu, orc, what, tol=TOL, lagged=False):
    """Element-wise comparison; G (the stored macroscopic flux) only exists in
    the lagged reading."""
    fg, Wg, Gg = gpu.state()
    fo, Wo, Go = orc.state()
    # momentum components share one scale: a component that is zero up to
    # rounding (v in Couette flow) has no meaningful relative error of its own
    errs = {"f": rel_linf(fg, fo), "rho": rel_linf(Wg[:, 0], Wo[:, 0]),
            "momentum": rel_linf(Wg[:, 1:], Wo[:, 1:])}
    if lagged:
        errs["G"] = rel_linf(Gg, Go)
    say(what, {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= tol, (what, k, v)
    return errs


def test_couette_full_run(sd, oracle_mod):
    """Planar Couette flow, 4 x 32, Re = 10, CFL 0.5, 5000 steps from rest: the
    whole run on the GPU against the oracle, and the profile against the
    diffusion series."""
    say("couette 4x32, 5000 steps")
    mesh, bcs = meshgen.couette(4, 32, 0.1)
    g = sd.Solver(mesh, bcs, nu=0.01, cfl=0.5)
    o = oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5)
    assert g.dt == pytest.approx(o.dt, rel=1e-15)
    g.step(5000)
    o.step(5000)
    compare(g, o, "couette")
    rho, u, v = g.macros()
    y = o.geometry()["cy"]
    series = 0.1 * y + sum(2 * 0.1 / (m * math.pi) * (-1) ** m * np.sin(m * math.pi * y)
                           * math.exp(-(m * math.pi) ** 2 * 0.01 * 5000 * g.dt) for m in range(1, 400))
    assert np.abs(u - series).max() < 1e-5


def _free_slip_couette():
    mesh, bcs = meshgen.couette(5, 12)
    bcs = list(bcs)
    bcs[0] = meshgen.bc(meshgen.SYMMETRY)
    return mesh, bcs


def _half_channel():
    """Upper half of a channel: inlet on the left, outlet on the right, a wall
    on top and the centre line below as a symmetry side."""
    mesh = meshgen.structured(np.linspace(0.0, 1.0, 14), meshgen.tanh_nodes(7, 1.0), tag_bottom=3, tag_right=1,
                              tag_top=0, tag_left=2)
    return mesh, [meshgen.bc(meshgen.WALL), meshgen.bc(meshgen.OUTLET), meshgen.bc(meshgen.INLET, u=0.05),
                  meshgen.bc(meshgen.SYMMETRY)]


def _small_cases():
    return {
        "cavity_23": (lambda: meshgen.cavity(23), dict(nu=0.001, cfl=0.5)),
        "couette_5x16": (lambda: meshgen.couette(5, 16), dict(nu=0.01, cfl=0.5)),
        "ogrid_37x11": (lambda: meshgen.cylinder_ogrid(37, 11, seed=4), dict(nu=0.0025, cfl=0.5, u0=0.1)),
        "periodic_tri_9": (lambda: meshgen.jittered_periodic_triangles(9, seed=6), dict(nu=0.004, cfl=0.5)),
        "hexagons_7x5": (lambda: meshgen.hexagon_strip(7, 5), dict(nu=0.01, cfl=0.5)),
        "inlet_outlet_13x9": (lambda: meshgen.inlet_outlet_box(13, 9), dict(nu=0.005, cfl=0.5)),
        "hybrid_ogrid_40x12": (lambda: meshgen.cylinder_ogrid(40, 12, seed=7, quad_layers=4),
                               dict(nu=0.0025, cfl=0.5, u0=0.1)),
        "hybrid_cavity_17": (lambda: (meshgen.split_some(meshgen.cavity(17)[0], 0.3, seed=4), meshgen.cavity(17)[1]),
                             dict(nu=0.001, cfl=0.5)),
        "symmetry_couette_rot": (lambda: meshgen.rotate(*_free_slip_couette(), 0.37), dict(nu=0.01, cfl=0.5)),
        "symmetry_half_channel": (lambda: _half_channel(), dict(nu=0.005, cfl=0.5)),
        "relabeled_cavity_11": (lambda: (meshgen.relabel(meshgen.cavity(11)[0], seed=2)[0], meshgen.cavity(11)[1]),
                                dict(nu=0.002, cfl=0.5)),
    }


# "fused": the library's choice (the structured step on tensor-product quad
# meshes, the general fused step otherwise); "general": the general fused step
# on every mesh
PATHS = {"fused": dict(tile_cells=0), "general": dict(structured=1),
         "fused_t16_b64": dict(tile_cells=16, block_threads=64), "two_kernel": dict(tile_cells=-1)}


@pytest.mark.parametrize("name", sorted(_small_cases()))
@pytest.mark.parametrize("macro", [1, 0])
@pytest.mark.parametrize("path", sorted(PATHS))
def test_random_state_window(sd, oracle_mod, name, macro, path):
    """A seeded generic state (every term of the step active) advanced 40
    steps on ragged small meshes covering walls, a moving lid, far-field inlet,
    outlet, periodic gluing, triangles, hexagons (eight lanes per cell) and a
    shuffled cell order; both macroscopic-flux readings; the fused tiled step
    (two tile shapes) and the two-kernel step."""
    build, kw = _small_cases()[name]
    kw = dict(kw, **PATHS[path])
    mesh, bcs = build()
    if macro == 0:
        kw = dict(kw, tau=0.0, cfl=0.2)
    say("window", name, "macro", macro, "path", path)
    okw = {k: v for k, v in kw.items() if k not in ("tile_cells", "block_threads", "structured")}
    o = oracle_mod.Oracle(mesh, bcs, macro=macro, **okw)
    if macro == 0 and o.dt > 2.0 * o.tau:
        pytest.skip("lagged flux is unstable at this dt/tau")
    g = sd.Solver(mesh, bcs, macro=macro, **kw)
    f, W, G = meshgen.random_state(o.n_cells, seed=17)
    if macro == 1:
        G[:] = 0.0
    o.set_state(f, W, G)
    g.set_state(f, W, G)
    o.step(1)
    g.step(1)
    compare(g, o, f"{name} step 1", lagged=macro == 0)
    o.step(39)
    g.step(39)
    compare(g, o, f"{name} step 40", lagged=macro == 0)


@pytest.mark.parametrize("sched", [{}, {"tile_cells": 32, "block_threads": 128}])
def test_cavity_256_window(sd, oracle_mod, sched):
    """Lid-driven cavity, 256 x 256 tanh mesh (stretching 1.5), Re = 1000,
    CFL 0.5, from rest: the first 60 steps of the full-size case, on the
    default schedule and on the one the bench's headline runs."""
    say("cavity 256, 60 steps", sched)
    mesh, bcs = meshgen.cavity(256)
    g = sd.Solver(mesh, bcs, nu=0.1 / 1000, cfl=0.5, **sched)
    o = oracle_mod.Oracle(mesh, bcs, nu=0.1 / 1000, cfl=0.5)
    g.step(60)
    o.step(60)
    compare(g, o, "cavity256")
    assert g.mass() == pytest.approx(o.mass(), rel=1e-13)


def test_cylinder_200k_window(sd, oracle_mod):
    """Flow past a cylinder at Re = 40 on the 400 x 250 jittered triangle
    O-grid (200,000 cells), far-field inflow 0.1: the first 12 steps of the
    full-size case, FP64."""
    say("cylinder 200k, 12 steps")
    mesh, bcs = meshgen.cylinder_ogrid(400, 250, seed=0)
    kw = dict(nu=0.1 * 1.0 / 40, cfl=0.5, u0=0.1)
    g = sd.Solver(mesh, bcs, **kw)
    o = oracle_mod.Oracle(mesh, bcs, **kw)
    assert g.n_cells == 200000
    g.step(12)
    o.step(12)
    compare(g, o, "cylinder200k")


@pytest.mark.parametrize("case", ["cavity256_t32_b128", "cylinder200k_t64_b256"])
def test_full_size_generic_state_window(sd, oracle_mod, case):
    """Full-size meshes from a seeded generic state (every term of the step
    active in every cell from the first step): the 256 x 256 cavity at Re 1000
    on the 32-cell / 128-thread schedule and the 200,000-triangle cylinder at
    Re 40 on the 64-cell / 256-thread schedule, 40 steps, FP64, compared with
    the oracle after the first step and after the 40th."""
    if case.startswith("cavity"):
        mesh, bcs = meshgen.cavity(256)
        kw = dict(nu=0.1 / 1000, cfl=0.5)
        sched = dict(tile_cells=32, block_threads=128)
    else:
        mesh, bcs = meshgen.cylinder_ogrid(400, 250, seed=0)
        kw = dict(nu=0.1 / 40, cfl=0.5, u0=0.1)
        sched = dict(tile_cells=64, block_threads=256)
    say("full-size generic window", case)
    g = sd.Solver(mesh, bcs, **sched, **kw)
    o = oracle_mod.Oracle(mesh, bcs, **kw)
    f, W, G = meshgen.random_state(o.n_cells, seed=23, amp=0.02)
    G[:] = 0.0
    o.set_state(f, W, G)
    g.set_state(f, W, G)
    o.step(1)
    g.step(1)
    compare(g, o, f"{case} step 1")
    o.step(39)
    g.step(39)
    compare(g, o, f"{case} step 40")
    assert g.mass() == pytest.approx(o.mass(), rel=1e-13)


def test_fused_and_two_kernel_paths_agree(sd):
    """The fused tiled step and the two-kernel step on the full 200k-cell
    cylinder mesh, several tile shapes: equal to rounding after 50 steps."""
    mesh, bcs = meshgen.cylinder_ogrid(400, 250, seed=0)
    kw = dict(nu=0.0025, cfl=0.5, u0=0.1)
    ref = sd.Solver(mesh, bcs, tile_cells=-1, **kw)
    ref.step(50)
    fr, Wr, _ = ref.state()
    for tc, bt in ((0, 256), (32, 128), (16, 64), (32, 256)):
        say("fused", tc, bt, sd.tiling(mesh, bcs, tile_cells=tc, **kw))
        g = sd.Solver(mesh, bcs, tile_cells=tc, block_threads=bt, **kw)
        g.step(50)
        f, W, _ = g.state()
        assert rel_linf(f, fr) <= 1e-13 and rel_linf(W, Wr) <= 1e-13


@pytest.mark.parametrize("n", [31, 64])
def test_residual_and_mass_match_oracle(sd, oracle_mod, n):
    """n = 64: 4096 cells, a multiple of 2048, so the rows carry padding."""
    mesh, bcs = meshgen.cavity(n)
    g = sd.Solver(mesh, bcs, nu=0.001, cfl=0.5)
    o = oracle_mod.Oracle(mesh, bcs, nu=0.001, cfl=0.5)
    assert g.residual() == math.inf and o.residual() == math.inf
    for _ in range(3):
        g.step(200)
        o.step(200)
        rg, ro = g.residual(), o.residual()
        assert rg == pytest.approx(ro, rel=1e-10)
        assert g.mass() == pytest.approx(o.mass(), rel=1e-13)


def test_exact_conservation_periodic(sd):
    """Each face flux leaves one cell exactly as it enters the other: total
    mass on a periodic mesh stays at its initial value to rounding of the
    final sum over 2000 steps from a generic state."""
    mesh, bcs = meshgen.jittered_periodic_triangles(24, seed=8)
    g = sd.Solver(mesh, bcs, nu=0.004, cfl=0.5)
    f, W, _ = meshgen.random_state(g.n_cells, seed=5)
    g.set_state(f, W)
    m0 = g.mass()
    g.step(2000)
    assert abs(g.mass() - m0) / m0 <= 1e-13


def test_deterministic_and_order_independent(sd):
    """Two runs give bit-identical states; RCM on/off agrees to rounding."""
    mesh, bcs = meshgen.cylinder_ogrid(64, 20, seed=2)
    runs = []
    for reorder in (True, True, False):
        g = sd.Solver(mesh, bcs, nu=0.002, cfl=0.5, u0=0.1, reorder=reorder)
        g.step(300)
        runs.append(g.state())
    for a, b in zip(runs[0], runs[1]):
        assert np.array_equal(a, b)
    for a, b in zip(runs[0], runs[2]):
        assert rel_linf(a, b) <= 1e-13


def test_step_zero_and_errors(sd):
    mesh, bcs = meshgen.cavity(9)
    g = sd.Solver(mesh, bcs, nu=0.01, cfl=0.5)
    f0, W0, _ = g.state()
    g.step(0)
    f1, W1, _ = g.state()
    assert np.array_equal(f0, f1) and np.array_equal(W0, W1)
    with pytest.raises(sd.SdugksError) as ei:
        g.step(-1)
    assert ei.value.code == sd.EINVAL
    assert g.info()["step"] == 0 and g.info()["n_cells"] == 81


def test_poison_is_detected_and_isolated(sd):
    """A NaN in one instance's f is caught by the residual check and blocks
    further steps of that instance only; set_state clears it."""
    mesh, bcs = meshgen.cavity(12)
    a = sd.Solver(mesh, bcs, nu=0.002, cfl=0.5)
    b = sd.Solver(mesh, bcs, nu=0.002, cfl=0.5)
    a.step(10)
    b.step(10)
    a.poison(37, 4)
    a.step(2)
    b.step(2)
    with pytest.raises(sd.SdugksError) as ei:
        a.residual()
    assert ei.value.code == sd.EDIVERGED
    with pytest.raises(sd.SdugksError):
        a.step(1)
    b.residual()
    rho, u, v = b.macros()
    assert np.isfinite(rho).all() and np.isfinite(u).all()
    f, W, _ = b.state()
    a.set_state(f, W)
    a.step(1)


DEGENERATE = {
    "cavity_1": lambda: meshgen.cavity(1),              # one cell, four boundary faces, no neighbour
    "cavity_2": lambda: meshgen.cavity(2),              # every cell touches two walls
    "couette_1x4": lambda: meshgen.couette(1, 4),       # each cell is its own periodic neighbour
    "couette_2x2": lambda: meshgen.couette(2, 2),
    "periodic_tri_1": lambda: meshgen.jittered_periodic_triangles(1, seed=2),   # two triangles, all faces glued
}


@pytest.mark.parametrize("precision", ["FP64", "FP32DEV"])
@pytest.mark.parametrize("name", sorted(DEGENERATE))
def test_degenerate_meshes(sd, oracle_mod, name, precision):
    """Meshes at the edge of what the method allows: a single cell, cells with
    more boundary faces than neighbours, a cell glued to itself through a
    periodic pair, a two-triangle periodic square.  50 steps from a generic
    state against the oracle, FP64 at the parity bar and the FP32 deviation
    form within its window bar."""
    mesh, bcs = DEGENERATE[name]()
    kw = dict(nu=0.01, cfl=0.5)
    o = oracle_mod.Oracle(mesh, bcs, **kw)
    g = sd.Solver(mesh, bcs, precision=getattr(sd, precision), **kw)
    f, W, _ = meshgen.random_state(o.n_cells, seed=31, amp=0.02)
    o.set_state(f, W)
    g.set_state(f, W)
    o.step(50)
    g.step(50)
    compare(g, o, f"{name} {precision}", tol=TOL if precision == "FP64" else 2e-6)


@pytest.mark.parametrize("precision,tol", [("FP64", 1e-13), ("FP32DEV", 2e-6)])
def test_quarter_turn_symmetry_on_gpu(sd, precision, tol):
    """The fused step on a cavity turned an exact quarter turn, (x, y) ->
    (-y, x), with the lid turned alike, gives the turned flow: the kernels'
    x and y components (lattice, normals, gradients, foot points) are not
    mixed up anywhere."""
    n = 32
    mesh, bcs = meshgen.cavity(n)
    rm = dict(mesh)
    rm["node_xy"] = np.ascontiguousarray(np.stack([-mesh["node_xy"][:, 1], mesh["node_xy"][:, 0]], axis=1))
    rb = [meshgen.bc(meshgen.WALL), meshgen.bc(meshgen.WALL, u=0.0, v=0.1)]
    kw = dict(nu=0.002, cfl=0.5, precision=getattr(sd, precision))
    g1 = sd.Solver(mesh, bcs, **kw)
    g2 = sd.Solver(rm, rb, **kw)
    g1.step(300)
    g2.step(300)
    r1, u1, v1 = g1.macros()
    r2, u2, v2 = g2.macros()
    say("quarter turn", precision, np.abs(r1 - r2).max(), np.abs(u2 + v1).max(), np.abs(v2 - u1).max())
    assert np.abs(r1 - r2).max() <= tol and np.abs(u2 + v1).max() <= tol and np.abs(v2 - u1).max() <= tol
    assert np.abs(v1).max() > 1e-3

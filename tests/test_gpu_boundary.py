"""Boundary face fluxes (wall force, face density) of the HIP diagnostic
against the oracle's, face by face on the same seeded states.

FP64 instances agree within 1e-12 relative per column (scale: the column's
largest magnitude over the faces), like the step itself; the FP32 deviation
form stores f in FP32, so its fluxes carry the FP32 rounding of the stored
state (bound 1e-6)."""
import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)


@pytest.fixture(scope="module")
def sd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2007_07347_amd import sdugks
    return sdugks


CASES = {
    "cavity": (lambda: meshgen.cavity(20), dict(nu=1e-3)),
    "ogrid": (lambda: meshgen.cylinder_ogrid(48, 16, seed=3), dict(nu=2.5e-3, u0=0.1)),
    "couette": (lambda: meshgen.couette(4, 16), dict(nu=1e-2)),
    "inout": (lambda: meshgen.inlet_outlet_box(10, 7), dict(nu=5e-3, u0=0.05)),
    "hexagons": (lambda: meshgen.hexagon_strip(6, 4), dict(nu=5e-3)),
    "symmetry": (lambda: meshgen.rotate(*_free_slip(), 0.6), dict(nu=1e-2)),
}


def _free_slip():
    mesh, bcs = meshgen.couette(4, 10)
    bcs = list(bcs)
    bcs[0] = meshgen.bc(meshgen.SYMMETRY)
    return mesh, bcs


def colwise(a, b):
    scale = np.maximum(np.abs(b).max(0), 1e-300)
    return (np.abs(a - b).max(0) / scale).max()


def pair(sd, oracle_mod, name, seed, **extra):
    mk, kw = CASES[name]
    mesh, bcs = mk()
    g = sd.Solver(mesh, bcs, cfl=0.5, **kw, **extra)
    o = oracle_mod.Oracle(mesh, bcs, cfl=0.5, **kw)
    f, _, _ = meshgen.random_state(g.n_cells, seed=seed, amp=0.02)
    W = np.c_[f.sum(1), f @ EX, f @ EY]
    g.set_state(f, W)
    fg, Wg, _ = g.state()       # the stored state (FP32 deviations rounded) on both sides
    o.set_state(fg, Wg)
    return g, o, mesh, bcs


@pytest.mark.parametrize("path", [dict(), dict(tile_cells=-1)], ids=["fused", "two_kernel"])
@pytest.mark.parametrize("name", ["cavity", "ogrid", "couette", "inout", "hexagons", "symmetry"])
def test_boundary_flux_matches_oracle(sd, oracle_mod, name, path):
    g, o, mesh, bcs = pair(sd, oracle_mod, name, seed=31, **path)
    for rnd in range(2):
        fg, sg = g.boundary_flux()
        fo, tags = o.boundary_flux()
        assert fg.shape == fo.shape
        if len(fo):
            assert colwise(fg, fo) <= 1e-12, (name, rnd)
        for t in range(len(bcs)):
            _, st = g.boundary_flux(t)
            so = fo[tags == t, :3].sum(0)
            assert np.abs(st - so).max() <= 1e-12 * max(np.abs(fo[:, :3]).max() * max(len(fo), 1), 1e-300)
        g.step(7)
        o.step(7)


def test_boundary_flux_fp32_deviation_form(sd, oracle_mod):
    g, o, mesh, bcs = pair(sd, oracle_mod, "ogrid", seed=32, precision=sd.FP32DEV)
    fg, _ = g.boundary_flux()
    fo, _ = o.boundary_flux()
    assert colwise(fg, fo) <= 1e-6


def test_cylinder_wall_force_full_mesh(sd, oracle_mod):
    """The 200,000-cell O-grid: wall face fluxes (400 faces) and the summed
    force on the cylinder from a generic state."""
    mesh, bcs = meshgen.cylinder_ogrid(400, 250, seed=0)
    kw = dict(nu=0.0025, cfl=0.5, u0=0.1)
    g = sd.Solver(mesh, bcs, **kw)
    o = oracle_mod.Oracle(mesh, bcs, **kw)
    f, _, _ = meshgen.random_state(g.n_cells, seed=33, amp=0.01)
    W = np.c_[f.sum(1), f @ EX, f @ EY]
    g.set_state(f, W)
    o.set_state(f, W)
    fg, force = g.boundary_flux(0)
    fo, tags = o.boundary_flux()
    assert colwise(fg, fo) <= 1e-12
    fw = fo[tags == 0, 1:3].sum(0)
    assert np.abs(force[1:] - fw).max() <= 1e-12 * np.abs(fo[tags == 0, 1:3]).sum()


def test_boundary_flux_rejects_bad_tag(sd):
    mesh, bcs = meshgen.cavity(6)
    g = sd.Solver(mesh, bcs, nu=0.01)
    with pytest.raises(sd.SdugksError) as ei:
        g.boundary_flux(len(bcs))
    assert ei.value.code == sd.EINVAL

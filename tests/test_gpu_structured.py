"""The structured step (tensor-product quad meshes, one lane per face) on the
GPU: element-wise parity with the FP64 oracle from generic states on meshes
covering every side condition, ragged tiles and periodic gluing in x, y or
both, down to two cells along an axis; agreement with the general fused step; the batched form bitwise equal
to stepping alone; the full-size 256 x 256 cavity."""
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_linf(x, y):
    d = np.abs(x - y).max()
    s = np.abs(y).max()
    return d / s if s > 0 else d


def _half_channel():
    mesh = meshgen.structured(np.linspace(0.0, 1.0, 14), meshgen.tanh_nodes(7, 1.0), tag_bottom=3, tag_right=1,
                              tag_top=0, tag_left=2)
    return mesh, [meshgen.bc(meshgen.WALL), meshgen.bc(meshgen.OUTLET), meshgen.bc(meshgen.INLET, u=0.05),
                  meshgen.bc(meshgen.SYMMETRY)]


def _periodic_y_channel():
    """Walls left (at rest) and right (moving along y), periodic in y."""
    mesh = meshgen.structured(meshgen.tanh_nodes(9, 1.2), np.linspace(0.0, 0.5, 20), tag_bottom=0, tag_right=2,
                              tag_top=1, tag_left=3)
    return mesh, [meshgen.bc(meshgen.PERIODIC, partner=1, shift=(0.0, 0.5)),
                  meshgen.bc(meshgen.PERIODIC, partner=0, shift=(0.0, -0.5)),
                  meshgen.bc(meshgen.WALL, v=0.05), meshgen.bc(meshgen.WALL)]


CASES = {
    "cavity_23": (lambda: meshgen.cavity(23), dict(nu=1e-3, cfl=0.5)),
    "cavity_40x40_lid": (lambda: meshgen.cavity(40, U=0.05), dict(nu=4e-4, cfl=0.5)),
    # a last tile column one cell wide, ragged tile rows of both shapes
    "cavity_33": (lambda: meshgen.cavity(33), dict(nu=1e-3, cfl=0.5)),
    "couette_4x32": (lambda: meshgen.couette(4, 32, 0.1), dict(nu=0.01, cfl=0.5)),
    "periodic_box_18x9": (lambda: meshgen.periodic_box(18, 9), dict(nu=0.004, cfl=0.5)),
    # several full tiles of either shape in both directions, wrapped across tiles
    "periodic_box_40x30": (lambda: meshgen.periodic_box(40, 30), dict(nu=0.004, cfl=0.5)),
    "periodic_y_channel": (_periodic_y_channel, dict(nu=0.003, cfl=0.5)),
    "inlet_outlet_13x9": (lambda: meshgen.inlet_outlet_box(13, 9), dict(nu=0.005, cfl=0.5)),
    "half_channel_symmetry": (_half_channel, dict(nu=0.005, cfl=0.5)),
    "relabeled_cavity_17": (lambda: (meshgen.relabel(meshgen.cavity(17)[0], seed=2)[0], meshgen.cavity(17)[1]),
                            dict(nu=0.002, cfl=0.5)),
    # the smallest structured meshes: two cells along an axis, every cell on
    # two walls; two periodic columns (each cell's left and right neighbour
    # the same cell, the halo wrapped across both sides); both axes periodic
    "cavity_2": (lambda: meshgen.cavity(2), dict(nu=1e-3, cfl=0.5)),
    "couette_2x3": (lambda: meshgen.couette(2, 3), dict(nu=0.01, cfl=0.5)),
    "periodic_box_2x2": (lambda: meshgen.periodic_box(2, 2), dict(nu=0.004, cfl=0.5)),
}


def test_every_case_takes_the_structured_step(sd):
    for name, (build, kw) in CASES.items():
        mesh, bcs = build()
        t = sd.tiling(mesh, bcs, **kw)
        assert t["structured"], name
        assert not sd.tiling(mesh, bcs, structured=1, **kw)["structured"]


@pytest.mark.parametrize("macro", [1, 0])
@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("name", sorted(CASES))
def test_window_against_oracle(sd, oracle_mod, name, scheme, macro):
    """A seeded generic state advanced 40 steps, FP64, every reading the
    general step supports (both macroscopic-flux time levels, both schemes)."""
    if scheme == 1 and macro == 0:
        pytest.skip("the original scheme has no lagged flux")
    build, kw = CASES[name]
    mesh, bcs = build()
    if macro == 0:
        kw = dict(kw, cfl=0.2)
    say("structured window", name, "scheme", scheme, "macro", macro)
    o = oracle_mod.Oracle(mesh, bcs, macro=macro, scheme=scheme, **kw)
    if macro == 0 and o.dt > 2.0 * o.tau:
        pytest.skip("lagged flux is unstable at this dt/tau")
    g = sd.Solver(mesh, bcs, macro=macro, scheme=scheme, structured=2, **kw)
    f, W, G = meshgen.random_state(o.n_cells, seed=31, amp=0.02)
    if macro == 1:
        G[:] = 0.0
    o.set_state(f, W, G)
    g.set_state(f, W, G)
    for n in (1, 39):
        o.step(n)
        g.step(n)
        fg, Wg, Gg = g.state()
        fo, Wo, Go = o.state()
        errs = {"f": rel_linf(fg, fo), "rho": rel_linf(Wg[:, 0], Wo[:, 0]), "mom": rel_linf(Wg[:, 1:], Wo[:, 1:])}
        if macro == 0:
            errs["G"] = rel_linf(Gg, Go)
        say(name, n, {k: f"{v:.2e}" for k, v in errs.items()})
        for k, v in errs.items():
            assert v <= TOL, (name, n, k, v)
    assert g.mass() == pytest.approx(o.mass(), rel=1e-13)
    g.close()


@pytest.mark.parametrize("macro", [1, 0])
@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("prec", ["fp32dev", "fp32neq"])
@pytest.mark.parametrize("name", ["cavity_2", "cavity_23", "cavity_33", "cavity_40x40_lid", "couette_2x3", "couette_4x32",
                                  "periodic_box_2x2", "periodic_box_18x9", "periodic_box_40x30", "inlet_outlet_13x9"])
def test_fp32_window_against_oracle(sd, oracle_mod, name, prec, scheme, macro):
    """The FP32 storage forms on the structured step, both schemes and both
    macroscopic-flux time levels, 40 steps from a generic state, with the bars
    of the general step's FP32 windows (f and rho relative, momentum over the
    flows' scale rho0 U, U = 0.1)."""
    if scheme == 1 and macro == 0:
        pytest.skip("the original scheme has no lagged flux")
    build, kw = CASES[name]
    mesh, bcs = build()
    if macro == 0:
        kw = dict(kw, cfl=0.2)
    p = sd.FP32DEV if prec == "fp32dev" else sd.FP32NEQ
    o = oracle_mod.Oracle(mesh, bcs, macro=macro, scheme=scheme, **kw)
    if macro == 0 and o.dt > 2.0 * o.tau:
        pytest.skip("lagged flux is unstable at this dt/tau")
    g = sd.Solver(mesh, bcs, precision=p, macro=macro, scheme=scheme, structured=2, **kw)
    f, W, G = meshgen.random_state(o.n_cells, seed=23, amp=0.02)
    if macro == 1:
        G[:] = 0.0
    o.set_state(f, W, G)
    g.set_state(f, W, G)
    o.step(40)
    g.step(40)
    fg, Wg, _ = g.state()
    fo, Wo, _ = o.state()
    ef, er = rel_linf(fg, fo), rel_linf(Wg[:, 0], Wo[:, 0])
    em = np.abs(Wg[:, 1:] - Wo[:, 1:]).max() / max(np.abs(Wo[:, 1:]).max(), 0.1)
    say(name, prec, "scheme", scheme, "macro", macro, f"f {ef:.2e} rho {er:.2e} mom {em:.2e}")
    assert ef <= 2e-6 and er <= 2e-6 and em <= 2e-6


@pytest.mark.parametrize("prec", ["f64", "fp32dev", "fp32neq"])
def test_structured_and_general_steps_agree(sd, prec):
    """Both fused steps on the 64 x 64 cavity from the same generic state: the
    same scheme to rounding after 100 steps.  FP64: 1e-13.  The FP32 forms
    round what they store, so the last-bit differences of the two kernels'
    arithmetic can round a stored value the other way: FP32NEQ 1e-7 (one
    FP32 rounding of the stored part, |f - feq| <= 0.3 in this state, over
    max |f| = 0.46); FP32DEV, whose face arithmetic is FP32, 1e-6."""
    p = {"f64": sd.FP64, "fp32dev": sd.FP32DEV, "fp32neq": sd.FP32NEQ}[prec]
    mesh, bcs = meshgen.cavity(64)
    a = sd.Solver(mesh, bcs, nu=2e-4, cfl=0.5, precision=p, structured=2)
    b = sd.Solver(mesh, bcs, nu=2e-4, cfl=0.5, precision=p, structured=1)
    f, W, _ = meshgen.random_state(a.n_cells, seed=8, amp=0.02)
    a.set_state(f, W)
    b.set_state(f, W)
    a.step(100)
    b.step(100)
    fa, Wa, _ = a.state()
    fb, Wb, _ = b.state()
    tol = {"f64": 1e-13, "fp32neq": 1e-7, "fp32dev": 1e-6}[prec]
    say(prec, "structured vs general", rel_linf(fa, fb), rel_linf(Wa, Wb))
    assert rel_linf(fa, fb) <= tol and rel_linf(Wa, Wb) <= tol


def test_batch_equals_alone(sd):
    """Structured members of all three precisions with general members in one
    batch (three structured launches and two general ones per step): every
    member bitwise equal to stepping it alone, over graph replays and an odd
    step count."""
    specs = [(meshgen.cavity(23), dict(nu=1e-3)), (meshgen.cavity(50), dict(nu=2e-4, precision=1)),
             (meshgen.couette(4, 32), dict(nu=1e-2, precision=2)), (meshgen.periodic_box(18, 9), dict(nu=4e-3)),
             (meshgen.cylinder_ogrid(40, 12, seed=2), dict(nu=2.5e-3, u0=0.1)),
             (meshgen.cavity(30), dict(nu=1e-3, structured=1, precision=1))]

    def make(seed):
        out = []
        for k, ((mesh, bcs), kw) in enumerate(specs):
            s = sd.Solver(mesh, bcs, cfl=0.5, **kw)
            f, W, _ = meshgen.random_state(s.n_cells, seed=seed + k, amp=0.01)
            s.set_state(f, W)
            out.append(s)
        return out

    alone, batched = make(40), make(40)
    b = sd.Batch(batched)
    for n in (1, 37, 70):
        for s in alone:
            s.step(n)
        b.step(n)
        for sa, sb in zip(alone, batched):
            for x, y in zip(sa.state(), sb.state()):
                assert np.array_equal(x, y), n
    b.close()


@pytest.fixture(scope="module")
def cavity_256_oracle(oracle_mod):
    """The oracle's 40 steps of the 256 x 256 cavity from a generic state
    (shared by the three precision forms)."""
    mesh, bcs = meshgen.cavity(256)
    kw = dict(nu=1e-4, cfl=0.5)
    o = oracle_mod.Oracle(mesh, bcs, **kw)
    f, W, _ = meshgen.random_state(o.n_cells, seed=5, amp=0.02)
    o.set_state(f, W)
    o.step(40)
    return mesh, bcs, kw, (f, W), o.state()


@pytest.mark.parametrize("prec", ["f64", "fp32dev", "fp32neq"])
def test_cavity_256_full_size(sd, cavity_256_oracle, prec):
    """The 256 x 256 tanh cavity at Re 1000 on the structured step from a
    generic state, in each precision form (the FP64 and FP32
    non-equilibrium forms are the ones the bench times on the structured
    step at this size): 40 steps against the oracle, with the FP64 bar and
    the FP32 window bars."""
    mesh, bcs, kw, (f, W), (fo, Wo, _) = cavity_256_oracle
    p = {"f64": sd.FP64, "fp32dev": sd.FP32DEV, "fp32neq": sd.FP32NEQ}[prec]
    g = sd.Solver(mesh, bcs, structured=2, precision=p, **kw)
    g.set_state(f, W)
    g.step(40)
    fg, Wg, _ = g.state()
    g.close()
    ef, er = rel_linf(fg, fo), rel_linf(Wg[:, 0], Wo[:, 0])
    em = rel_linf(Wg[:, 1:], Wo[:, 1:])
    say("cavity256 structured", prec, f"f {ef:.2e} rho {er:.2e} mom {em:.2e}")
    if prec == "f64":
        assert ef <= TOL and er <= TOL and em <= TOL
    else:
        em = np.abs(Wg[:, 1:] - Wo[:, 1:]).max() / max(np.abs(Wo[:, 1:]).max(), 0.1)
        assert ef <= 2e-6 and er <= 2e-6 and em <= 2e-6

"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test names the passage of Zhong et al. (arXiv:2007.07347) it follows and
is chosen so that a plausible slip in the oracle (a dropped term, a wrong
sign or index, a swapped operand) fails it.  None of these tests compares the
oracle with itself or with the HIP path.
"""
import math

import numpy as np
import pytest

import meshgen

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)


# ---------------------------------------------------------------- equilibrium
def test_feq_rest_state_is_lattice_weights(oracle_mod):
    """At rest the discrete equilibrium is rho times the D2Q9 weights."""
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    np.testing.assert_array_equal(oracle_mod.feq(1.0, 0.0, 0.0), w)
    np.testing.assert_allclose(oracle_mod.feq(2.5, 0.0, 0.0), 2.5 * w, rtol=0, atol=4e-16)


def test_feq_moments(oracle_mod):
    """Eq. Macro applied to the equilibrium: mass, momentum and the isothermal
    momentum flux rho (c_s^2 I + u u) with c_s^2 = 1/3, exactly (to rounding)."""
    rng = np.random.default_rng(1)
    for _ in range(200):
        rho = rng.uniform(0.5, 2.0)
        ux, uy = rng.uniform(-0.3, 0.3, size=2)
        fe = oracle_mod.feq(rho, ux, uy)
        tol = 8 * np.finfo(float).eps * rho
        assert abs(fe.sum() - rho) <= tol
        assert abs((EX * fe).sum() - rho * ux) <= tol
        assert abs((EY * fe).sum() - rho * uy) <= tol
        assert abs((EX * EX * fe).sum() - rho * (1 / 3 + ux * ux)) <= tol
        assert abs((EX * EY * fe).sum() - rho * ux * uy) <= tol
        assert abs((EY * EY * fe).sum() - rho * (1 / 3 + uy * uy)) <= tol


# ------------------------------------------------------------------- geometry
def test_geometry_cartesian_closed_form(oracle_mod):
    """Centroids, areas and h on a uniform grid; dt = CFL h / sqrt(2)."""
    mesh, bcs = meshgen.couette(4, 32, 0.1)
    o = oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5)
    g = o.geometry()
    h = 1 / 32
    np.testing.assert_allclose(g["area"], h * h, rtol=1e-13)
    i = np.arange(128) % 4
    j = np.arange(128) // 4
    np.testing.assert_allclose(g["cx"], (i + 0.5) * h, rtol=1e-13)
    np.testing.assert_allclose(g["cy"], (j + 0.5) * h, rtol=1e-13)
    np.testing.assert_allclose(g["h"], h, rtol=1e-13)
    assert o.n_faces == 4 * 33 + 32 * 4 and o.n_boundary_faces == 8
    assert abs(o.dt - 0.5 * h / math.sqrt(2)) < 1e-17
    assert o.tau == pytest.approx(0.03, rel=1e-15)


def test_geometry_closes_and_tiles(oracle_mod):
    """On any mesh the scaled outward normals of a cell sum to zero (closed
    polygon) and the areas add up to the domain area."""
    mesh, bcs = meshgen.cylinder_ogrid(40, 20, seed=3)
    o = oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5)
    g = o.geometry()
    fc = o.faces()
    sx = np.zeros(o.n_cells)
    sy = np.zeros(o.n_cells)
    np.add.at(sx, fc["owner"], fc["lnx"])
    np.add.at(sy, fc["owner"], fc["lny"])
    inner = fc["nbr"] >= 0
    np.add.at(sx, fc["nbr"][inner], -fc["lnx"][inner])
    np.add.at(sy, fc["nbr"][inner], -fc["lny"][inner])
    assert np.abs(sx).max() < 1e-13 and np.abs(sy).max() < 1e-13
    # annulus area between the two polygons inscribed in r = 0.5 and r = 20
    n = 40
    poly = lambda r: 0.5 * n * r * r * math.sin(2 * math.pi / n)  # noqa: E731
    assert g["area"].sum() == pytest.approx(poly(20.0) - poly(0.5), rel=1e-12)


# ------------------------------------------------------------ least squares
@pytest.mark.parametrize("which", ["cartesian", "triangles", "ogrid", "hybrid"])
def test_lsq_exact_on_linear_fields(oracle_mod, which):
    """The LLSR normal equations return the exact gradient of a linear field
    alpha + beta . x on every cell (any non-degenerate stencil), with the
    boundary points carrying the field's value at the face midpoints."""
    if which == "cartesian":
        mesh, bcs = meshgen.cavity(12)
    elif which == "triangles":
        mesh, bcs = meshgen.jittered_periodic_triangles(6, seed=2)
    elif which == "hybrid":
        mesh, bcs = meshgen.cylinder_ogrid(24, 10, seed=5, quad_layers=4)
    else:
        mesh, bcs = meshgen.cylinder_ogrid(24, 10, seed=5)
    o = oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5)
    g = o.geometry()
    fc = o.faces()
    beta = np.array([0.7, -1.3])
    fld = 2.0 + beta[0] * g["cx"] + beta[1] * g["cy"]
    bfld = 2.0 + beta[0] * fc["xm"] + beta[1] * fc["ym"]
    if which == "triangles":
        # periodic images carry the partner's value, which a non-periodic linear
        # field does not: check the cells whose stencil does not cross the seam
        keep = (g["cx"] > 0.25) & (g["cx"] < 0.75) & (g["cy"] > 0.25) & (g["cy"] < 0.75)
    else:
        keep = np.ones(o.n_cells, bool)
    for mode in (0, 1):
        gr = o.lsq_gradient(fld, bfld, mode)
        np.testing.assert_allclose(gr[keep], np.broadcast_to(beta, gr[keep].shape), rtol=0, atol=1e-11)
    # without the boundary points the boundary cells would be wrong
    if which != "triangles":
        gr = o.lsq_gradient(fld, np.zeros_like(bfld), 0)
        assert np.abs(gr - beta).max() > 1e-3


def test_lsq_weights_equal_cramer(oracle_mod):
    """Precomputed weights and a fresh Cramer solve give the same gradient."""
    mesh, bcs = meshgen.cylinder_ogrid(24, 10, seed=5)
    o = oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5)
    fld = np.random.default_rng(0).normal(size=o.n_cells)
    bf = np.random.default_rng(1).normal(size=o.n_faces)
    g0, g1 = o.lsq_gradient(fld, bf, 0), o.lsq_gradient(fld, bf, 1)
    np.testing.assert_allclose(g0, g1, rtol=0, atol=1e-9 * np.abs(g1).max())


# ------------------------------------------------------------- face identity
def test_face_mass_flux_identity(oracle_mod):
    """Eq. f_t_n+1 with c1 (1 + b) = 1: the face mass flux sum_i l (e_i.n) f_face
    equals l n . sum_i e_i fbar (the face equilibrium carries the face momentum)."""
    mesh, bcs = meshgen.cylinder_ogrid(24, 10, seed=5)
    o = oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5)
    f, W, G = meshgen.random_state(o.n_cells, seed=4)
    o.set_state(f, W, G)
    fbar, fface, phi = o.face_states()
    fc = o.faces()
    lhs = phi.sum(axis=1)
    rhs = fc["lnx"] * (fbar @ EX) + fc["lny"] * (fbar @ EY)
    scale = np.hypot(fc["lnx"], fc["lny"]) * np.abs(fbar).sum(axis=1)
    assert np.all(np.abs(lhs - rhs) <= 1e-14 * scale)
    # and the momentum flux is not the same identity (the transform is non-trivial)
    assert np.abs(phi @ EX - (fc["lnx"] * (fbar @ (EX * EX)) + fc["lny"] * (fbar @ (EX * EY)))).max() > 1e-8


# --------------------------------------------------- invariants of the step
def _periodic_tri(oracle_mod, **kw):
    mesh, bcs = meshgen.jittered_periodic_triangles(8, seed=7)
    return oracle_mod.Oracle(mesh, bcs, **kw)


def test_uniform_equilibrium_is_fixed_point(oracle_mod):
    """A uniform equilibrium on a periodic jittered triangle mesh stays put:
    fbar+ differences vanish, so the gradient and net fluxes vanish."""
    o = _periodic_tri(oracle_mod, nu=0.01, cfl=0.5, rho0=1.0, u0=0.05, v0=-0.03)
    f0, W0, _ = o.state()
    o.step(1000)
    f1, W1, _ = o.state()
    assert np.abs(f1 - f0).max() <= 1e-13
    assert np.abs(W1 - W0).max() <= 1e-13


@pytest.mark.parametrize("macro", [0, 1])
def test_mass_conserved_on_periodic_domain(oracle_mod, macro):
    """Eq. MacroUpdate telescopes over faces: total mass sum V rho is constant
    to rounding on a closed (periodic) domain, from a generic state."""
    o = _periodic_tri(oracle_mod, nu=0.01, cfl=0.5, macro=macro)
    f, W, G = meshgen.random_state(o.n_cells, seed=11)
    G -= G.mean(axis=0)   # M changes by -dt sum_j G_j: any G with zero sum keeps it closed
    o.set_state(f, W, G)
    m0 = o.mass()
    o.step(2000)
    assert abs(o.mass() - m0) / m0 <= 1e-13


def test_wall_mass_budget(oracle_mod):
    """With walls (non-equilibrium extrapolation is not mass-tight) the mass
    change of one step equals -dt times the boundary-face mass flux."""
    mesh, bcs = meshgen.cavity(10)
    o = oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5, macro=1)
    f, W, G = meshgen.random_state(o.n_cells, seed=12)
    o.set_state(f, W, G)
    fc = o.faces()
    bnd = fc["nbr"] < 0
    for _ in range(5):
        _, _, phi = o.face_states()
        m0 = o.mass()
        o.step(1)
        expect = -o.dt * phi[bnd].sum()
        assert abs((o.mass() - m0) - expect) <= 1e-15 * abs(m0) + 1e-12 * abs(expect)


def test_current_mode_keeps_W_equal_to_moments(oracle_mod):
    """In the same-step (current) mode the psi-moment of Eq. fn+1 gives
    (1 + dt/tau) sum psi f^{n+1} = (1 + dt/tau) W^{n+1}: W stays the moment of f."""
    mesh, bcs = meshgen.cavity(10)
    o = oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5, macro=1)
    f, W, G = meshgen.random_state(o.n_cells, seed=13)
    W = np.c_[f.sum(1), f @ EX, f @ EY]
    o.set_state(f, W, G)
    for _ in range(20):
        o.step(1)
        f, W, _ = o.state()
        mom = np.c_[f.sum(1), f @ EX, f @ EY]
        assert np.abs(mom - W).max() <= 1e-13


# ------------------------------------------------------- assembly / ordering
def _tiny_cases():
    m1, b1 = meshgen.periodic_box(2, 2)
    m2, b2 = meshgen.cavity(3)
    m2 = {k: v for k, v in m2.items()}
    m3, b3 = meshgen.cylinder_ogrid(4, 1, r_far=1.0, seed=9)   # 8 triangles, wall + inlet
    m4, b4 = meshgen.structured(np.linspace(0, 1, 4), np.linspace(0, 1, 5), 0, 1, 2, 3), \
        [meshgen.bc(meshgen.WALL), meshgen.bc(meshgen.OUTLET), meshgen.bc(meshgen.WALL, u=0.1),
         meshgen.bc(meshgen.INLET, u=0.05, v=0.01)]
    m5, b5 = meshgen.split_some(meshgen.cavity(4)[0], 0.5, seed=2), meshgen.cavity(4)[1]   # quads and triangles
    return [(m1, b1), (m2, b2), (m3, b3), (m4, b4), (m5, b5)]


@pytest.mark.parametrize("case", range(5))
def test_brute_force_equals_assembled(oracle_mod, case):
    """Per-face evaluation with a fresh Cramer solve and face-order scatter
    agrees with the assembled per-cell gather over 50 steps."""
    mesh, bcs = _tiny_cases()[case]
    res = []
    for assembly in (0, 1):
        o = oracle_mod.Oracle(mesh, bcs, nu=0.02, cfl=0.5, assembly=assembly)
        f, W, G = meshgen.random_state(o.n_cells, seed=21 + case)
        o.set_state(f, W, G)
        o.step(50)
        res.append(o.state())
    for a, b in zip(res[0], res[1]):
        assert np.abs(a - b).max() <= 1e-14 * max(1.0, np.abs(b).max())


@pytest.mark.parametrize("which", ["cavity", "ogrid", "couette", "hybrid"])
def test_relabel_and_orientation_invariance(oracle_mod, which):
    """Renumbering cells, rotating polygon node lists and flipping boundary
    edges (which changes face owners and normal orientations, including the
    exact ties e_i . n = 0) leaves the solution unchanged after un-permuting."""
    if which == "cavity":
        mesh, bcs = meshgen.cavity(8)
    elif which == "couette":
        mesh, bcs = meshgen.couette(4, 8)
    elif which == "hybrid":
        mesh, bcs = meshgen.cylinder_ogrid(16, 6, seed=1, quad_layers=2)
    else:
        mesh, bcs = meshgen.cylinder_ogrid(16, 6, seed=1)
    mesh2, perm = meshgen.relabel(mesh, seed=5)
    o1 = oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5)
    o2 = oracle_mod.Oracle(mesh2, bcs, nu=0.01, cfl=0.5)
    f, W, G = meshgen.random_state(o1.n_cells, seed=3)
    o1.set_state(f, W, G)
    o2.set_state(f[perm], W[perm], G[perm])
    o1.step(100)
    o2.step(100)
    for a, b in zip(o1.state(), o2.state()):
        assert np.abs(a[perm] - b).max() <= 1e-13 * max(1.0, np.abs(a).max())


def test_mirror_symmetry(oracle_mod):
    """The cavity mirrored about x = 1/2 with the lid velocity negated gives
    the mirrored flow: u(x, y) -> -u(1-x, y), v(x, y) -> v(1-x, y)."""
    n = 10
    mesh, _ = meshgen.cavity(n)
    mm = meshgen.mirror_x(mesh)
    o1 = oracle_mod.Oracle(mesh, [meshgen.bc(meshgen.WALL), meshgen.bc(meshgen.WALL, u=0.1)], nu=0.002, cfl=0.5)
    o2 = oracle_mod.Oracle(mm, [meshgen.bc(meshgen.WALL), meshgen.bc(meshgen.WALL, u=-0.1)], nu=0.002, cfl=0.5)
    o1.step(300)
    o2.step(300)
    r1, u1, v1 = o1.macros()
    r2, u2, v2 = o2.macros()
    # mirror_x keeps cell ids: cell c of the mirrored mesh is the image of cell c
    assert np.abs(r1 - r2).max() <= 1e-13
    assert np.abs(u1 + u2).max() <= 1e-13
    assert np.abs(v1 - v2).max() <= 1e-13
    assert np.abs(u1).max() > 1e-3          # the flow is not trivially zero


def test_quarter_turn_symmetry(oracle_mod):
    """The cavity turned a quarter turn about the origin, with the lid velocity
    turned alike, gives the turned flow: (u, v) -> (-v, u) in every cell.  The
    D2Q9 set maps onto itself under the turn, so a mix-up of the x and y
    lattice components anywhere (a transposed operand, a swapped row) breaks
    this while the mirror test above still holds."""
    n = 10
    mesh, bcs = meshgen.cavity(n)
    # the turn done exactly, (x, y) -> (-y, x): a turn through cos and sin
    # leaves faces tilted by 1e-17, and velocities that lie exactly along a
    # face (the averaged upwind tie) would then pick one side
    rm = dict(mesh)
    rm["node_xy"] = np.ascontiguousarray(np.stack([-mesh["node_xy"][:, 1], mesh["node_xy"][:, 0]], axis=1))
    rb = [meshgen.bc(meshgen.WALL), meshgen.bc(meshgen.WALL, u=0.0, v=0.1)]
    o1 = oracle_mod.Oracle(mesh, bcs, nu=0.002, cfl=0.5)
    o2 = oracle_mod.Oracle(rm, rb, nu=0.002, cfl=0.5)
    assert o2.dt == pytest.approx(o1.dt, rel=1e-14)
    o1.step(300)
    o2.step(300)
    r1, u1, v1 = o1.macros()
    r2, u2, v2 = o2.macros()
    # rotate keeps cell ids: cell c of the turned mesh is the image of cell c
    assert np.abs(r1 - r2).max() <= 1e-13
    assert np.abs(u2 + v1).max() <= 1e-13
    assert np.abs(v2 - u1).max() <= 1e-13
    assert np.abs(v1).max() > 1e-3          # both components are exercised


# --------------------------------------------------------------- physics
@pytest.mark.parametrize("ny", [8, 16])
def test_couette_steady_profile_is_linear(oracle_mod, ny):
    """Couette flow (paper, Couette case): the steady solution is u = U y / H,
    v = 0.  With the boundary value carried to the foot point the discrete
    steady state reproduces the linear profile to rounding."""
    mesh, bcs = meshgen.couette(4, ny, 0.1)
    o = oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5)
    y = o.geometry()["cy"]
    eps, steps = 1.0, 0
    while eps > 1e-12 and steps < 40000:
        o.step(1000)
        steps += 1000
        eps = o.residual()
    assert eps <= 1e-12
    rho, u, v = o.macros()
    assert np.abs(u - 0.1 * y).max() <= 1e-12
    assert np.abs(v).max() <= 1e-13
    assert np.abs(rho - 1.0).max() <= 1e-12


def _couette_series(y, t, U=0.1, nu=0.01, H=1.0, terms=400):
    s = U * y / H
    for m in range(1, terms):
        s = s + 2 * U / (m * math.pi) * (-1) ** m * np.sin(m * math.pi * y / H) * math.exp(-(m * math.pi) ** 2 * nu * t / H ** 2)
    return s


def test_couette_startup_series(oracle_mod):
    """Impulsively started Couette flow (4 x 32, Re = 10, CFL 0.5, 5000 steps)
    against the Fourier series of the diffusion equation: the transient decays
    at rate nu (m pi / H)^2, so a wrong tau or dt shows up."""
    mesh, bcs = meshgen.couette(4, 32, 0.1)
    o = oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5)
    y = o.geometry()["cy"]
    err = []
    for n in (1000, 4000):
        o.step(n - (1000 if n == 4000 else 0))
        _, u, _ = o.macros()
        err.append(np.abs(u - _couette_series(y, n * o.dt)).max() / 0.1)
    assert err[0] < 3e-3 and err[1] < 3e-4
    # x-invariance: the four cells of each row agree
    _, u, _ = o.macros()
    assert np.abs(u.reshape(32, 4) - u.reshape(32, 4)[:, :1]).max() <= 1e-15


def test_shear_wave_decay_rate(oracle_mod):
    """Doubly periodic shear wave u = U0 sin(2 pi y): the amplitude decays at
    nu k^2 only if tau = nu / c_s^2 (a relation tau = nu would be off 3x)."""
    n, nu = 64, 0.0025
    mesh, bcs = meshgen.periodic_box(n, n)
    o = oracle_mod.Oracle(mesh, bcs, nu=nu, cfl=0.5)
    y = o.geometry()["cy"]
    s = np.sin(2 * np.pi * y)
    u = 0.01 * s
    f = np.array([oracle_mod.feq(1.0, uu, 0.0) for uu in u])
    o.set_state(f, np.c_[np.ones(n * n), u, np.zeros(n * n)])
    k2 = (2 * np.pi) ** 2
    T = 1.0 / (nu * k2)
    amp = lambda: np.dot(o.macros()[1], s) / np.dot(s, s)  # noqa: E731
    n1 = int(0.2 * T / o.dt)
    o.step(n1)
    a1 = amp()
    n2 = int(0.6 * T / o.dt)
    o.step(n2 - n1)
    a2 = amp()
    rate = -math.log(a2 / a1) / ((n2 - n1) * o.dt)
    assert abs(rate / (nu * k2) - 1.0) < 2e-3


def test_residual_definition(oracle_mod):
    """The convergence residual (paper, cavity case): relative L2 change of
    (U, V) since the last check; infinite while the snapshot is at rest."""
    mesh, bcs = meshgen.cavity(6)
    o = oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5)
    o.step(10)
    assert o.residual() == math.inf          # snapshot was the rest state
    _, W0, _ = o.state()
    o.step(7)
    _, W1, _ = o.state()
    U0, V0 = W0[:, 1] / W0[:, 0], W0[:, 2] / W0[:, 0]
    U1, V1 = W1[:, 1] / W1[:, 0], W1[:, 2] / W1[:, 0]
    want = math.sqrt(((U1 - U0) ** 2 + (V1 - V0) ** 2).sum() / (U0 ** 2 + V0 ** 2).sum())
    assert o.residual() == pytest.approx(want, rel=1e-12)
    assert o.residual() == 0.0


def _quarter_turn(mesh, bcs):
    """(x, y) -> (-y, x) exactly, wall velocities alike (a turn through
    trigonometric factors would leave faces that are parallel to x or y
    slightly tilted, and the step treats a velocity exactly tangent to a face
    differently from one that crosses it by a hair)."""
    m = dict(mesh)
    xy = mesh["node_xy"]
    m["node_xy"] = np.ascontiguousarray(np.stack([-xy[:, 1], xy[:, 0]], axis=1))
    b = [dict(x) for x in bcs]
    for x in b:
        x["u"], x["v"] = -x["v"], x["u"]
    return m, b


def test_residual_is_rotation_invariant(oracle_mod):
    """The residual sums |u - u_snap|^2 over both velocity components: on the
    cavity turned by a quarter turn (the lid then moves along y, and the flow
    is the turned flow, since the lattice is invariant under quarter turns)
    every residual of the run is the same.  A residual that dropped or
    mis-weighted one component would differ between the two."""
    mesh, bcs = meshgen.cavity(6)
    runs = []
    for m, b in ((mesh, bcs), _quarter_turn(mesh, bcs)):
        o = oracle_mod.Oracle(m, b, nu=0.01, cfl=0.5)
        o.step(10)
        o.residual()
        eps = []
        for k in range(3):
            o.step(5 + k)
            eps.append(o.residual())
        runs.append(eps)
    assert all(0.0 < e < math.inf for e in runs[0])
    assert runs[1] == pytest.approx(runs[0], rel=1e-12)


def test_residual_of_a_state_that_does_not_change(oracle_mod):
    """A uniform equilibrium moving through a doubly periodic box is a fixed
    point of the step: its residual stays at rounding level (against the
    snapshot taken when the state was set, then against the last check),
    while the velocity it is divided by is 0.05."""
    mesh, bcs = meshgen.periodic_box(5, 4)
    o = oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5, rho0=1.0, u0=0.05, v0=-0.02)
    o.step(3)
    assert o.residual() < 1e-14
    o.step(4)
    assert o.residual() < 1e-14


def test_lagged_and_current_share_the_steady_state(oracle_mod):
    """Both readings of the macroscopic-flux time level have the same fixed
    point equations (G* = 0 per cell, f* = feq(W*) - (tau/V) F*), which fix the
    state up to its mass level (the step is homogeneous of degree one in (f, W)
    and the non-equilibrium-extrapolation walls leak mass during the transient
    at a rate that differs between the two).  Run a small cavity to steady
    state both ways (dt < tau, where the lagged form is stable) and compare the
    velocities and the density relative to the total mass."""
    mesh, bcs = meshgen.cavity(8)
    res = []
    for macro in (0, 1):
        o = oracle_mod.Oracle(mesh, bcs, nu=0.02, cfl=0.5, macro=macro)
        assert o.dt < o.tau
        eps, steps = 1.0, 0
        while eps > 1e-12 and steps < 60000:
            o.step(1000)
            steps += 1000
            eps = o.residual()
        assert eps <= 1e-12
        rho, u, v = o.macros()
        res.append((rho / o.mass(), u, v))
    for a, b in zip(res[0], res[1]):
        assert np.abs(a - b).max() <= 1e-10


# ---- boundary fluxes (wall force, surface pressure)

def test_boundary_flux_couette_wall_stress(oracle_mod):
    """Steady Couette flow: the x-momentum leaving the fluid through each wall
    is the viscous stress rho nu U/H times the wall width (bottom wall dragged
    forward, moving top wall held back), the y-momentum is the pressure
    rho c_s^2 = rho/3 times the width, and no mass crosses a wall."""
    for ny in (8, 16):
        mesh, bcs = meshgen.couette(4, ny)
        o = oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5)
        g = o.geometry()
        n = o.n_cells
        f = np.array([oracle_mod.feq(1.0, 0.1 * y, 0.0) for y in g["cy"]])
        o.set_state(f, np.c_[np.ones(n), 0.1 * g["cy"], np.zeros(n)])
        o.step(3000)
        out, tag = o.boundary_flux()
        width = 4.0 / ny
        shear = 0.01 * 0.1 / 1.0 * width
        for t, sgn in ((0, 1.0), (1, -1.0)):
            s = out[tag == t].sum(0)
            assert abs(s[1] - sgn * shear) <= 1e-12 * shear
            assert abs(s[2] + sgn * width / 3.0) <= 1e-13 * width
            assert abs(s[0]) <= 1e-15
            assert np.allclose(out[tag == t, 3], 1.0, rtol=0, atol=1e-13)


def test_boundary_flux_at_rest_is_pressure_only(oracle_mod):
    """A fluid at rest pushes on every resting wall face with rho/3 times its
    scaled normal and nothing else; over a closed wall (the cylinder) the
    pushes cancel."""
    mesh, bcs = meshgen.cylinder_ogrid(24, 8, seed=1)
    o = oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5)
    n = o.n_cells
    o.set_state(np.tile(oracle_mod.feq(1.3, 0.0, 0.0), (n, 1)), np.tile([1.3, 0.0, 0.0], (n, 1)))
    out, tag = o.boundary_flux()
    fc = o.faces()
    sel = fc["nbr"] < 0
    wall = tag == 0
    lnx, lny = fc["lnx"][sel][wall], fc["lny"][sel][wall]
    assert np.abs(out[wall, 1] - 1.3 / 3 * lnx).max() <= 1e-15
    assert np.abs(out[wall, 2] - 1.3 / 3 * lny).max() <= 1e-15
    assert np.abs(out[wall, 0]).max() <= 1e-16 and np.abs(out[wall, 3] - 1.3).max() <= 1e-15
    assert np.abs(out[wall, 1:3].sum(0)).max() <= 1e-15


def test_boundary_flux_closes_the_momentum_budget(oracle_mod):
    """Interior face fluxes cancel between their two cells, so one step
    changes the total momentum by -dt times the momentum leaving through the
    boundary faces, evaluated on the state the step starts from."""
    for mesh, bcs, kw in ((*meshgen.cavity(10), dict(nu=0.01)),
                          (*meshgen.cylinder_ogrid(24, 8, seed=3), dict(nu=0.004, u0=0.1)),
                          (*meshgen.inlet_outlet_box(8, 6), dict(nu=0.01, u0=0.05))):
        o = oracle_mod.Oracle(mesh, bcs, cfl=0.5, **kw)
        f, W, _ = meshgen.random_state(o.n_cells, seed=21, amp=0.02)
        o.set_state(f, np.c_[f.sum(1), f @ EX, f @ EY])
        area = o.geometry()["area"]
        for _ in range(3):
            out, _ = o.boundary_flux()
            _, W0, _ = o.state()
            o.step(1)
            _, W1, _ = o.state()
            dmom = (area[:, None] * (W1[:, 1:] - W0[:, 1:])).sum(0)
            expect = -o.dt * out[:, 1:3].sum(0)
            scale = np.abs(area[:, None] * W0[:, 1:]).sum()
            assert np.abs(dmom - expect).max() <= 1e-14 * scale


# ---- symmetry boundary

def _couette_free_slip(ny=16):
    """Couette cell with the bottom wall replaced by a symmetry line."""
    mesh, bcs = meshgen.couette(4, ny)
    bcs = [dict(b) for b in bcs]
    bcs[0] = meshgen.bc(meshgen.SYMMETRY)
    return mesh, bcs


def test_symmetry_uniform_parallel_flow_is_fixed_point(oracle_mod):
    """A uniform equilibrium flow along a (slanted) symmetry line is steady:
    the boundary state is the inner state itself."""
    mesh, bcs = _couette_free_slip(8)
    ang = 0.37
    bcs[1] = meshgen.bc(meshgen.WALL, u=0.08)          # top wall moving with the flow
    mesh, bcs = meshgen.rotate(mesh, bcs, ang)
    o = oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5)
    n = o.n_cells
    u, v = 0.08 * math.cos(ang), 0.08 * math.sin(ang)
    f0 = np.tile(oracle_mod.feq(1.1, u, v), (n, 1))
    o.set_state(f0, np.tile([1.1, 1.1 * u, 1.1 * v], (n, 1)))
    o.step(200)
    f, W, _ = o.state()
    assert np.abs(f - f0).max() <= 1e-14


def test_inlet_outlet_uniform_flow_is_fixed_point(oracle_mod):
    """A channel with an inlet at (rho0, U), an outlet and free-slip sides,
    started from the uniform equilibrium of the inlet state, stays there: the
    inlet supplies that state, the outlet carries the inner state out and the
    sides reflect a normal velocity that is zero.  A wrong sign or index in
    either open boundary breaks it."""
    mesh = meshgen.structured(np.linspace(0.0, 1.0, 9), meshgen.tanh_nodes(6, 1.0), tag_bottom=3, tag_right=1,
                              tag_top=4, tag_left=2)
    U = 0.06
    bcs = [meshgen.bc(meshgen.WALL), meshgen.bc(meshgen.OUTLET), meshgen.bc(meshgen.INLET, rho=1.0, u=U, v=0.0),
           meshgen.bc(meshgen.SYMMETRY), meshgen.bc(meshgen.SYMMETRY)]
    o = oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5)
    n = o.n_cells
    f0 = np.tile(oracle_mod.feq(1.0, U, 0.0), (n, 1))
    o.set_state(f0, np.tile([1.0, U, 0.0], (n, 1)))
    o.step(300)
    f, W, _ = o.state()
    assert np.abs(f - f0).max() <= 1e-14
    # the same channel started at rest is driven towards the inlet velocity
    o2 = oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5)
    o2.step(300)
    _, u, _ = o2.macros()
    assert u.min() > 0.0


def test_symmetry_couette_free_slip_moves_with_the_wall(oracle_mod):
    """A moving wall over a free-slip (symmetry) plane drags the whole layer
    to its own velocity: the steady state is u = U everywhere, with no shear
    left on the wall (the diffusive transient decays as exp(-nu (pi/2H)^2 t))."""
    mesh, bcs = _couette_free_slip(16)
    o = oracle_mod.Oracle(mesh, bcs, nu=0.05, cfl=0.5)
    o.step(30000)
    rho, u, v = o.macros()
    assert np.abs(u - 0.1).max() <= 1e-10 and np.abs(v).max() <= 1e-12
    out, tag = o.boundary_flux()
    assert np.abs(out[tag == 1, 1]).sum() <= 1e-12


def test_symmetry_brute_force_equals_assembled(oracle_mod):
    mesh, bcs = meshgen.rotate(*_couette_free_slip(6), 0.9)
    res = []
    for assembly in (0, 1):
        o = oracle_mod.Oracle(mesh, bcs, nu=0.02, cfl=0.5, assembly=assembly)
        f, W, G = meshgen.random_state(o.n_cells, seed=41)
        o.set_state(f, W, G)
        o.step(50)
        res.append(o.state())
    for a, b in zip(res[0], res[1]):
        assert np.abs(a - b).max() <= 1e-14 * max(1.0, np.abs(b).max())


# ---- the original (half-step) scheme, the A/B of the paper's simplification

def test_original_scheme_state_round_trip_and_conservation(oracle_mod):
    """The original scheme keeps ft = f - (dt/2) Omega internally: f survives
    set/get unchanged, and mass is conserved to rounding on a periodic mesh."""
    mesh, bcs = meshgen.jittered_periodic_triangles(10, seed=2)
    o = oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5, scheme=1)
    f, _, _ = meshgen.random_state(o.n_cells, seed=3)
    W = np.c_[f.sum(1), f @ EX, f @ EY]
    o.set_state(f, W)
    f2, W2, _ = o.state()
    assert np.abs(f2 - f).max() <= 1e-15 and np.array_equal(W2, W)
    m0 = o.mass()
    o.step(300)
    assert abs(o.mass() - m0) <= 1e-14 * m0
    # a uniform equilibrium stays put
    n = o.n_cells
    fe = np.tile(oracle_mod.feq(1.05, 0.03, -0.02), (n, 1))
    o.set_state(fe, np.tile([1.05, 1.05 * 0.03, -1.05 * 0.02], (n, 1)))
    o.step(200)
    assert np.abs(o.state()[0] - fe).max() <= 1e-14


def test_original_scheme_couette_and_viscosity(oracle_mod):
    """The original scheme also reproduces steady Couette flow exactly and
    decays a shear wave at nu k^2 (64^2, within 1e-3)."""
    mesh, bcs = meshgen.couette(4, 8)
    o = oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5, scheme=1)
    g = o.geometry()
    n = o.n_cells
    fe = np.array([oracle_mod.feq(1.0, 0.1 * y, 0.0) for y in g["cy"]])
    o.set_state(fe, np.c_[np.ones(n), 0.1 * g["cy"], np.zeros(n)])
    o.step(5000)
    _, u, v = o.macros()
    assert np.abs(u - 0.1 * g["cy"]).max() <= 1e-12 and np.abs(v).max() <= 1e-12
    nb = 64
    mesh, bcs = meshgen.periodic_box(nb, nb)
    o = oracle_mod.Oracle(mesh, bcs, nu=0.0025, cfl=0.5, scheme=1)
    g = o.geometry()
    k = 2 * math.pi
    u = 0.01 * np.sin(k * g["cy"])
    o.set_state(np.array([oracle_mod.feq(1.0, x, 0.0) for x in u]), np.c_[np.ones(nb * nb), u, np.zeros(nb * nb)])
    steps = int(20.0 / o.dt)
    o.step(steps)
    _, uu, _ = o.macros()
    rate = -math.log(2 * np.mean(uu * np.sin(k * g["cy"])) / 0.01) / (steps * o.dt)
    assert abs(rate / (0.0025 * k * k) - 1.0) <= 1e-3


def test_original_scheme_brute_force_equals_assembled(oracle_mod):
    mesh, bcs = _tiny_cases()[3]
    res = []
    for assembly in (0, 1):
        o = oracle_mod.Oracle(mesh, bcs, nu=0.02, cfl=0.5, assembly=assembly, scheme=1)
        f, W, _ = meshgen.random_state(o.n_cells, seed=43)
        o.set_state(f, W)
        o.step(50)
        res.append(o.state())
    for a, b in zip(res[0], res[1]):
        assert np.abs(a - b).max() <= 1e-14 * max(1.0, np.abs(b).max())


def test_original_scheme_has_no_lagged_flux(oracle_mod):
    mesh, bcs = meshgen.cavity(4)
    with pytest.raises(ValueError):
        oracle_mod.Oracle(mesh, bcs, nu=0.01, cfl=0.5, scheme=1, macro=0)


# ---------------------------------------------------------------- threads
@pytest.mark.parametrize("assembly", [0, 1])
def test_oracle_threads_do_not_change_results(oracle_mod, assembly):
    """The oracle's per-cell and per-face loops run on several threads for the
    CPU baseline: every cell and face is computed by the same operations on
    the same operands whatever thread takes it, so 1 and N threads give
    identical bits (cavity with a lid and a periodic jittered triangle mesh,
    from a generic state)."""
    for mesh, bcs, kw in ((*meshgen.cavity(19), dict(nu=1e-3, cfl=0.5)),
                          (*meshgen.jittered_periodic_triangles(9, seed=2), dict(nu=4e-3, cfl=0.5))):
        out = []
        for threads in (1, 4):
            assert oracle_mod.set_threads(threads) == threads
            o = oracle_mod.Oracle(mesh, bcs, assembly=assembly, **kw)
            f, W, G = meshgen.random_state(o.n_cells, seed=11, amp=0.03)
            o.set_state(f, W, 0 * G)
            o.step(25)
            out.append(o.state())
        oracle_mod.set_threads(1)
        for a, b in zip(*out):
            assert np.array_equal(a, b)

"""Flow around a circular cylinder: drag and lift coefficients, surface
pressure coefficient and recirculation length (Section IV, flows around a
circular cylinder).

C_d = F_d / (0.5 rho_inf u_inf^2 d) and C_l = F_l / (0.5 rho_inf u_inf^2 d),
with (F_d, F_l) the force the fluid exerts on the wall: the momentum leaving
the fluid through the wall faces, summed on the GPU by the library's boundary
face fluxes.  C_p = (p - p_inf) / (0.5 rho_inf u_inf^2) on each wall face with
p = rho_f / 3 from the face density.  The recirculation length L is the
distance from the rear of the cylinder to the point of the wake axis where
the streamwise velocity turns positive again; the paper reports L/R.  These
are post-processing steps on the solver's outputs (face fluxes and cell
macros), not part of the time step.
"""
from __future__ import annotations

import math

import numpy as np


def force_coefficients(solver, wall_tag=0, rho_inf=1.0, u_inf=0.1, d=1.0):
    """(C_d, C_l) of the current state; the free stream is along +x."""
    _, s = solver.boundary_flux(wall_tag)
    q = 0.5 * rho_inf * u_inf * u_inf * d
    return s[1] / q, s[2] / q


def wall_faces(mesh, bcs, wall_tag=0):
    """Indices (into the solver's boundary-face order: the non-periodic boundary
    edges in the caller's order) and midpoints of the faces of one tag."""
    from .sdugks import BC_PERIODIC
    tags = np.asarray(mesh["bedge_tag"])
    plain = [e for e in range(len(tags)) if bcs[tags[e]]["type"] != BC_PERIODIC]
    rows = [r for r, e in enumerate(plain) if tags[e] == wall_tag]
    edges = np.asarray(mesh["bedge_nodes"])[[plain[r] for r in rows]]
    xy = np.asarray(mesh["node_xy"])
    mid = 0.5 * (xy[edges[:, 0]] + xy[edges[:, 1]])
    return np.asarray(rows, dtype=np.int64), mid


def pressure_coefficient(solver, mesh, bcs, wall_tag=0, rho_inf=1.0, u_inf=0.1, center=(0.0, 0.0)):
    """(theta, C_p) on the wall faces, theta measured from the rear (+x) axis,
    sorted by theta in [0, 2 pi)."""
    faces, _ = solver.boundary_flux()
    rows, mid = wall_faces(mesh, bcs, wall_tag)
    theta = np.mod(np.arctan2(mid[:, 1] - center[1], mid[:, 0] - center[0]), 2.0 * math.pi)
    cp = (faces[rows, 3] / 3.0 - rho_inf / 3.0) / (0.5 * rho_inf * u_inf * u_inf)
    order = np.argsort(theta)
    return theta[order], cp[order]


def axis_velocity(cx, cy, u, xs, k=8):
    """u at the points (x, 0) by a least-squares plane through the k nearest
    cell centres of each point."""
    out = np.empty(len(xs))
    for j, x in enumerate(xs):
        d2 = (cx - x) ** 2 + cy ** 2
        near = np.argpartition(d2, k)[:k]
        A = np.c_[np.ones(k), cx[near] - x, cy[near]]
        coef, *_ = np.linalg.lstsq(A, u[near], rcond=None)
        out[j] = coef[0]
    return out


def recirculation_length(solver, mesh, bcs, radius=0.5, x_max=15.0, n=3000, **geometry_kw):
    """Length L of the recirculation bubble behind the cylinder (0 when the
    flow does not separate): the point of the wake axis x > radius where the
    reverse flow behind the cylinder ends (u turns non-negative after its last
    negative sample), minus radius."""
    from .sdugks import geometry
    g = geometry(mesh, bcs, **geometry_kw)
    _, u, _ = solver.macros()
    band = np.abs(g["cy"]) < 1.0
    ahead = g["cx"] > radius
    sel = band & ahead
    cx, cy, uu = g["cx"][sel], g["cy"][sel], u[sel]
    xs = radius + (x_max - radius) * (np.arange(1, n + 1) / n) ** 2
    ua = axis_velocity(cx, cy, uu, xs)
    # the reverse flow runs from the rear stagnation point to the
    # reattachment point: the bubble ends after the last negative sample (a
    # sign flicker of the interpolation right at the wall does not end it)
    neg = np.nonzero(ua < 0.0)[0]
    if len(neg) == 0:
        return 0.0
    k = neg[-1] + 1
    if k >= len(xs):
        return float("nan")
    x0, x1, u0, u1 = xs[k - 1], xs[k], ua[k - 1], ua[k]
    return float(x0 - u0 * (x1 - x0) / (u1 - u0) - radius)


def run_steady(sd, mesh, bcs, re, u_inf=0.1, d=1.0, tol=1e-8, interval=1000, max_steps=4_000_000, wall_tag=0,
               **kw):
    """March a cylinder case from the free stream until the velocity residual
    of successive checks falls below tol; returns the solver and a summary."""
    nu = u_inf * d / re
    s = sd.Solver(mesh, bcs, nu=nu, u0=u_inf, **kw)
    steps, eps = 0, math.inf
    while steps < max_steps:
        s.step(interval)
        steps += interval
        eps = s.residual()
        if eps <= tol:
            break
    cd, cl = force_coefficients(s, wall_tag, 1.0, u_inf, d)
    return s, {"Re": re, "steps": steps, "residual": eps, "Cd": cd, "Cl": cl, "dt": s.dt, "tau": s.tau}


def dominant_frequency(t, x):
    """Frequency of the strongest periodic component of the samples x(t)
    (uniform spacing): the peak of the periodogram of the mean-removed,
    Hann-windowed signal, refined by a parabola through the peak and its two
    neighbours (in log power)."""
    t = np.asarray(t, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    dt = t[1] - t[0]
    y = (x - x.mean()) * np.hanning(len(x))
    n = 8 * len(y)                                   # zero padding: finer bins
    p = np.abs(np.fft.rfft(y, n)) ** 2
    k = int(np.argmax(p[1:])) + 1
    if 1 <= k < len(p) - 1:
        a, b, c = np.log(p[k - 1] + 1e-300), np.log(p[k] + 1e-300), np.log(p[k + 1] + 1e-300)
        den = a - 2.0 * b + c
        k = k + (0.5 * (a - c) / den if den != 0.0 else 0.0)
    return k / (n * dt)


def kicked_start(solver, mesh, bcs, u_inf, amp, center=(1.5, 0.0), width=0.5, **geometry_kw):
    """Free stream with a transverse velocity bump amp * u_inf *
    exp(-|x - center|^2 / width) in the near wake, at equilibrium: a seed for
    the shedding instability so that it saturates sooner."""
    from .sdugks import geometry
    g = geometry(mesh, bcs, **geometry_kw)
    n = len(g["cx"])
    v = amp * u_inf * np.exp(-((g["cx"] - center[0]) ** 2 + (g["cy"] - center[1]) ** 2) / width)
    solver.set_macros(np.ones(n), np.full(n, u_inf), v)


def run_shedding(sd, mesh, bcs, re, u_inf=0.1, d=1.0, t_transient=600.0, t_sample=400.0, sample_every=200,
                 wall_tag=0, kick=0.0, **kw):
    """Unsteady case: march from the free stream (with an optional transverse
    kick in the near wake, else shedding starts from the asymmetry of the
    mesh) for t_transient, then sample the force coefficients every
    sample_every steps for t_sample.  Returns the Strouhal number
    St = f d / u_inf of the lift oscillation, the mean drag, the lift and drag
    amplitudes and the samples."""
    nu = u_inf * d / re
    s = sd.Solver(mesh, bcs, nu=nu, u0=u_inf, **kw)
    if kick:
        kicked_start(s, mesh, bcs, u_inf, kick, nu=nu, u0=u_inf, **kw)
    n_tr = int(round(t_transient / s.dt))
    s.step(n_tr)
    n_s = int(round(t_sample / (s.dt * sample_every)))
    ts, cds, cls = [], [], []
    for k in range(n_s):
        s.step(sample_every)
        cd, cl = force_coefficients(s, wall_tag, 1.0, u_inf, d)
        ts.append((n_tr + (k + 1) * sample_every) * s.dt)
        cds.append(cd)
        cls.append(cl)
    ts, cds, cls = np.array(ts), np.array(cds), np.array(cls)
    f = dominant_frequency(ts, cls)
    return s, {"Re": re, "St": f * d / u_inf, "Cd_mean": float(cds.mean()), "Cl_amp": float(0.5 * (cls.max() - cls.min())),
               "Cd_amp": float(0.5 * (cds.max() - cds.min())), "steps": n_tr + n_s * sample_every, "dt": s.dt,
               "t": ts, "Cd": cds, "Cl": cls}

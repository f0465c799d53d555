"""Seeded synthetic inputs shared by the solver library and the CPU oracle.

This module builds raw 2-D meshes (node coordinates, counter-clockwise cell
polygons, tagged boundary edges), boundary-condition tables and seeded
initial states.  It contains none of the scheme's arithmetic: no geometry
(areas, normals, centroids), no equilibrium, no flux.  Both the HIP path and
the oracle derive everything else from these arrays on their own.

Mesh dictionary layout (all numpy, C-contiguous):
  node_xy     float64 [n_nodes, 2]
  cell_ptr    int32   [n_cells + 1]   CSR offsets into cell_nodes
  cell_nodes  int32   [sum deg]       node ids of each polygon, counter-clockwise
  bedge_nodes int32   [n_bedges, 2]   the two end nodes of every boundary edge
  bedge_tag   int32   [n_bedges]      index into the boundary-condition table

Boundary-condition table: a list of dicts
  {"type": WALL|INLET|OUTLET|PERIODIC, "rho", "u", "v", "partner", "shift"}
following the paper's Section on boundary conditions: a wall imposes the
wall velocity with the density of the adjacent cell, an inlet imposes
(rho_inf, u_inf), an outlet copies the adjacent cell, and a periodic tag is
glued to its partner tag by the translation `shift` (this tag's edges plus
`shift` land on the partner's edges).
"""
from __future__ import annotations

import math

import numpy as np

WALL, INLET, OUTLET, PERIODIC, SYMMETRY = 1, 2, 3, 4, 5


def bc(type_, rho=1.0, u=0.0, v=0.0, partner=-1, shift=(0.0, 0.0)):
    return {"type": int(type_), "rho": float(rho), "u": float(u), "v": float(v),
            "partner": int(partner), "shift": (float(shift[0]), float(shift[1]))}


def _pack(node_xy, cells, bedges, tags):
    cell_ptr = np.zeros(len(cells) + 1, dtype=np.int32)
    cell_ptr[1:] = np.cumsum([len(c) for c in cells])
    cell_nodes = np.concatenate([np.asarray(c, dtype=np.int32) for c in cells]) if cells else np.zeros(0, np.int32)
    return {
        "node_xy": np.ascontiguousarray(node_xy, dtype=np.float64),
        "cell_ptr": cell_ptr,
        "cell_nodes": np.ascontiguousarray(cell_nodes, dtype=np.int32),
        "bedge_nodes": np.ascontiguousarray(np.asarray(bedges, dtype=np.int32).reshape(-1, 2)),
        "bedge_tag": np.ascontiguousarray(np.asarray(tags, dtype=np.int32)),
    }


def structured(xs, ys, tag_bottom, tag_right, tag_top, tag_left):
    """Quad mesh on the tensor grid xs x ys (both increasing), vectorised.

    Cell (i, j) has nodes (i,j), (i+1,j), (i+1,j+1), (i,j+1) (counter-clockwise)
    and cell id j*nx + i.  Boundary edges get the four side tags.
    """
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.asarray(ys, dtype=np.float64)
    nx, ny = len(xs) - 1, len(ys) - 1
    X, Y = np.meshgrid(xs, ys)
    node_xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    nid = lambda i, j: j * (nx + 1) + i  # noqa: E731
    I, J = np.meshgrid(np.arange(nx), np.arange(ny))
    I, J = I.ravel(), J.ravel()
    cn = np.stack([nid(I, J), nid(I + 1, J), nid(I + 1, J + 1), nid(I, J + 1)], axis=1).astype(np.int32)
    bedges, tags = [], []
    i = np.arange(nx)
    j = np.arange(ny)
    bedges.append(np.stack([nid(i, 0), nid(i + 1, 0)], 1)); tags.append(np.full(nx, tag_bottom))
    bedges.append(np.stack([nid(nx, j), nid(nx, j + 1)], 1)); tags.append(np.full(ny, tag_right))
    bedges.append(np.stack([nid(i + 1, ny), nid(i, ny)], 1)); tags.append(np.full(nx, tag_top))
    bedges.append(np.stack([nid(0, j + 1), nid(0, j)], 1)); tags.append(np.full(ny, tag_left))
    return {
        "node_xy": np.ascontiguousarray(node_xy),
        "cell_ptr": np.arange(0, 4 * nx * ny + 1, 4, dtype=np.int32),
        "cell_nodes": np.ascontiguousarray(cn.ravel()),
        "bedge_nodes": np.ascontiguousarray(np.concatenate(bedges).astype(np.int32)),
        "bedge_tag": np.ascontiguousarray(np.concatenate(tags).astype(np.int32)),
    }


def couette(nx=4, ny=32, U=0.1, height=1.0):
    """Planar Couette channel (paper, Couette flow case): square cells of side
    height/ny, nx columns, periodic in x, bottom wall at rest, top wall moving
    at (U, 0)."""
    h = height / ny
    width = nx * h
    xs = np.arange(nx + 1) * h
    ys = np.arange(ny + 1) * h
    mesh = structured(xs, ys, tag_bottom=0, tag_right=3, tag_top=1, tag_left=2)
    bcs = [bc(WALL, u=0.0), bc(WALL, u=U),
           bc(PERIODIC, partner=3, shift=(width, 0.0)),
           bc(PERIODIC, partner=2, shift=(-width, 0.0))]
    return mesh, bcs


def tanh_nodes(n, beta=1.5, length=1.0):
    """n+1 nodes on [0, length] clustered toward both ends by a tanh map with
    stretching factor beta."""
    s = np.arange(n + 1, dtype=np.float64) / n
    x = 0.5 * (1.0 + np.tanh(beta * (2.0 * s - 1.0)) / math.tanh(beta))
    x[0], x[-1] = 0.0, 1.0
    return length * x


def cavity(n, beta=1.5, U=0.1, length=1.0):
    """Lid-driven square cavity on an n x n tanh-stretched quad mesh.  Tag 0:
    the three resting walls; tag 1: the lid y = length moving at (U, 0)."""
    xs = tanh_nodes(n, beta, length)
    mesh = structured(xs, xs, tag_bottom=0, tag_right=0, tag_top=1, tag_left=0)
    return mesh, [bc(WALL, u=0.0), bc(WALL, u=U)]


def periodic_box(nx, ny, lx=1.0, ly=1.0):
    """Doubly periodic rectangle of uniform quads (tags: 0 bottom, 1 right,
    2 top, 3 left)."""
    xs = np.linspace(0.0, lx, nx + 1)
    ys = np.linspace(0.0, ly, ny + 1)
    mesh = structured(xs, ys, tag_bottom=0, tag_right=1, tag_top=2, tag_left=3)
    bcs = [bc(PERIODIC, partner=2, shift=(0.0, ly)), bc(PERIODIC, partner=3, shift=(-lx, 0.0)),
           bc(PERIODIC, partner=0, shift=(0.0, -ly)), bc(PERIODIC, partner=1, shift=(lx, 0.0))]
    return mesh, bcs


def _split_quads(quads, coin):
    """Split counter-clockwise quads (a,b,c,d) along a diagonal picked by coin:
    coin 0 -> a-c, coin 1 -> b-d.  Both children stay counter-clockwise."""
    a, b, c, d = quads.T
    t1 = np.where(coin[:, None] == 0, np.stack([a, b, c], 1), np.stack([a, b, d], 1))
    t2 = np.where(coin[:, None] == 0, np.stack([a, c, d], 1), np.stack([b, c, d], 1))
    tris = np.empty((2 * len(quads), 3), dtype=np.int32)
    tris[0::2] = t1
    tris[1::2] = t2
    return tris


def jittered_periodic_triangles(n, seed=0, jitter=0.2, length=1.0):
    """Doubly periodic square of 2 n^2 triangles: interior nodes jittered by
    up to `jitter` of the spacing (seeded), boundary nodes left on the grid so
    the periodic sides still coincide, every quad split on a seeded diagonal."""
    rng = np.random.default_rng(seed)
    xs = np.linspace(0.0, length, n + 1)
    X, Y = np.meshgrid(xs, xs)
    node_xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    h = length / n
    jit = rng.uniform(-jitter, jitter, size=node_xy.shape) * h
    nid = lambda i, j: j * (n + 1) + i  # noqa: E731
    I, J = np.meshgrid(np.arange(n + 1), np.arange(n + 1))
    interior = ((I > 0) & (I < n) & (J > 0) & (J < n)).ravel()
    node_xy[interior] += jit[interior]
    I, J = np.meshgrid(np.arange(n), np.arange(n))
    I, J = I.ravel(), J.ravel()
    quads = np.stack([nid(I, J), nid(I + 1, J), nid(I + 1, J + 1), nid(I, J + 1)], 1).astype(np.int32)
    tris = _split_quads(quads, rng.integers(0, 2, size=len(quads)))
    i = np.arange(n)
    bedges = np.concatenate([np.stack([nid(i, 0), nid(i + 1, 0)], 1), np.stack([nid(n, i), nid(n, i + 1)], 1),
                             np.stack([nid(i + 1, n), nid(i, n)], 1), np.stack([nid(0, i + 1), nid(0, i)], 1)])
    tags = np.concatenate([np.full(n, 0), np.full(n, 1), np.full(n, 2), np.full(n, 3)])
    mesh = {
        "node_xy": np.ascontiguousarray(node_xy),
        "cell_ptr": np.arange(0, 3 * len(tris) + 1, 3, dtype=np.int32),
        "cell_nodes": np.ascontiguousarray(tris.ravel()),
        "bedge_nodes": np.ascontiguousarray(bedges.astype(np.int32)),
        "bedge_tag": np.ascontiguousarray(tags.astype(np.int32)),
    }
    bcs = [bc(PERIODIC, partner=2, shift=(0.0, length)), bc(PERIODIC, partner=3, shift=(-length, 0.0)),
           bc(PERIODIC, partner=0, shift=(0.0, -length)), bc(PERIODIC, partner=1, shift=(length, 0.0))]
    return mesh, bcs


def cylinder_ogrid(n_theta=400, n_r=250, r_wall=0.5, r_far=20.0, jitter=0.1, seed=0, U=0.1, quad_layers=0):
    """Annular O-grid around a circular cylinder of diameter 2*r_wall, split into
    triangles (paper, flow around a circular cylinder, on a synthetic mesh).

    Radii grow geometrically, r_k = r_wall (r_far/r_wall)^(k/n_r); interior
    nodes are jittered radially by U(-jitter, jitter) of the smaller adjacent
    radial spacing and tangentially by U(-jitter, jitter) of r_k * dtheta; each
    quad is split along a seeded diagonal, except those of the first
    quad_layers rings next to the wall (a hybrid mesh: quads in the boundary
    layer, triangles outside, like the paper's cylinder meshes).  Tag 0: the
    cylinder wall (at rest); tag 1: the far-field circle with the free stream
    (1, U, 0).
    """
    rng = np.random.default_rng(seed)
    k = np.arange(n_r + 1, dtype=np.float64)
    r = r_wall * (r_far / r_wall) ** (k / n_r)
    dth = 2.0 * math.pi / n_theta
    th = np.arange(n_theta) * dth
    R, TH = np.meshgrid(r, th, indexing="ij")  # [n_r+1, n_theta]
    dr = np.diff(r)
    dr_loc = np.empty_like(r)
    dr_loc[1:-1] = np.minimum(dr[:-1], dr[1:])
    dr_loc[0], dr_loc[-1] = dr[0], dr[-1]
    jr = rng.uniform(-jitter, jitter, size=R.shape) * dr_loc[:, None]
    jt = rng.uniform(-jitter, jitter, size=R.shape) * (R * dth)
    jr[0], jr[-1], jt[0], jt[-1] = 0.0, 0.0, 0.0, 0.0
    Rj = R + jr
    THj = TH + jt / R
    node_xy = np.stack([(Rj * np.cos(THj)).ravel(), (Rj * np.sin(THj)).ravel()], axis=1)
    nid = lambda kk, m: kk * n_theta + (m % n_theta)  # noqa: E731
    K, M = np.meshgrid(np.arange(n_r), np.arange(n_theta), indexing="ij")
    K, M = K.ravel(), M.ravel()
    quads = np.stack([nid(K, M), nid(K + 1, M), nid(K + 1, M + 1), nid(K, M + 1)], 1).astype(np.int32)
    coin = rng.integers(0, 2, size=len(quads))
    m = np.arange(n_theta)
    bedges = np.concatenate([np.stack([nid(0, m + 1), nid(0, m)], 1), np.stack([nid(n_r, m), nid(n_r, m + 1)], 1)])
    tags = np.concatenate([np.zeros(n_theta), np.ones(n_theta)])
    bcs = [bc(WALL, u=0.0), bc(INLET, rho=1.0, u=U, v=0.0)]
    if quad_layers <= 0:
        tris = _split_quads(quads, coin)
        mesh = {
            "node_xy": np.ascontiguousarray(node_xy),
            "cell_ptr": np.arange(0, 3 * len(tris) + 1, 3, dtype=np.int32),
            "cell_nodes": np.ascontiguousarray(tris.ravel()),
            "bedge_nodes": np.ascontiguousarray(bedges.astype(np.int32)),
            "bedge_tag": np.ascontiguousarray(tags.astype(np.int32)),
        }
        return mesh, bcs
    keep = K < quad_layers
    tris = _split_quads(quads[~keep], coin[~keep])
    cells = [list(q) for q in quads[keep]] + [list(t) for t in tris]
    return _pack(node_xy, cells, bedges, tags), bcs


def split_some(mesh, frac, seed=0):
    """The same mesh with a seeded fraction of its quads each split into two
    triangles along a seeded diagonal (a hybrid quad/triangle mesh); split
    quads are replaced in place by their two triangles, boundary edges are
    unchanged."""
    rng = np.random.default_rng(seed)
    ptr, nodes = mesh["cell_ptr"], mesh["cell_nodes"]
    cells = []
    for c in range(len(ptr) - 1):
        poly = nodes[ptr[c]:ptr[c + 1]]
        if len(poly) == 4 and rng.uniform() < frac:
            t = _split_quads(np.asarray([poly]), rng.integers(0, 2, size=1))
            cells += [list(t[0]), list(t[1])]
        else:
            cells.append(list(poly))
    return _pack(mesh["node_xy"], cells, mesh["bedge_nodes"], mesh["bedge_tag"])


def relabel(mesh, seed):
    """Same mesh with cells in a seeded random order and every polygon's node
    list rotated by a seeded offset (orientation kept counter-clockwise), and
    boundary edges shuffled and reversed at random.  Returns (mesh, perm)
    where new cell c is old cell perm[c]."""
    rng = np.random.default_rng(seed)
    ptr, nodes = mesh["cell_ptr"], mesh["cell_nodes"]
    n = len(ptr) - 1
    perm = rng.permutation(n).astype(np.int64)
    cells = []
    for c in perm:
        poly = nodes[ptr[c]:ptr[c + 1]]
        s = int(rng.integers(0, len(poly)))
        cells.append(np.roll(poly, -s))
    be = mesh["bedge_nodes"].copy()
    flip = rng.integers(0, 2, size=len(be)).astype(bool)
    be[flip] = be[flip][:, ::-1]
    order = rng.permutation(len(be))
    out = _pack(mesh["node_xy"], cells, be[order], mesh["bedge_tag"][order])
    return out, perm


def mirror_x(mesh, x_axis=0.5):
    """Mirror image of a mesh about the vertical line x = x_axis; every polygon
    is reversed so it stays counter-clockwise."""
    xy = mesh["node_xy"].copy()
    xy[:, 0] = 2.0 * x_axis - xy[:, 0]
    ptr, nodes = mesh["cell_ptr"], mesh["cell_nodes"]
    cells = [nodes[ptr[c]:ptr[c + 1]][::-1] for c in range(len(ptr) - 1)]
    return _pack(xy, cells, mesh["bedge_nodes"], mesh["bedge_tag"])


def rotate(mesh, bcs, angle):
    """The mesh rotated by `angle` (radians) about the origin, with the
    boundary table's velocities and periodic shifts rotated alike."""
    c, s = math.cos(angle), math.sin(angle)
    xy = mesh["node_xy"] @ np.array([[c, s], [-s, c]])
    out = dict(mesh)
    out["node_xy"] = np.ascontiguousarray(xy)
    nb = []
    for b in bcs:
        b = dict(b)
        b["u"], b["v"] = c * b["u"] - s * b["v"], s * b["u"] + c * b["v"]
        sx, sy = b["shift"]
        b["shift"] = (c * sx - s * sy, s * sx + c * sy)
        nb.append(b)
    return out, nb


def random_state(n_cells, seed, amp=0.05, rho0=1.0):
    """A seeded, generic (non-equilibrium) state for parity windows:
    f[c, i] = rho0/9 * (1 + amp*U(-1,1)), W[c] = (rho0 (1 + amp U), rho0 amp U, rho0 amp U),
    G[c] = rho0 amp U * 1e-3 (a lagged macroscopic flux).  Any state is a valid
    input to one step of the scheme; this one excites every term."""
    rng = np.random.default_rng(seed)
    f = rho0 / 9.0 * (1.0 + amp * rng.uniform(-1.0, 1.0, size=(n_cells, 9)))
    W = np.empty((n_cells, 3))
    W[:, 0] = rho0 * (1.0 + amp * rng.uniform(-1.0, 1.0, size=n_cells))
    W[:, 1:] = rho0 * amp * rng.uniform(-1.0, 1.0, size=(n_cells, 2))
    G = rho0 * amp * 1e-3 * rng.uniform(-1.0, 1.0, size=(n_cells, 3))
    return np.ascontiguousarray(f), np.ascontiguousarray(W), np.ascontiguousarray(G)


def log_uniform_int(rng, lo, hi, size=None):
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))).astype(np.int64)


def hexagon_strip(nx, ny, lx=1.0, ly=1.0, lid_u=0.1):
    """Structured box whose vertical edges carry a midpoint node, so every
    cell is a hexagon with two collinear faces on each side (six faces per
    cell).  Tags: 0 = resting walls, 1 = lid y = ly moving at (lid_u, 0)."""
    xs = np.linspace(0.0, lx, nx + 1)
    ys = np.linspace(0.0, ly, 2 * ny + 1)          # every other row is a midpoint row
    X, Y = np.meshgrid(xs, ys)
    node_xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    nid = lambda i, j: j * (nx + 1) + i  # noqa: E731
    cells = []
    for j in range(ny):
        for i in range(nx):
            b, m, t = 2 * j, 2 * j + 1, 2 * j + 2
            cells.append([nid(i, b), nid(i + 1, b), nid(i + 1, m), nid(i + 1, t), nid(i, t), nid(i, m)])
    bedges, tags = [], []
    for i in range(nx):
        bedges.append((nid(i, 0), nid(i + 1, 0))); tags.append(0)
        bedges.append((nid(i, 2 * ny), nid(i + 1, 2 * ny))); tags.append(1)
    for j in range(2 * ny):
        bedges.append((nid(0, j), nid(0, j + 1))); tags.append(0)
        bedges.append((nid(nx, j), nid(nx, j + 1))); tags.append(0)
    return _pack(node_xy, cells, bedges, tags), [bc(WALL), bc(WALL, u=lid_u)]


def inlet_outlet_box(nx, ny, u_in=0.05):
    """Channel on [0,1]^2: inlet (rho 1, u_in) on the left, outlet on the right,
    walls at rest below and above (all four boundary types but periodic)."""
    xs = np.linspace(0.0, 1.0, nx + 1)
    ys = tanh_nodes(ny, 1.0)
    mesh = structured(xs, ys, tag_bottom=0, tag_right=1, tag_top=0, tag_left=2)
    return mesh, [bc(WALL), bc(OUTLET), bc(INLET, rho=1.0, u=u_in, v=0.0)]


def serving_trace(seed=7, n_requests=24, rate=20.0, couette_n=(8, 32), cavity_n=(16, 64),
                  cylinder_cells=(1_000, 20_000), re_range=(10.0, 400.0), cylinder_re=(10.0, 40.0)):
    """Seeded finite trace of steady-state solve requests: Poisson arrivals at
    `rate` per second, kinds uniform over Couette (4 x N, N log-uniform),
    lid-driven cavity (N x N tanh mesh, N log-uniform) and cylinder O-grid
    (cells log-uniform, n_theta : n_r = 8 : 5, triangles), Reynolds numbers
    uniform (cylinders kept in the steady range).  Returns a list of dicts
    {rid, arrival, kind, mesh, bcs, params, n_cells}; params hold nu (lid or
    free-stream speed 0.1 over the length scale 1), cfl 0.5 and u0."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(n_requests):
        t += rng.exponential(1.0 / rate)
        kind = ("couette", "cavity", "cylinder")[int(rng.integers(0, 3))]
        if kind == "couette":
            n = int(log_uniform_int(rng, *couette_n))
            re = float(rng.uniform(re_range[0], min(re_range[1], 40.0)))
            mesh, bcs = couette(4, n, U=0.1)
            params = {"nu": 0.1 / re, "cfl": 0.5}
        elif kind == "cavity":
            n = int(log_uniform_int(rng, *cavity_n))
            re = float(rng.uniform(*re_range))
            mesh, bcs = cavity(n, beta=1.5, U=0.1)
            params = {"nu": 0.1 / re, "cfl": 0.5}
        else:
            cells = float(np.exp(rng.uniform(math.log(cylinder_cells[0]), math.log(cylinder_cells[1]))))
            n_r = max(4, int(round(math.sqrt(cells * 5.0 / 16.0))))
            n_theta = max(8, int(round(n_r * 8.0 / 5.0)))
            re = float(rng.uniform(*cylinder_re))
            mesh, bcs = cylinder_ogrid(n_theta, n_r, seed=int(rng.integers(0, 2**31)), U=0.1)
            params = {"nu": 0.1 * 1.0 / re, "cfl": 0.5, "u0": 0.1}
        out.append({"rid": rid, "arrival": t, "kind": kind, "mesh": mesh, "bcs": bcs, "params": params,
                    "n_cells": len(mesh["cell_ptr"]) - 1, "re": re})
    return out

"""Python handle on the FP64 CPU oracle of the sDUGKS step.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark.  The solver package never imports it.

The arithmetic lives in ``sdugks_oracle.c`` (plain C, FP64, no FMA
contraction); this module only builds it with gcc and marshals arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sdugks_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

LAGGED, CURRENT = 0, 1
ASSEMBLED, BRUTE = 0, 1

_lib = None


def build(force=True):
    """Compile the oracle with gcc (-O2, no contraction, no fast-math, OpenMP
    over cells and faces; one thread unless set_threads says otherwise)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-fopenmp", "-Wall", "-Wno-unused-result", SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    lib = C.CDLL(LIB)
    P = C.c_void_p
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [C.c_int, P, C.c_int, P, P, C.c_int, P, P, C.c_int, P, P, P, P, P, C.c_char_p]
    lib.orc_free.argtypes = [P]
    lib.orc_info.argtypes = [P, P, P]
    lib.orc_geometry.argtypes = [P, P, P, P, P]
    lib.orc_faces.argtypes = [P] + [P] * 9
    lib.orc_set_state.argtypes = [P, P, P, P]
    lib.orc_get_state.argtypes = [P, P, P, P]
    lib.orc_step.argtypes = [P, C.c_int]
    lib.orc_residual.argtypes = [P]
    lib.orc_residual.restype = C.c_double
    lib.orc_mass.argtypes = [P]
    lib.orc_mass.restype = C.c_double
    lib.orc_feq.argtypes = [C.c_double, C.c_double, C.c_double, P]
    lib.orc_lsq_gradient.argtypes = [P, P, P, P, C.c_int]
    lib.orc_set_threads.argtypes = [C.c_int]
    lib.orc_max_threads.restype = C.c_int
    lib.orc_set_threads(1)
    lib.orc_face_states.argtypes = [P, P, P, P]
    _lib = lib
    return lib


def set_threads(n):
    """Threads of the oracle's per-cell and per-face loops (results do not
    depend on it); returns the count in effect."""
    lib = _load()
    lib.orc_set_threads(int(n))
    return int(lib.orc_max_threads())


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def feq(rho, ux, uy):
    out = np.zeros(9)
    _load().orc_feq(float(rho), float(ux), float(uy), _p(out))
    return out


class Oracle:
    """One simulated case.  Arrays come back cell-major in the caller's order."""

    def __init__(self, mesh, bcs, nu=0.0, tau=0.0, cfl=0.5, dt=0.0, rho0=1.0, u0=0.0, v0=0.0,
                 macro=CURRENT, assembly=ASSEMBLED, scheme=0):
        lib = _load()
        self._keep = []

        def arr(x, dt_):
            a = np.ascontiguousarray(x, dtype=dt_)
            self._keep.append(a)
            return a

        xy = arr(mesh["node_xy"], np.float64)
        cp = arr(mesh["cell_ptr"], np.int32)
        cn = arr(mesh["cell_nodes"], np.int32)
        be = arr(mesh["bedge_nodes"], np.int32)
        bt = arr(mesh["bedge_tag"], np.int32)
        btype = arr([b["type"] for b in bcs], np.int32)
        bval = arr([[b["rho"], b["u"], b["v"], b["shift"][0], b["shift"][1]] for b in bcs], np.float64)
        bpart = arr([b["partner"] for b in bcs], np.int32)
        prm = arr([nu, tau, cfl, dt, rho0, u0, v0], np.float64)
        iprm = arr([macro, assembly, scheme], np.int32)
        err = C.create_string_buffer(256)
        self.n_cells = len(cp) - 1
        h = lib.orc_create(len(xy), _p(xy), self.n_cells, _p(cp), _p(cn), len(be), _p(be), _p(bt),
                           len(bcs), _p(btype), _p(bval), _p(bpart), _p(prm), _p(iprm), err)
        if not h:
            raise ValueError("oracle: " + err.value.decode())
        self._h = C.c_void_p(h)
        self._lib = lib
        d = np.zeros(7)
        iv = np.zeros(4, dtype=np.int32)
        lib.orc_info(self._h, _p(d), _p(iv))
        self.dt, self.tau, self.h_min, self.a, self.b, self.c1, self.lam = (float(x) for x in d)
        self.n_faces, self.n_boundary_faces, self.n_singular = int(iv[1]), int(iv[2]), int(iv[3])

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.orc_free(self._h)
            self._h = None

    def geometry(self):
        n = self.n_cells
        area, cx, cy, h = (np.zeros(n) for _ in range(4))
        self._lib.orc_geometry(self._h, _p(area), _p(cx), _p(cy), _p(h))
        return {"area": area, "cx": cx, "cy": cy, "h": h}

    def faces(self):
        n = self.n_faces
        ow, nb, bc = (np.zeros(n, np.int32) for _ in range(3))
        fl = [np.zeros(n) for _ in range(6)]
        self._lib.orc_faces(self._h, _p(ow), _p(nb), _p(bc), *[_p(x) for x in fl])
        return {"owner": ow, "nbr": nb, "bc": bc, "lnx": fl[0], "lny": fl[1], "xm": fl[2], "ym": fl[3],
                "tx": fl[4], "ty": fl[5]}

    def set_state(self, f, W, G=None):
        n = self.n_cells
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(n, 9)
        W = np.ascontiguousarray(W, dtype=np.float64).reshape(n, 3)
        G = np.zeros((n, 3)) if G is None else np.ascontiguousarray(G, dtype=np.float64).reshape(n, 3)
        self._lib.orc_set_state(self._h, _p(f), _p(W), _p(G))

    def state(self):
        n = self.n_cells
        f, W, G = np.zeros((n, 9)), np.zeros((n, 3)), np.zeros((n, 3))
        self._lib.orc_get_state(self._h, _p(f), _p(W), _p(G))
        return f, W, G

    def macros(self):
        _, W, _ = self.state()
        return W[:, 0], W[:, 1] / W[:, 0], W[:, 2] / W[:, 0]

    def step(self, n=1):
        self._lib.orc_step(self._h, int(n))

    def residual(self):
        return float(self._lib.orc_residual(self._h))

    def mass(self):
        return float(self._lib.orc_mass(self._h))

    def lsq_gradient(self, field, bfield=None, mode=0):
        """Least-squares gradient of a cell field; bfield[f] is the field's value
        at the midpoint of boundary face f (entries of interior faces unused)."""
        field = np.ascontiguousarray(field, dtype=np.float64)
        bfield = np.zeros(self.n_faces) if bfield is None else np.ascontiguousarray(bfield, dtype=np.float64)
        g = np.zeros((self.n_cells, 2))
        self._lib.orc_lsq_gradient(self._h, _p(field), _p(bfield), _p(g), int(mode))
        return g

    def face_states(self):
        n = self.n_faces
        fbar, fface, phi = np.zeros((n, 9)), np.zeros((n, 9)), np.zeros((n, 9))
        self._lib.orc_face_states(self._h, _p(fbar), _p(fface), _p(phi))
        return fbar, fface, phi

    def boundary_flux(self):
        """Fluxes through the plain (not periodic) boundary faces on the current
        state, one row per face in the caller's order of those boundary edges:
        (mass flux, x-momentum flux, y-momentum flux, face density).  The fluxes
        are the moments (1, e_x, e_y) of l (e_i . n) f_face (Eq. MesoFlux and
        Eq. MacroFlux) with n pointing out of the fluid, so the momentum columns
        are the force the fluid exerts on the boundary; the face density is the
        zeroth moment of the reconstructed fbar (pressure = density / 3)."""
        fc = self.faces()
        fbar, _, phi = self.face_states()
        sel = np.nonzero(fc["nbr"] < 0)[0]
        ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
        ey = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)
        out = np.zeros((len(sel), 4))
        for r, f in enumerate(sel):
            out[r, 0] = sum(phi[f, i] for i in range(9))
            out[r, 1] = sum(ex[i] * phi[f, i] for i in range(9))
            out[r, 2] = sum(ey[i] * phi[f, i] for i in range(9))
            out[r, 3] = sum(fbar[f, i] for i in range(9))
        return out, fc["bc"][sel]

"""Python binding of libsdugks.so (the C ABI in include/sdugks.h).

Argument marshalling only: every step of the scheme runs in the library's HIP
kernels.  PyTorch supplies device memory (the workspace tensor) and the
stream.  Importing this module fails loudly when the library is not built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsdugks.so")

OK, EINVAL, ENOMEM, EHIP, EDIVERGED, ENODEV = 0, -1, -2, -3, -4, -5
BC_WALL, BC_INLET, BC_OUTLET, BC_PERIODIC, BC_SYMMETRY = 1, 2, 3, 4, 5
FP64, FP32DEV, FP32NEQ = 0, 1, 2
MACRO_LAGGED, MACRO_CURRENT = 0, 1
SCHEME_SIMPLIFIED, SCHEME_ORIGINAL = 0, 1

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
                      "(hipcc --offload-arch=gfx950)")


class Mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("node_xy", C.c_void_p), ("n_cells", C.c_int32),
                ("cell_ptr", C.c_void_p), ("cell_nodes", C.c_void_p), ("n_bedges", C.c_int32),
                ("bedge_nodes", C.c_void_p), ("bedge_tag", C.c_void_p)]


class BC(C.Structure):
    _fields_ = [("type", C.c_int32), ("partner", C.c_int32), ("rho", C.c_double), ("u", C.c_double),
                ("v", C.c_double), ("shift_x", C.c_double), ("shift_y", C.c_double)]


class Params(C.Structure):
    _fields_ = [("nu", C.c_double), ("tau", C.c_double), ("cfl", C.c_double), ("dt", C.c_double),
                ("rho0", C.c_double), ("u0", C.c_double), ("v0", C.c_double), ("precision", C.c_int32),
                ("macro_flux", C.c_int32), ("reorder", C.c_int32), ("residual_interval", C.c_int32),
                ("tile_cells", C.c_int32), ("block_threads", C.c_int32), ("scheme", C.c_int32),
                ("structured", C.c_int32)]


_lib = C.CDLL(LIB_PATH)
_P = C.c_void_p
_sig = {
    "sdugks_geometry": [_P, _P, C.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P],
    "sdugks_state_bytes": [_P, _P, C.c_int32, _P, _P],
    "sdugks_tiling": [_P, _P, C.c_int32, _P, _P, _P, _P, _P, _P],
    "sdugks_create": [_P, _P, C.c_int32, _P, _P, _P, C.c_size_t, _P],
    "sdugks_step": [_P, C.c_int64],
    "sdugks_step_eager": [_P, C.c_int64],
    "sdugks_set_macros": [_P, _P, _P, _P],
    "sdugks_macros": [_P, _P, _P, _P],
    "sdugks_get_state": [_P, _P, _P, _P],
    "sdugks_set_state": [_P, _P, _P, _P],
    "sdugks_residual": [_P, _P],
    "sdugks_mass": [_P, _P],
    "sdugks_info": [_P, _P, _P, _P, _P],
    "sdugks_boundary_flux": [_P, C.c_int32, _P, _P, _P],
    "sdugks_step_profiled": [_P, C.c_int64, _P, _P, C.c_int32, _P],
    "sdugks_destroy": [_P],
    "sdugks_last_error": [],
    "sdugks_batch_create": [_P, C.c_int32, _P, _P],
    "sdugks_batch_set_members": [_P, _P, C.c_int32],
    "sdugks_batch_step": [_P, C.c_int64],
    "sdugks_batch_residual": [_P, _P],
    "sdugks_residuals_static": [_P, C.c_int32, _P],
    "sdugks_debug_batch_fail": [_P],
    "sdugks_batch_destroy": [_P],
    "sdugks_debug_poison": [_P, C.c_int32, C.c_int32],
}
for _name, _args in _sig.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = C.c_int
_lib.sdugks_last_error.restype = C.c_char_p

EXPORTED = tuple(_sig)


class SdugksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sdugks error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != OK:
        raise SdugksError(rc, _lib.sdugks_last_error().decode())


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


class _Inputs:
    """Keeps the marshalled numpy arrays alive while the structs point at them."""

    def __init__(self, mesh, bcs, nu=0.0, tau=0.0, cfl=0.5, dt=0.0, rho0=1.0, u0=0.0, v0=0.0,
                 precision=FP64, macro=MACRO_CURRENT, reorder=True, residual_interval=1000, tile_cells=0,
                 block_threads=0, scheme=0, structured=0):
        self.xy = np.ascontiguousarray(mesh["node_xy"], dtype=np.float64)
        self.cp = np.ascontiguousarray(mesh["cell_ptr"], dtype=np.int32)
        self.cn = np.ascontiguousarray(mesh["cell_nodes"], dtype=np.int32)
        self.be = np.ascontiguousarray(mesh["bedge_nodes"], dtype=np.int32)
        self.bt = np.ascontiguousarray(mesh["bedge_tag"], dtype=np.int32)
        self.mesh = Mesh(len(self.xy), _ptr(self.xy), len(self.cp) - 1, _ptr(self.cp), _ptr(self.cn),
                         len(self.bt), _ptr(self.be), _ptr(self.bt))
        self.n_bc = len(bcs)
        self.bcs = (BC * max(1, len(bcs)))()
        for k, b in enumerate(bcs):
            self.bcs[k] = BC(b["type"], b.get("partner", -1), b.get("rho", 1.0), b.get("u", 0.0), b.get("v", 0.0),
                             b.get("shift", (0.0, 0.0))[0], b.get("shift", (0.0, 0.0))[1])
        self.prm = Params(nu, tau, cfl, dt, rho0, u0, v0, precision, macro, 1 if reorder else 0, residual_interval,
                          tile_cells, block_threads, scheme, structured)
        self.n_cells = len(self.cp) - 1

    def args(self):
        return C.byref(self.mesh), self.bcs, self.n_bc, C.byref(self.prm)


def geometry(mesh, bcs, **kw):
    """Host-only mesh build: dt, tau, h_min, n_faces and per-cell area and
    centroid (caller order), and the internal cell order."""
    inp = _Inputs(mesh, bcs, **kw)
    n = inp.n_cells
    dt, tau, hmin = C.c_double(), C.c_double(), C.c_double()
    nf = C.c_int32()
    area, cx, cy = np.zeros(n), np.zeros(n), np.zeros(n)
    perm = np.zeros(n, np.int32)
    _check(_lib.sdugks_geometry(*inp.args(), C.byref(dt), C.byref(tau), C.byref(hmin), C.byref(nf),
                                _ptr(area), _ptr(cx), _ptr(cy), _ptr(perm)))
    return {"dt": dt.value, "tau": tau.value, "h_min": hmin.value, "n_faces": nf.value,
            "area": area, "cx": cx, "cy": cy, "perm": perm}


def tiling(mesh, bcs, **kw):
    """Host-only: tile size, tile count and the largest local / first-ring
    cell counts of the fused step for this mesh (tile size 0: two-kernel
    step), and whether the structured step is used."""
    inp = _Inputs(mesh, bcs, **kw)
    v = [C.c_int32() for _ in range(5)]
    _check(_lib.sdugks_tiling(*inp.args(), *[C.byref(x) for x in v]))
    return {"tile_cells": v[0].value, "n_tiles": v[1].value, "max_local": v[2].value, "max_ring1": v[3].value,
            "structured": bool(v[4].value)}


def state_bytes(mesh, bcs, **kw):
    inp = _Inputs(mesh, bcs, **kw)
    b = C.c_size_t()
    _check(_lib.sdugks_state_bytes(*inp.args(), C.byref(b)))
    return b.value


class Solver:
    """One sDUGKS instance on the current GPU.  Device memory is a torch uint8
    tensor handed to the library as its workspace; work is enqueued on the
    torch stream current at creation (or the one given)."""

    def __init__(self, mesh, bcs, stream=None, **kw):
        import torch
        self._lib = _lib
        self._inp = _Inputs(mesh, bcs, **kw)
        self.n_cells = self._inp.n_cells
        nbytes = state_bytes(mesh, bcs, **kw)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _check(_lib.sdugks_create(*self._inp.args(), C.c_void_p(self.stream.cuda_stream),
                                  C.c_void_p(self.workspace.data_ptr()), C.c_size_t(nbytes), C.byref(h)))
        self._h = h
        dt, tau = C.c_double(), C.c_double()
        _check(_lib.sdugks_info(self._h, C.byref(dt), C.byref(tau), None, None))
        self.dt, self.tau = dt.value, tau.value

    @property
    def handle(self):
        return self._h

    def step(self, n=1):
        _check(_lib.sdugks_step(self._h, int(n)))

    def step_eager(self, n=1):
        """The same steps launched one by one (no graph replay)."""
        _check(_lib.sdugks_step_eager(self._h, int(n)))

    def step_profiled(self, n):
        ms = np.zeros(8)
        names = (C.c_char_p * 8)()
        k = C.c_int32()
        _check(_lib.sdugks_step_profiled(self._h, int(n), _ptr(ms), names, 8, C.byref(k)))
        return {names[j].decode(): float(ms[j]) for j in range(k.value)}

    def macros(self):
        n = self.n_cells
        rho, u, v = np.zeros(n), np.zeros(n), np.zeros(n)
        _check(_lib.sdugks_macros(self._h, _ptr(rho), _ptr(u), _ptr(v)))
        return rho, u, v

    def state(self):
        n = self.n_cells
        f, W, G = np.zeros((n, 9)), np.zeros((n, 3)), np.zeros((n, 3))
        _check(_lib.sdugks_get_state(self._h, _ptr(f), _ptr(W), _ptr(G)))
        return f, W, G

    def set_state(self, f, W, G=None):
        n = self.n_cells
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(n, 9)
        W = np.ascontiguousarray(W, dtype=np.float64).reshape(n, 3)
        G = np.zeros((n, 3)) if G is None else np.ascontiguousarray(G, dtype=np.float64).reshape(n, 3)
        _check(_lib.sdugks_set_state(self._h, _ptr(f), _ptr(W), _ptr(G)))

    def set_macros(self, rho, u, v):
        """Equilibrium state of the given per-cell density and velocity
        (computed on the device)."""
        n = self.n_cells
        arrs = [np.ascontiguousarray(np.broadcast_to(np.asarray(x, dtype=np.float64), (n,))) for x in (rho, u, v)]
        _check(_lib.sdugks_set_macros(self._h, *[_ptr(a) for a in arrs]))

    def residual(self):
        e = C.c_double()
        _check(_lib.sdugks_residual(self._h, C.byref(e)))
        return e.value

    def mass(self):
        m = C.c_double()
        _check(_lib.sdugks_mass(self._h, C.byref(m)))
        return m.value

    def info(self):
        dt, tau, n = C.c_double(), C.c_double(), C.c_int32()
        st = C.c_int64()
        _check(_lib.sdugks_info(self._h, C.byref(dt), C.byref(tau), C.byref(st), C.byref(n)))
        return {"dt": dt.value, "tau": tau.value, "step": st.value, "n_cells": n.value}

    def poison(self, cell, i):
        _check(_lib.sdugks_debug_poison(self._h, int(cell), int(i)))

    def boundary_flux(self, tag=-1):
        """Fluxes through the plain boundary faces on the current state:
        (faces [n][4] = mass flux, x-momentum flux, y-momentum flux, face
        density, in the order of the non-periodic boundary edges; sums [3] of
        the three fluxes over the faces of `tag`, all faces when tag < 0).
        The momentum columns are the force the fluid exerts on the boundary."""
        n = C.c_int32()
        _check(_lib.sdugks_boundary_flux(self._h, int(tag), None, None, C.byref(n)))
        faces = np.zeros((n.value, 4))
        sums = np.zeros(3)
        _check(_lib.sdugks_boundary_flux(self._h, int(tag), faces.ctypes.data if n.value else None,
                                         sums.ctypes.data, None))
        return faces, sums

    def close(self):
        # the library is reached through the object: at interpreter exit the
        # module globals may already be gone when this runs from __del__
        lib = getattr(self, "_lib", None)
        if getattr(self, "_h", None) and lib is not None:
            lib.sdugks_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


class Batch:
    """Many instances advanced together by one launch per step (the members
    stay usable alone).  With no stream given the library makes its own."""

    def __init__(self, members, stream=None):
        self._lib = _lib
        self.members = list(members)
        arr = (C.c_void_p * len(self.members))(*[m.handle for m in self.members])
        self.stream = stream
        b = C.c_void_p()
        _check(_lib.sdugks_batch_create(arr, len(self.members),
                                        C.c_void_p(stream.cuda_stream) if stream is not None else None, C.byref(b)))
        self._b = b

    def _call(self, rc):
        # a failed table rebuild leaves the library's batch without members
        if rc in (ENOMEM, EHIP):
            self.members = []
        _check(rc)

    def set_members(self, members):
        members = list(members)
        arr = (C.c_void_p * len(members))(*[m.handle for m in members])
        self._call(_lib.sdugks_batch_set_members(self._b, arr, len(members)))
        self.members = members

    def step(self, n=1):
        self._call(_lib.sdugks_batch_step(self._b, int(n)))

    def residuals(self):
        """Residual of every member in member order (one launch, one
        synchronisation); NaN for a member whose state is not finite, and
        SdugksError(EDIVERGED) raised after all entries are filled."""
        eps = np.zeros(len(self.members))
        rc = _lib.sdugks_batch_residual(self._b, _ptr(eps) if len(eps) else None)
        if rc == EDIVERGED:
            err = SdugksError(rc, _lib.sdugks_last_error().decode())
            err.residuals = eps
            raise err
        self._call(rc)
        return eps

    def debug_fail_next_build(self):
        _check(_lib.sdugks_debug_batch_fail(self._b))

    def close(self):
        lib = getattr(self, "_lib", None)
        if getattr(self, "_b", None) and lib is not None:
            lib.sdugks_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        self.close()

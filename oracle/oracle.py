"""ctypes wrapper of the FP64 CPU oracle (oracle/st_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg; the product package never imports it.

Arrays follow the oracle's conventions: positions and velocities [np, 3]
float64 (C order), diameters [np] float64, fields [3, nz, ny, nx] float64.
"""
import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_LIB = os.path.join(HERE, "libst_oracle.so")


class _Mesh(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("interp", ctypes.c_int32),
        ("drag", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("L", ctypes.c_double * 3),
        ("rho_f", ctypes.c_double),
        ("mu_f", ctypes.c_double),
        ("g", ctypes.c_double * 3),
        ("rho_p", ctypes.c_double),
        ("parcel_weight", ctypes.c_double),
    ]


@dataclass
class MeshParams:
    """Mesh and material parameters (the oracle's or_mesh)."""
    n: tuple = (32, 32, 32)
    L: tuple = (0.1, 0.1, 0.1)
    rho_f: float = 1.2
    mu_f: float = 1.8e-5
    g: tuple = (0.0, 0.0, -9.81)
    rho_p: float = 1000.0
    parcel_weight: float = 1.0
    interp: int = 0  # 0 trilinear, 1 nearest grid point
    drag: int = 0    # 0 Stokes, 1 Schiller-Naumann

    def to_c(self):
        m = _Mesh()
        m.n[:] = [int(v) for v in self.n]
        m.interp = int(self.interp)
        m.drag = int(self.drag)
        m.L[:] = [float(v) for v in self.L]
        m.rho_f = float(self.rho_f)
        m.mu_f = float(self.mu_f)
        m.g[:] = [float(v) for v in self.g]
        m.rho_p = float(self.rho_p)
        m.parcel_weight = float(self.parcel_weight)
        return m

    @property
    def h(self):
        return np.array(self.L, dtype=np.float64) / np.array(self.n, dtype=np.float64)

    @property
    def field_shape(self):
        return (3, self.n[2], self.n[1], self.n[0])


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_D = ctypes.c_double


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def default_threads():
    """Threads for the particle-parallel drivers: OMP_NUM_THREADS when set,
    else the host's cores, at most 16 (a GPU machine's share of its host)."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return min(16, os.cpu_count() or 1)


class Oracle:
    """Loaded oracle library; every method copies its inputs."""

    def __init__(self, path=DEFAULT_LIB):
        if not os.path.exists(path) and path == DEFAULT_LIB:
            from . import build as _b
            _b.build(out=path)
        lib = ctypes.CDLL(path)
        M = ctypes.POINTER(_Mesh)
        sigs = {
            "or_cells": (None, [M, _I64, _P, _P]),
            "or_interp_many": (None, [M, _P, _I64, _P, _P]),
            "or_interp_transpose": (None, [M, _P, _P, _P]),
            "or_tau": (_D, [M, _D]),
            "or_mass": (_D, [M, _D]),
            "or_drag_factor": (_D, [M, _D, _P]),
            "or_step": (None, [M, _P, _I64, _P, _P, _P, _D, _I32, _P]),
            "or_run": (None, [M, _P, _I64, _P, _P, _P, _D, _I32, _I32, _P]),
            "or_run_rotating": (None, [M, _P, _P, _I64, _P, _P, _P, _D, _I32, _P]),
            "or_adjoint": (ctypes.c_int, [M, _P, _I64, _P, _P, _P, _D, _I32, _P, _P, _P]),
            "or_adjoint_run": (ctypes.c_int, [M, _I32, _P, _I32, _P, _P, _I32, _I64, _P, _P,
                                              _P, _P, _P, _P]),
            "or_run_par": (ctypes.c_int, [M, _P, _I64, _P, _P, _P, _D, _I32, _I32, _P, _I32]),
            "or_adjoint_run_par": (ctypes.c_int, [M, _I32, _P, _I32, _P, _P, _I32, _I64, _P,
                                                  _P, _P, _P, _P, _P, _I32]),
            "or_ec_estimate": (None, [_I64, _I32, _P, _P, _P, _P]),
            "or_hilbert_index": (_I64, [_I32, _P]),
            "or_hilbert_positions": (ctypes.c_int, [_I32, _I64, _I64, _I64, _I64, _P, _P, _P]),
            "or_bounding_boxes": (None, [_I64, _P, _P, _I64, _I64, _I64, _P]),
        }
        for name, (res, args) in sigs.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        self.lib = lib

    # -- pieces -----------------------------------------------------------
    def cells(self, mesh, x):
        x = _f64(x, (-1, 3))
        c = np.zeros(x.shape, dtype=np.int32)
        m = mesh.to_c()
        self.lib.or_cells(ctypes.byref(m), x.shape[0], _ptr(x), _ptr(c))
        return c

    def interp(self, mesh, Uf, x):
        Uf = _f64(Uf, mesh.field_shape)
        x = _f64(x, (-1, 3))
        out = np.zeros_like(x)
        m = mesh.to_c()
        self.lib.or_interp_many(ctypes.byref(m), _ptr(Uf), x.shape[0], _ptr(x), _ptr(out))
        return out

    def interp_transpose(self, mesh, x, a):
        """Ubar = sum over particles of the interpolation transpose of a."""
        x = _f64(x, (-1, 3))
        a = _f64(a, (-1, 3))
        Ubar = np.zeros(mesh.field_shape, dtype=np.float64)
        m = mesh.to_c()
        for p in range(x.shape[0]):
            self.lib.or_interp_transpose(ctypes.byref(m), _ptr(x[p]), _ptr(a[p]), _ptr(Ubar))
        return Ubar

    def tau(self, mesh, d):
        m = mesh.to_c()
        return self.lib.or_tau(ctypes.byref(m), float(d))

    def mass(self, mesh, d):
        m = mesh.to_c()
        return self.lib.or_mass(ctypes.byref(m), float(d))

    def drag_factor(self, mesh, d, slip):
        m = mesh.to_c()
        s = _f64(slip, (3,))
        return self.lib.or_drag_factor(ctypes.byref(m), float(d), _ptr(s))

    # -- time stepping -----------------------------------------------------
    def run(self, mesh, Uf, x, up, d, dt, nsteps, nsub=1, Su_int=None):
        """Returns (x, up, Su_int) after nsteps calls of the step."""
        Uf = _f64(Uf, mesh.field_shape)
        x = _f64(x, (-1, 3)).copy()
        up = _f64(up, (-1, 3)).copy()
        d = _f64(d, (-1,))
        assert x.shape == up.shape and d.shape[0] == x.shape[0]
        S = (np.zeros(mesh.field_shape, dtype=np.float64) if Su_int is None
             else _f64(Su_int, mesh.field_shape).copy())
        m = mesh.to_c()
        self.lib.or_run(ctypes.byref(m), _ptr(Uf), x.shape[0], _ptr(x), _ptr(up),
                        _ptr(d), float(dt), int(nsteps), int(nsub), _ptr(S))
        return x, up, S

    def run_par(self, mesh, Uf, x, up, d, dt, nsteps, nsub=1, Su_int=None, threads=None):
        """run() with the particles split over `threads` threads (all cores by
        default); the per-cell sums are added in a different order."""
        threads = threads or default_threads()
        Uf = _f64(Uf, mesh.field_shape)
        x = _f64(x, (-1, 3)).copy()
        up = _f64(up, (-1, 3)).copy()
        d = _f64(d, (-1,))
        assert x.shape == up.shape and d.shape[0] == x.shape[0]
        S = (np.zeros(mesh.field_shape, dtype=np.float64) if Su_int is None
             else _f64(Su_int, mesh.field_shape).copy())
        m = mesh.to_c()
        rc = self.lib.or_run_par(ctypes.byref(m), _ptr(Uf), x.shape[0], _ptr(x), _ptr(up),
                                 _ptr(d), float(dt), int(nsteps), int(nsub), _ptr(S),
                                 int(threads))
        if rc != 0:
            raise MemoryError("or_run_par could not allocate its per-thread sources")
        return x, up, S

    def run_rotating(self, mesh, U0, cs, x, up, d, dt, nsteps, Su_int=None):
        U0 = _f64(U0, mesh.field_shape)
        cs = _f64(cs, (-1,))
        assert cs.shape[0] >= 2 * nsteps
        x = _f64(x, (-1, 3)).copy()
        up = _f64(up, (-1, 3)).copy()
        d = _f64(d, (-1,))
        S = (np.zeros(mesh.field_shape, dtype=np.float64) if Su_int is None
             else _f64(Su_int, mesh.field_shape).copy())
        m = mesh.to_c()
        self.lib.or_run_rotating(ctypes.byref(m), _ptr(U0), _ptr(cs), x.shape[0], _ptr(x),
                                 _ptr(up), _ptr(d), float(dt), int(nsteps), _ptr(S))
        return x, up, S

    def ec_estimate(self, kind, S_last, state):
        """One extrapolator-corrector call; `state` is a dict with arrays
        'S_prev2' and 'ext_prev' (updated in place).  Returns the source to
        apply."""
        S_last = _f64(S_last)
        for k in ("S_prev2", "ext_prev"):
            assert state[k].dtype == np.float64 and state[k].flags.c_contiguous
            assert state[k].size == S_last.size
        out = np.empty_like(S_last)
        self.lib.or_ec_estimate(S_last.size, int(kind), _ptr(S_last), _ptr(state["S_prev2"]),
                                _ptr(state["ext_prev"]), _ptr(out))
        return out

    def hilbert_index(self, order, xyz):
        c = np.ascontiguousarray(xyz, dtype=np.int32).reshape(3)
        return int(self.lib.or_hilbert_index(int(order), _ptr(c)))

    def hilbert_positions(self, order, nseg, seg_begin, seg_end, per_seg, L, u):
        """Positions [n, 3] of segments [seg_begin, seg_end), per_seg each."""
        n = (seg_end - seg_begin) * per_seg
        u = _f64(u, (n, 3))
        Lc = _f64(L, (3,))
        x = np.zeros((n, 3))
        r = self.lib.or_hilbert_positions(int(order), int(nseg), int(seg_begin), int(seg_end),
                                          int(per_seg), _ptr(Lc), _ptr(u), _ptr(x))
        if r != 0:
            raise ValueError("or_hilbert_positions rejected its arguments")
        return x

    def bounding_boxes(self, x, ids, id0, per_part, nparts):
        """[nparts, 6] boxes (min xyz, max xyz) of the id partitions."""
        x = _f64(x, (-1, 3))
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        box = np.zeros((nparts, 6))
        self.lib.or_bounding_boxes(x.shape[0], _ptr(x), _ptr(ids), int(id0), int(per_part),
                                   int(nparts), _ptr(box))
        return box

    def adjoint(self, mesh, Uf, x0, up0, d, dt, nsteps, lam):
        """Returns (dL/dUf, dL/dd) for dL/dSu_int = lam."""
        Uf = _f64(Uf, mesh.field_shape)
        x0 = _f64(x0, (-1, 3))
        up0 = _f64(up0, (-1, 3))
        d = _f64(d, (-1,))
        lam = _f64(lam, mesh.field_shape)
        Ubar = np.zeros(mesh.field_shape, dtype=np.float64)
        dbar = np.zeros(d.shape[0], dtype=np.float64)
        m = mesh.to_c()
        rc = self.lib.or_adjoint(ctypes.byref(m), _ptr(Uf), x0.shape[0], _ptr(x0), _ptr(up0),
                                 _ptr(d), float(dt), int(nsteps), _ptr(lam), _ptr(Ubar),
                                 _ptr(dbar))
        if rc != 0:
            raise MemoryError("oracle adjoint could not allocate its tape")
        return Ubar, dbar

    def adjoint_run(self, mesh, fields, field_of_step, dt_of_step, nsub, x0, up0, d, lam):
        """Reverse pass of a run whose step n takes nsub sub-steps of
        dt_of_step[n] / nsub with field fields[field_of_step[n]].  Returns
        (dL/d fields [nfields, 3, nz, ny, nx], dL/dd)."""
        F = np.ascontiguousarray(fields, dtype=np.float64).reshape((-1,) + mesh.field_shape)
        fs = np.ascontiguousarray(field_of_step, dtype=np.int32).reshape(-1)
        dts = np.ascontiguousarray(dt_of_step, dtype=np.float64).reshape(-1)
        assert fs.shape == dts.shape
        x0 = _f64(x0, (-1, 3))
        up0 = _f64(up0, (-1, 3))
        d = _f64(d, (-1,))
        lam = _f64(lam, mesh.field_shape)
        Ubar = np.zeros(F.shape, dtype=np.float64)
        dbar = np.zeros(d.shape[0], dtype=np.float64)
        m = mesh.to_c()
        rc = self.lib.or_adjoint_run(ctypes.byref(m), F.shape[0], _ptr(F), fs.shape[0], _ptr(fs),
                                     _ptr(dts), int(nsub), x0.shape[0], _ptr(x0), _ptr(up0),
                                     _ptr(d), _ptr(lam), _ptr(Ubar), _ptr(dbar))
        if rc != 0:
            raise ValueError("oracle adjoint rejected its arguments or could not allocate")
        return Ubar, dbar

    def adjoint_run_par(self, mesh, fields, field_of_step, dt_of_step, nsub, x0, up0, d, lam,
                        threads=None):
        """adjoint_run() with the particles split over `threads` threads."""
        threads = threads or default_threads()
        F = np.ascontiguousarray(fields, dtype=np.float64).reshape((-1,) + mesh.field_shape)
        fs = np.ascontiguousarray(field_of_step, dtype=np.int32).reshape(-1)
        dts = np.ascontiguousarray(dt_of_step, dtype=np.float64).reshape(-1)
        assert fs.shape == dts.shape
        x0 = _f64(x0, (-1, 3))
        up0 = _f64(up0, (-1, 3))
        d = _f64(d, (-1,))
        lam = _f64(lam, mesh.field_shape)
        Ubar = np.zeros(F.shape, dtype=np.float64)
        dbar = np.zeros(d.shape[0], dtype=np.float64)
        m = mesh.to_c()
        rc = self.lib.or_adjoint_run_par(ctypes.byref(m), F.shape[0], _ptr(F), fs.shape[0],
                                         _ptr(fs), _ptr(dts), int(nsub), x0.shape[0], _ptr(x0),
                                         _ptr(up0), _ptr(d), _ptr(lam), _ptr(Ubar), _ptr(dbar),
                                         int(threads))
        if rc != 0:
            raise ValueError("oracle adjoint rejected its arguments or could not allocate")
        return Ubar, dbar


_cache = {}


def load(path=DEFAULT_LIB):
    if path not in _cache:
        _cache[path] = Oracle(path)
    return _cache[path]

"""CPU oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.

A plain FP64 reference of the time step of the 16-velocity third-order
isothermal lattice Boltzmann model with corner transport upwind advection of
Sofonea et al., arXiv:1802.01272 (C source in ``lbm_oracle.c``), plus the
thermodynamic closed forms the tests pin it with (``thermo.py``).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares nothing with the HIP library
in ``paper_1802_01272_amd``.

Field layout: ``f[k, j, i]`` (numpy array of shape (16, Ly, Lx), float64).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class _Params(ctypes.Structure):
    _fields_ = [
        ("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32),
        ("ds", ctypes.c_double), ("dt", ctypes.c_double),
        ("tau", ctypes.c_double), ("T", ctypes.c_double),
        ("a", ctypes.c_double), ("b", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("scheme", ctypes.c_int32), ("regularize", ctypes.c_int32),
        ("bc_y", ctypes.c_int32),
        ("u_wall", ctypes.c_double), ("rho_wall", ctypes.c_double),
        ("limiter", ctypes.c_int32), ("a2_eq", ctypes.c_int32),
        ("clamp_radius", ctypes.c_double), ("clamp_rho", ctypes.c_double),
    ]


@dataclass
class Params:
    """Parameters of one oracle run (names follow the paper)."""
    Lx: int
    Ly: int
    ds: float = 1.0
    dt: float = 0.25
    tau: float = 0.7
    T: float = 0.95
    a: float = 9.0 / 8.0
    b: float = 1.0 / 3.0
    kappa: float = 1.0
    scheme: int = 2
    regularize: int = 0
    bc_y: int = 0
    u_wall: float = 0.0
    rho_wall: float = 1.0
    limiter: int = 1
    a2_eq: int = 0
    clamp_radius: float = 0.0
    clamp_rho: float = 1.0

    def c(self) -> _Params:
        return _Params(self.Lx, self.Ly, self.ds, self.dt, self.tau, self.T,
                       self.a, self.b, self.kappa, self.scheme, self.regularize,
                       self.bc_y, self.u_wall, self.rho_wall, self.limiter,
                       self.a2_eq, self.clamp_radius, self.clamp_rho)


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            _build.build()
        lib = ctypes.CDLL(path)
        D = ctypes.POINTER(ctypes.c_double)
        P = ctypes.POINTER(_Params)
        i32 = ctypes.c_int
        lib.orc_velocity_set.argtypes = [D, D, D]
        lib.orc_feq.argtypes = [ctypes.c_double] * 4 + [D]
        lib.orc_force.argtypes = [ctypes.c_double] * 5 + [D, D]
        lib.orc_moments.argtypes = [D, D, D, D, D]
        lib.orc_pressure_vdw.argtypes = [ctypes.c_double] * 4
        lib.orc_pressure_vdw.restype = ctypes.c_double
        lib.orc_regularize_node.argtypes = [ctypes.c_double, D]
        for name in ("orc_grad5", "orc_grad3"):
            getattr(lib, name).argtypes = [i32, i32, ctypes.c_double, D, D, D]
        lib.orc_lap3.argtypes = [i32, i32, ctypes.c_double, D, D]
        lib.orc_advect.argtypes = [i32, i32] + [ctypes.c_double] * 4 + [i32, i32, D, D]
        lib.orc_init.argtypes = [P, D, D, D, D]
        lib.orc_step.argtypes = [P, D, D]
        lib.orc_step.restype = i32
        lib.orc_run.argtypes = [P, D, ctypes.c_int64]
        lib.orc_run.restype = i32
        lib.orc_step_region.argtypes = [P, D, i32, i32, i32, i32, D]
        lib.orc_step_region.restype = i32
        lib.orc_field_moments.argtypes = [P, D, D, D, D]
        lib.orc_reduce.argtypes = [P, D, ctypes.c_double, D]
        lib.orc_num_threads.restype = i32
        lib.orc_set_num_threads.argtypes = [i32]
        _LIB = lib
    return _LIB


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def velocity_set():
    """(xi_x, xi_y, w), each shape (16,)."""
    xx, xy, w = (np.zeros(16) for _ in range(3))
    _lib().orc_velocity_set(_ptr(xx), _ptr(xy), _ptr(w))
    return xx, xy, w


def feq(T, rho, ux, uy):
    out = np.zeros(16)
    _lib().orc_feq(T, rho, ux, uy, _ptr(out))
    return out


def force(rho, ux, uy, gx, gy, a2):
    out = np.zeros(16)
    a2 = np.ascontiguousarray(a2, dtype=np.float64)
    _lib().orc_force(rho, ux, uy, gx, gy, _ptr(a2), _ptr(out))
    return out


def moments(f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    r, ux, uy = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    a2 = np.zeros(3)
    _lib().orc_moments(_ptr(f), ctypes.byref(r), ctypes.byref(ux), ctypes.byref(uy), _ptr(a2))
    return r.value, ux.value, uy.value, a2


def pressure_vdw(T, a, b, rho):
    return _lib().orc_pressure_vdw(T, a, b, rho)


def regularize_node(T, f):
    f = np.array(f, dtype=np.float64)
    _lib().orc_regularize_node(T, _ptr(f))
    return f


def regularize_field(T, f):
    """Apply the regularized replacement to every node of a (16, Ly, Lx) field."""
    out = np.array(f, dtype=np.float64)
    _, Ly, Lx = out.shape
    for j in range(Ly):
        for i in range(Lx):
            out[:, j, i] = regularize_node(T, out[:, j, i])
    return out


def _stencil(name, field, ds, nout):
    field = np.ascontiguousarray(field, dtype=np.float64)
    Ly, Lx = field.shape
    outs = [np.zeros_like(field) for _ in range(nout)]
    getattr(_lib(), name)(Lx, Ly, ds, _ptr(field), *[_ptr(o) for o in outs])
    return outs if nout > 1 else outs[0]


def grad5(field, ds=1.0):
    return _stencil("orc_grad5", field, ds, 2)


def grad3(field, ds=1.0):
    return _stencil("orc_grad3", field, ds, 2)


def lap3(field, ds=1.0):
    return _stencil("orc_lap3", field, ds, 1)


def advect(field, cx, cy, ds=1.0, dt=0.25, scheme=2, limiter=1):
    field = np.ascontiguousarray(field, dtype=np.float64)
    Ly, Lx = field.shape
    out = np.zeros_like(field)
    _lib().orc_advect(Lx, Ly, ds, dt, cx, cy, scheme, limiter, _ptr(field), _ptr(out))
    return out


def init(p: Params, rho, ux, uy):
    rho, ux, uy = (np.ascontiguousarray(x, dtype=np.float64) for x in (rho, ux, uy))
    f = np.zeros((16, p.Ly, p.Lx))
    cp = p.c()
    _lib().orc_init(ctypes.byref(cp), _ptr(rho), _ptr(ux), _ptr(uy), _ptr(f))
    return f


def step(p: Params, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    cp = p.c()
    if _lib().orc_step(ctypes.byref(cp), _ptr(f), _ptr(out)) != 0:
        raise ValueError("oracle step rejected its parameters")
    return out


def run(p: Params, f, nsteps):
    f = np.array(f, dtype=np.float64, order="C")
    cp = p.c()
    if _lib().orc_run(ctypes.byref(cp), _ptr(f), int(nsteps)) != 0:
        raise ValueError("oracle run failed")
    return f


def step_region(p: Params, f, i0, i1, j0, j1):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros((16, j1 - j0, i1 - i0))
    cp = p.c()
    if _lib().orc_step_region(ctypes.byref(cp), _ptr(f), i0, i1, j0, j1, _ptr(out)) != 0:
        raise ValueError("oracle step_region rejected its arguments")
    return out


def field_moments(p: Params, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    rho, ux, uy = (np.zeros((p.Ly, p.Lx)) for _ in range(3))
    cp = p.c()
    _lib().orc_field_moments(ctypes.byref(cp), _ptr(f), _ptr(rho), _ptr(ux), _ptr(uy))
    return rho, ux, uy


STAT_NAMES = ("mass", "mom_x", "mom_y", "n_bubble", "n_nonfinite",
              "sx", "sy", "sxx", "sxy", "syy")


def reduce(p: Params, f, threshold):
    f = np.ascontiguousarray(f, dtype=np.float64)
    st = np.zeros(11)
    cp = p.c()
    _lib().orc_reduce(ctypes.byref(cp), _ptr(f), threshold, _ptr(st))
    return dict(zip(STAT_NAMES, st[:10]))


def num_threads() -> int:
    return _lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    _lib().orc_set_num_threads(int(n))

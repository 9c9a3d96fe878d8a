"""Python binding of the C ABI in include/lbm.h (argument marshalling only).

Every computation runs in the HIP library ``_lib/liblbm.so``; this module only
converts arguments.  PyTorch supplies the device workspace (a uint8 CUDA
tensor owned by the Python object) and the stream (torch's current stream).
Importing this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, fields
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ECFL, LBM_ENOMEM, LBM_EDEVICE, LBM_ENONFINITE, LBM_ESTATE = 0, -1, -2, -3, -4, -5, -6
FP64, FP32_DEV = 0, 1
PERIODIC, SHEAR_WALLS = 0, 1
ROUND_STOCHASTIC, ROUND_NEAREST = 0, 1
PAIR = 0  # waves_per_group of a launch shape: two wavefronts per strip (FP32 storage)
BATCH_PER_STEP, BATCH_PERSISTENT = 0, 1  # lbm_batch_set_mode


class LbmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("lbm status %d: %s" % (status, message))
        self.status = status


class CParams(ctypes.Structure):
    _fields_ = [
        ("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32),
        ("ds", ctypes.c_double), ("dt", ctypes.c_double),
        ("tau", ctypes.c_double), ("T", ctypes.c_double),
        ("a", ctypes.c_double), ("b", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("scheme", ctypes.c_int32), ("regularize", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("rho_ref", ctypes.c_double),
        ("bc_y", ctypes.c_int32),
        ("u_wall", ctypes.c_double), ("rho_wall", ctypes.c_double),
        ("clamp_radius", ctypes.c_double), ("clamp_rho", ctypes.c_double),
        ("rounding", ctypes.c_int32),
    ]


class CStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("mass", "mom_x", "mom_y")] + [
        ("n_bubble", ctypes.c_int64), ("n_nonfinite", ctypes.c_int64)] + [
        (n, ctypes.c_double) for n in ("sx", "sy", "sxx", "sxy", "syy", "cx", "cy", "Txx", "Txy", "Tyy",
                                       "a", "b", "D", "theta", "A_rel", "R_eq")]


@dataclass
class Params:
    """Parameters of one run; names and meaning as in include/lbm.h."""
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
    precision: int = FP64
    rho_ref: float = 1.0
    bc_y: int = PERIODIC
    u_wall: float = 0.0
    rho_wall: float = 1.0
    clamp_radius: float = 0.0
    clamp_rho: float = 1.0
    rounding: int = ROUND_STOCHASTIC

    def c(self) -> CParams:
        return CParams(*[getattr(self, f.name) for f in fields(self)])

    @classmethod
    def from_workload(cls, w, precision: int = FP64, **kw) -> "Params":
        p = cls(Lx=w.Lx, Ly=w.Ly, ds=w.ds, dt=w.dt, tau=w.tau, T=w.T, a=w.a, b=w.b, kappa=w.kappa,
                scheme=w.scheme, regularize=w.regularize, precision=precision, rho_ref=w.rho_ref,
                bc_y=w.bc_y, u_wall=w.u_wall, rho_wall=w.rho_wall)
        for k, v in kw.items():
            setattr(p, k, v)
        return p


def _load():
    # torch's bundled HIP runtime carries the same soname (libamdhip64.so.7) as
    # the one the library links against; loading torch first makes the library
    # bind to that runtime, so torch's memory and streams and the library's
    # kernels share one HIP runtime in the process.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError("HIP library %s is missing: run `python -c 'import __graft_entry__ as g; g.build()'`"
                          % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(CParams)
    vp = ctypes.c_void_p
    D = ctypes.POINTER(ctypes.c_double)
    st = ctypes.c_int
    sig = {
        "lbm_version": ([], ctypes.c_char_p),
        "lbm_last_error": ([], ctypes.c_char_p),
        "lbm_validate": ([P], st),
        "lbm_workspace_bytes": ([P], ctypes.c_size_t),
        "lbm_init": ([P, vp, ctypes.c_size_t, vp, D, D, D, ctypes.POINTER(vp)], st),
        "lbm_init_device": ([P, vp, ctypes.c_size_t, vp, vp, vp, vp, ctypes.POINTER(vp)], st),
        "lbm_attach": ([P, vp, ctypes.c_size_t, ctypes.c_int64, ctypes.POINTER(vp)], st),
        "lbm_step": ([vp, ctypes.c_int64, vp], st),
        "lbm_step_timed": ([vp, ctypes.c_int64, vp, D], st),
        "lbm_step_count": ([vp], ctypes.c_int64),
        "lbm_moments": ([vp, D, D, D, vp], st),
        "lbm_moments_device": ([vp, vp, vp, vp, vp], st),
        "lbm_get_f": ([vp, D, vp], st),
        "lbm_set_f": ([vp, D, vp], st),
        "lbm_get_f_device": ([vp, vp, vp], st),
        "lbm_set_f_device": ([vp, vp, vp], st),
        "lbm_reduce": ([vp, ctypes.c_double, ctypes.POINTER(CStats), vp], st),
        "lbm_state_device": ([vp, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int64)], st),
        "lbm_reduce_field_static": ([P, vp, ctypes.c_double, ctypes.POINTER(CStats), vp], st),
        "lbm_set_launch": ([vp, ctypes.c_int32, ctypes.c_int32], st),
        "lbm_get_launch": ([vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)], st),
        "lbm_autotune": ([P, vp, ctypes.c_size_t, vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                          ctypes.POINTER(ctypes.c_int32)], st),
        "lbm_destroy": ([vp], None),
        "lbm_batch_workspace_bytes": ([ctypes.c_int32, P], ctypes.c_size_t),
        "lbm_batch_init": ([ctypes.c_int32, P, vp, ctypes.c_size_t, vp, ctypes.POINTER(D), ctypes.POINTER(D),
                            ctypes.POINTER(D), ctypes.POINTER(vp)], st),
        "lbm_batch_step": ([vp, ctypes.c_int64, ctypes.c_int32, vp], st),
        "lbm_batch_set_launch": ([vp, ctypes.c_int32, vp], st),
        "lbm_batch_autotune": ([vp, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_int32)], st),
        "lbm_batch_run": ([vp, ctypes.c_int32], vp),
        "lbm_init_batch": ([ctypes.c_int32, P, vp, ctypes.c_size_t, vp, ctypes.POINTER(D), ctypes.POINTER(D),
                            ctypes.POINTER(D), ctypes.POINTER(vp)], st),
        "lbm_step_batch": ([vp, ctypes.c_int64, vp], st),
        "lbm_batch_set_mode": ([vp, ctypes.c_int32, vp], st),
        "lbm_batch_get_mode": ([vp], ctypes.c_int32),
        "lbm_batch_set_wait_limit": ([vp, ctypes.c_uint32, vp], st),
        "lbm_batch_sync_status": ([vp, vp], st),
        "lbm_batch_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


LIB = _load()


def _check(status: int):
    if status != LBM_OK:
        raise LbmError(status, LIB.lbm_last_error().decode())


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def version() -> str:
    return LIB.lbm_version().decode()


def validate(p: Params) -> int:
    """Host-only parameter check; returns the lbm_status code."""
    cp = p.c()
    return LIB.lbm_validate(ctypes.byref(cp))


def workspace_bytes(p: Params) -> int:
    cp = p.c()
    return int(LIB.lbm_workspace_bytes(ctypes.byref(cp)))


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the lattice Boltzmann library runs on the device only")
    return torch


def _stream_handle(torch, stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _workspace(torch, nbytes: int):
    # torch's caching allocator returns blocks aligned to at least 512 bytes
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")
    assert ws.data_ptr() % 256 == 0
    return ws


_STAT_NAMES = [f[0] for f in CStats._fields_]


def _stats_dict(cs: CStats) -> Dict[str, float]:
    return {n: getattr(cs, n) for n in _STAT_NAMES}


class Run:
    """One run of the stepper with its device workspace."""

    def __init__(self, p: Params, rho0: np.ndarray, ux0: np.ndarray, uy0: np.ndarray, stream=None,
                 workspace=None, _attach_step: Optional[int] = None):
        torch = _torch()
        self.torch = torch
        self.p = p
        self._cp = p.c()
        n = workspace_bytes(p)
        if n == 0:
            _check(validate(p))
        self.ws = workspace if workspace is not None else _workspace(torch, n)
        self.handle = ctypes.c_void_p()
        s = _stream_handle(torch, stream)
        if _attach_step is not None:
            _check(LIB.lbm_attach(ctypes.byref(self._cp), ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                  int(_attach_step), ctypes.byref(self.handle)))
            return
        shape = (p.Ly, p.Lx)
        arrs = [np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), shape)) for a in (rho0, ux0, uy0)]
        _check(LIB.lbm_init(ctypes.byref(self._cp), ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), s,
                            *[_dptr(a) for a in arrs], ctypes.byref(self.handle)))

    @classmethod
    def attach(cls, p: Params, workspace, step: int) -> "Run":
        """Re-open a workspace (e.g. a restored checkpoint copy) holding a state after `step` steps."""
        return cls(p, None, None, None, workspace=workspace, _attach_step=step)

    # -- stepping ------------------------------------------------------------
    def step(self, n: int = 1, stream=None):
        _check(LIB.lbm_step(self.handle, int(n), _stream_handle(self.torch, stream)))

    def step_timed(self, n: int, stream=None) -> float:
        ms = ctypes.c_double()
        _check(LIB.lbm_step_timed(self.handle, int(n), _stream_handle(self.torch, stream), ctypes.byref(ms)))
        return ms.value

    @property
    def step_count(self) -> int:
        return int(LIB.lbm_step_count(self.handle))

    def set_launch(self, rows_per_wave: int, waves_per_group: int):
        _check(LIB.lbm_set_launch(self.handle, int(rows_per_wave), int(waves_per_group)))

    def get_launch(self):
        r, w = ctypes.c_int32(), ctypes.c_int32()
        _check(LIB.lbm_get_launch(self.handle, ctypes.byref(r), ctypes.byref(w)))
        return r.value, w.value

    # -- results -------------------------------------------------------------
    def moments(self, stream=None):
        shape = (self.p.Ly, self.p.Lx)
        rho, ux, uy = (np.empty(shape) for _ in range(3))
        _check(LIB.lbm_moments(self.handle, _dptr(rho), _dptr(ux), _dptr(uy), _stream_handle(self.torch, stream)))
        return rho, ux, uy

    def moments_device(self, stream=None):
        t = self.torch
        rho, ux, uy = (t.empty((self.p.Ly, self.p.Lx), dtype=t.float64, device="cuda") for _ in range(3))
        _check(LIB.lbm_moments_device(self.handle, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(ux.data_ptr()),
                                      ctypes.c_void_p(uy.data_ptr()), _stream_handle(t, stream)))
        return rho, ux, uy

    def get_f(self, stream=None) -> np.ndarray:
        f = np.empty((16, self.p.Ly, self.p.Lx))
        _check(LIB.lbm_get_f(self.handle, _dptr(f), _stream_handle(self.torch, stream)))
        return f

    def set_f(self, f: np.ndarray, stream=None):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (16, self.p.Ly, self.p.Lx)
        _check(LIB.lbm_set_f(self.handle, _dptr(f), _stream_handle(self.torch, stream)))

    def get_f_device(self, stream=None):
        t = self.torch
        f = t.empty((16, self.p.Ly, self.p.Lx), dtype=t.float64, device="cuda")
        _check(LIB.lbm_get_f_device(self.handle, ctypes.c_void_p(f.data_ptr()), _stream_handle(t, stream)))
        return f

    def reduce(self, threshold: float, stream=None, allow_nonfinite: bool = False) -> Dict[str, float]:
        cs = CStats()
        st = LIB.lbm_reduce(self.handle, float(threshold), ctypes.byref(cs), _stream_handle(self.torch, stream))
        if st == LBM_ENONFINITE and allow_nonfinite:
            return _stats_dict(cs)
        _check(st)
        return _stats_dict(cs)

    def state_device(self):
        """(device address, plane stride in values) of the current distribution
        field in the library's storage layout (see lbm_state_device)."""
        ptr, stride = ctypes.c_void_p(), ctypes.c_int64()
        _check(LIB.lbm_state_device(self.handle, ctypes.byref(ptr), ctypes.byref(stride)))
        return ptr.value, stride.value

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            LIB.lbm_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def reduce_field_static(p: Params, d_f: int, threshold: float, stream=None,
                        allow_nonfinite: bool = False) -> Dict[str, float]:
    """lbm_reduce_field_static: diagnostics of a device field at address d_f
    (storage layout of Run.state_device) without a run or a workspace; the
    library's own fixed device scratch holds the partial sums."""
    torch = _torch()
    cp = p.c()
    cs = CStats()
    st = LIB.lbm_reduce_field_static(ctypes.byref(cp), ctypes.c_void_p(d_f), float(threshold), ctypes.byref(cs),
                                     _stream_handle(torch, stream))
    if st == LBM_ENONFINITE and allow_nonfinite:
        return _stats_dict(cs)
    _check(st)
    return _stats_dict(cs)


def autotune(p: Params, steps_per_trial: int = 5, stream=None):
    """Time the candidate launch shapes on a scratch workspace; returns
    (rows_per_wave, waves_per_group) and remembers it for later runs of p's shape."""
    torch = _torch()
    ws = _workspace(torch, workspace_bytes(p))
    cp = p.c()
    r, w = ctypes.c_int32(), ctypes.c_int32()
    _check(LIB.lbm_autotune(ctypes.byref(cp), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                            _stream_handle(torch, stream), int(steps_per_trial), ctypes.byref(r), ctypes.byref(w)))
    del ws
    return r.value, w.value


class _Member(Run):
    """Borrowed handle of one run inside a Batch."""

    def __init__(self, batch: "Batch", index: int, p: Params):
        self.torch = batch.torch
        self.p = p
        self.handle = ctypes.c_void_p(LIB.lbm_batch_run(batch.handle, index))
        if not self.handle.value:
            raise LbmError(LBM_EINVAL, LIB.lbm_last_error().decode())
        self._batch = batch

    def close(self):
        self.handle = ctypes.c_void_p()


class Batch:
    """Independent runs advanced together by one grouped launch per step."""

    def __init__(self, params: Sequence[Params], fields_list, stream=None):
        torch = _torch()
        self.torch = torch
        self.params = list(params)
        n = len(self.params)
        self._cp = (CParams * n)(*[p.c() for p in self.params])
        nbytes = int(LIB.lbm_batch_workspace_bytes(n, self._cp))
        if nbytes == 0:
            for p in self.params:
                _check(validate(p))
            raise LbmError(LBM_EINVAL, "invalid batch")
        self.ws = _workspace(torch, nbytes)
        self._host = []
        P = ctypes.POINTER(ctypes.c_double)
        rho_p, ux_p, uy_p = (P * n)(), (P * n)(), (P * n)()
        for i, (p, (rho, ux, uy)) in enumerate(zip(self.params, fields_list)):
            arrs = [np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (p.Ly, p.Lx)))
                    for a in (rho, ux, uy)]
            self._host.append(arrs)
            rho_p[i], ux_p[i], uy_p[i] = (_dptr(a) for a in arrs)
        self.handle = ctypes.c_void_p()
        _check(LIB.lbm_batch_init(n, self._cp, ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                  _stream_handle(torch, stream), rho_p, ux_p, uy_p, ctypes.byref(self.handle)))
        self._host = None
        self.runs = [_Member(self, i, p) for i, p in enumerate(self.params)]

    def step(self, n: int, graph_steps: int = 0, stream=None):
        _check(LIB.lbm_batch_step(self.handle, int(n), int(graph_steps), _stream_handle(self.torch, stream)))

    def set_launch(self, rows_per_wave: int, stream=None):
        _check(LIB.lbm_batch_set_launch(self.handle, int(rows_per_wave), _stream_handle(self.torch, stream)))

    def set_mode(self, mode: int, stream=None):
        """BATCH_PER_STEP (one launch per step) or BATCH_PERSISTENT (FP32:
        one launch for many steps, items start when their neighbours finish)."""
        _check(LIB.lbm_batch_set_mode(self.handle, int(mode), _stream_handle(self.torch, stream)))

    @property
    def mode(self) -> int:
        return int(LIB.lbm_batch_get_mode(self.handle))

    def set_wait_limit(self, polls: int, stream=None):
        _check(LIB.lbm_batch_set_wait_limit(self.handle, int(polls), _stream_handle(self.torch, stream)))

    def sync_status(self, stream=None):
        """Raise LbmError if a persistent launch gave up a dependency wait."""
        _check(LIB.lbm_batch_sync_status(self.handle, _stream_handle(self.torch, stream)))

    def autotune(self, steps_per_trial: int = 3, stream=None) -> int:
        """Pick the launch mode and the rows per work item on the batch itself,
        one common value and then one per class of runs of a shape and
        boundary (remembered for later batches); advances every run by
        (steps_per_trial + 1) steps per trial (at least 17 for a trial of the
        persistent launch), 10 (FP64) or 20 (FP32) common trials plus up to
        1 + 4 per class.  Returns the common value."""
        rows = ctypes.c_int32()
        _check(LIB.lbm_batch_autotune(self.handle, int(steps_per_trial), _stream_handle(self.torch, stream),
                                      ctypes.byref(rows)))
        return rows.value

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            LIB.lbm_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""ctypes binding of the D3Q27 entry points of ``liboreg.so``
(``include/oreg3.h``): the ``lb3_*`` functions under their C names and a
``Lattice3`` class.  Argument marshalling only; the library is loaded by
``oreg`` (ImportError when it is missing, no fallback).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import oreg
from .oreg import LBError, check as _check_status  # noqa: F401  (re-exported error type)

_lib = oreg._lib
_H = ctypes.c_void_p
_VP = ctypes.c_void_p


class lb3_options(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("tau", ctypes.c_double), ("theta", ctypes.c_double),
        ("equilibrium", ctypes.c_int), ("storage", ctypes.c_int), ("collision", ctypes.c_int),
        ("rho0", ctypes.c_double),
        ("stream", ctypes.c_void_p), ("use_stream", ctypes.c_int),
        ("device", ctypes.c_int),
    ]


def _sig(name, res, args):
    fn = getattr(_lib, name)
    fn.restype = res
    fn.argtypes = args
    return fn


lb3_options_init = _sig("lb3_options_init", None, [ctypes.POINTER(lb3_options)])
lb3_create = _sig("lb3_create", ctypes.c_int, [ctypes.POINTER(lb3_options), ctypes.POINTER(_H)])
lb3_init = _sig("lb3_init", ctypes.c_int, [_H, _VP, _VP, _VP, _VP])
lb3_init_device = _sig("lb3_init_device", ctypes.c_int, [_H, _VP, _VP, _VP, _VP])
lb3_step = _sig("lb3_step", ctypes.c_int, [_H, ctypes.c_int64])
lb3_moments = _sig("lb3_moments", ctypes.c_int, [_H, _VP])
lb3_moments_device = _sig("lb3_moments_device", ctypes.c_int, [_H, _VP])
lb3_populations = _sig("lb3_populations", ctypes.c_int, [_H, _VP])
lb3_set_populations = _sig("lb3_set_populations", ctypes.c_int, [_H, _VP])
lb3_diagnostics = _sig("lb3_diagnostics", ctypes.c_int, [_H, _VP])
lb3_sync = _sig("lb3_sync", ctypes.c_int, [_H])
lb3_time = _sig("lb3_time", ctypes.c_int64, [_H])
lb3_device_bytes = _sig("lb3_device_bytes", ctypes.c_int64, [_H])
lb3_destroy = _sig("lb3_destroy", ctypes.c_int, [_H])
lb3_last_error = _sig("lb3_last_error", ctypes.c_char_p, [_H])

EXPORTED = ["lb3_options_init", "lb3_create", "lb3_init", "lb3_init_device", "lb3_step",
            "lb3_moments", "lb3_moments_device", "lb3_populations", "lb3_set_populations",
            "lb3_diagnostics", "lb3_sync", "lb3_time", "lb3_device_bytes", "lb3_destroy",
            "lb3_last_error"]


def check(status: int, handle=None) -> None:
    if status != oreg.LB_OK:
        raise LBError(status, (lb3_last_error(handle) or b"").decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Lattice3:
    """One periodic D3Q27 box resident on the GPU; arguments mirror
    ``lb3_options`` (string names as in ``oreg.Lattice``).  Fields are
    ``[nz, ny, nx]``, populations ``[27, nz, ny, nx]``."""

    def __init__(self, nx: int, ny: int, nz: int, tau: float, theta: float = 1.0 / 3.0,
                 equilibrium: str = "guided", storage: str = "f64", collision: str = "oreg",
                 rho0: float = 1.0, stream=None, device: int = -1):
        o = lb3_options()
        lb3_options_init(ctypes.byref(o))
        o.nx, o.ny, o.nz = int(nx), int(ny), int(nz)
        o.tau, o.theta = float(tau), float(theta)
        o.equilibrium = oreg.EQUILIBRIA[equilibrium]
        o.storage = oreg.STORAGES[storage]
        o.collision = oreg.COLLISIONS[collision]
        o.rho0 = float(rho0)
        if stream is not None:
            if hasattr(stream, "cuda_stream"):
                stream = stream.cuda_stream
            o.stream = int(stream) or None
            o.use_stream = 1
        o.device = int(device)
        h = _H()
        check(lb3_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.shape = (int(nz), int(ny), int(nx))
        self.options = o

    def close(self) -> None:
        if getattr(self, "_h", None):
            lb3_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    @property
    def time(self) -> int:
        return int(lb3_time(self._h))

    @property
    def device_bytes(self) -> int:
        return int(lb3_device_bytes(self._h))

    def init(self, rho, ux, uy, uz) -> None:
        """f(x, 0) = f^eq(rho, u): numpy arrays or float64 device tensors [nz, ny, nx]."""
        if oreg._is_device_tensor(rho):
            ptrs = [oreg._device_ptr(a, self.shape) for a in (rho, ux, uy, uz)]
            oreg._ready([rho, ux, uy, uz])
            check(lb3_init_device(self._h, *ptrs), self._h)
            return
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (rho, ux, uy, uz)]
        for a in arrs:
            if a.shape != self.shape:
                raise ValueError(f"field shape {a.shape} != {self.shape}")
        check(lb3_init(self._h, *[_ptr(a) for a in arrs]), self._h)

    def step(self, n: int = 1) -> None:
        check(lb3_step(self._h, int(n)), self._h)

    def sync(self) -> None:
        check(lb3_sync(self._h), self._h)

    def moments(self, out=None):
        """rho, ux, uy, uz of the pre-collision state, [4, nz, ny, nx]."""
        if out is not None and oreg._is_device_tensor(out):
            ptr = oreg._device_ptr(out, (4, *self.shape))
            oreg._ready([out])
            check(lb3_moments_device(self._h, ptr), self._h)
            return out
        res = np.empty((4, *self.shape))
        check(lb3_moments(self._h, _ptr(res)), self._h)
        return res

    def populations(self) -> np.ndarray:
        res = np.empty((27, *self.shape))
        check(lb3_populations(self._h, _ptr(res)), self._h)
        return res

    def set_populations(self, f) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64)
        if f.shape != (27, *self.shape):
            raise ValueError(f"populations shape {f.shape} != {(27, *self.shape)}")
        check(lb3_set_populations(self._h, _ptr(f)), self._h)

    def diagnostics(self) -> np.ndarray:
        """[mass, jx, jy, jz, kinetic energy, total energy, non-finite node count]."""
        res = np.empty(7)
        check(lb3_diagnostics(self._h, _ptr(res)), self._h)
        return res

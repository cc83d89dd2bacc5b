"""ctypes binding of ``liboreg.so`` (the C ABI declared in ``include/oreg.h``).

Only argument marshalling lives here: every step of the method runs in the
library's HIP kernels.  The module exposes the C entry points under their C
names (``lb_create``, ``lb_step``, ...) and a small ``Lattice`` class on top.
PyTorch, when used, only supplies device memory (``tensor.data_ptr()``) and a
HIP stream (``torch.cuda.current_stream().cuda_stream``).

Importing the module loads the library and raises ``ImportError`` if it has
not been built (``python -m paper_2501_16000_amd.build``); there is no other
implementation to fall back to.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIBRARY_PATH = os.path.join(_PKG, "liboreg.so")

if not os.path.exists(LIBRARY_PATH):
    raise ImportError(
        f"{LIBRARY_PATH} is missing: build it with `python -m paper_2501_16000_amd.build` "
        "(hipcc, gfx950)")

# One process holds one HIP runtime.  libamdhip64 is resolved by soname, so the
# first copy loaded serves every library; when PyTorch is installed, load it
# first so that its tensors, streams and this library share its runtime.
try:
    import torch  # noqa: F401
except ImportError:
    pass

_lib = ctypes.CDLL(LIBRARY_PATH)

# ----------------------------------------------------------------- enums --
LB_EQ_GUIDED, LB_EQ_POLY2 = 0, 1
LB_F64, LB_F32S, LB_F16S, LB_BF16S = 0, 1, 2, 3
LB_COLL_OREG, LB_COLL_BGK = 0, 1
LB_BC_PERIODIC, LB_BC_BOUNCEBACK = 0, 1
LB_OK, LB_EINVAL, LB_ENOMEM, LB_EDEVICE, LB_ESTATE, LB_ENONFINITE, LB_EAGAIN = 0, -1, -2, -3, -4, -5, -6

EQUILIBRIA = {"guided": LB_EQ_GUIDED, "poly2": LB_EQ_POLY2}
STORAGES = {"f64": LB_F64, "f32s": LB_F32S, "f16s": LB_F16S, "bf16s": LB_BF16S}
COLLISIONS = {"oreg": LB_COLL_OREG, "bgk": LB_COLL_BGK}
BOUNDARIES = {"periodic": LB_BC_PERIODIC, "bounceback": LB_BC_BOUNCEBACK}
STORAGE_BYTES = {LB_F64: 8, LB_F32S: 4, LB_F16S: 2, LB_BF16S: 2}


class lb_options(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("tau", ctypes.c_double), ("theta", ctypes.c_double),
        ("equilibrium", ctypes.c_int), ("storage", ctypes.c_int),
        ("collision", ctypes.c_int), ("boundary_x", ctypes.c_int),
        ("rho0", ctypes.c_double),
        ("stream", ctypes.c_void_p),
        ("use_stream", ctypes.c_int),
        ("device", ctypes.c_int),
        ("check_nonfinite", ctypes.c_int),
        ("fuse_steps", ctypes.c_int),
    ]


_H = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_VP = ctypes.c_void_p


def _sig(name, res, args):
    fn = getattr(_lib, name)
    fn.restype = res
    fn.argtypes = args
    return fn


lb_options_init = _sig("lb_options_init", None, [ctypes.POINTER(lb_options)])
lb_create = _sig("lb_create", ctypes.c_int,
                 [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                  ctypes.POINTER(_H)])
lb_create_ex = _sig("lb_create_ex", ctypes.c_int, [ctypes.POINTER(lb_options), ctypes.POINTER(_H)])
lb_init = _sig("lb_init", ctypes.c_int, [_H, _VP, _VP, _VP])
lb_init_device = _sig("lb_init_device", ctypes.c_int, [_H, _VP, _VP, _VP])
lb_step = _sig("lb_step", ctypes.c_int, [_H, ctypes.c_int64])
lb_moments = _sig("lb_moments", ctypes.c_int, [_H, _VP])
lb_moments_device = _sig("lb_moments_device", ctypes.c_int, [_H, _VP])
lb_populations = _sig("lb_populations", ctypes.c_int, [_H, _VP])
lb_set_populations = _sig("lb_set_populations", ctypes.c_int, [_H, _VP])
lb_diagnostics = _sig("lb_diagnostics", ctypes.c_int, [_H, _VP])
lb_density_profile = _sig("lb_density_profile", ctypes.c_int, [_H, _VP])
lb_diagnostics_device_noalloc = _sig("lb_diagnostics_device_noalloc", ctypes.c_int, [_H, _VP])
lb_sync = _sig("lb_sync", ctypes.c_int, [_H])
lb_time = _sig("lb_time", ctypes.c_int64, [_H])
lb_get_options = _sig("lb_get_options", ctypes.c_int, [_H, ctypes.POINTER(lb_options)])
lb_device_bytes = _sig("lb_device_bytes", ctypes.c_int64, [_H])
lb_destroy = _sig("lb_destroy", ctypes.c_int, [_H])
lb_status_string = _sig("lb_status_string", ctypes.c_char_p, [ctypes.c_int])
lb_last_error = _sig("lb_last_error", ctypes.c_char_p, [_H])
lb_copy_device = _sig("lb_copy_device", ctypes.c_int, [_VP, _VP, ctypes.c_int64, _VP])

EXPORTED = [
    "lb_options_init", "lb_create", "lb_create_ex", "lb_init", "lb_init_device", "lb_step",
    "lb_moments", "lb_moments_device", "lb_populations", "lb_set_populations",
    "lb_diagnostics", "lb_density_profile", "lb_sync", "lb_time", "lb_get_options",
    "lb_device_bytes", "lb_destroy", "lb_status_string", "lb_last_error", "lb_copy_device",
    "lb_diagnostics_device_noalloc",
]


class LBError(RuntimeError):
    """A failing ``lb_status`` with the library's message."""

    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{lb_status_string(status).decode()}: {message}")


def check(status: int, handle=None) -> None:
    if status != LB_OK:
        raise LBError(status, (lb_last_error(handle) or b"").decode())


def copy_device(src_ptr: int, dst_ptr: int, nbytes: int, stream: int = 0) -> None:
    """``lb_copy_device``: the plain streaming copy between two device buffers
    (the practical HBM ceiling); asynchronous on ``stream`` (a HIP stream
    handle, 0 for the null stream)."""
    check(lb_copy_device(src_ptr, dst_ptr, nbytes, stream or None))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _is_device_tensor(a) -> bool:
    return hasattr(a, "is_cuda") and a.is_cuda


def _ready(tensors) -> None:
    """Wait for torch's current stream on the tensors' device: the library
    reads them on the lattice's own stream, which is not ordered after
    torch's work."""
    import torch
    torch.cuda.current_stream(tensors[0].device).synchronize()


def _device_ptr(t, shape) -> int:
    import torch
    if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected a contiguous float64 device tensor of shape {shape}")
    return t.data_ptr()


class Lattice:
    """One D2Q9 lattice resident on the GPU.

    Parameters mirror ``lb_options``; string names select the enums:
    equilibrium 'guided' | 'poly2', storage 'f64' | 'f32s' | 'f16s' | 'bf16s',
    collision 'oreg' | 'bgk', boundary_x 'periodic' | 'bounceback'.
    ``fuse_steps`` 0 lets ``step`` fuse several time steps per launch when the
    lattice is large enough, 1 runs one sweep launch per step, 2 fuses at any
    size (identical results in every case).
    ``stream`` is a HIP stream handle (int, 0 = the null stream) or a
    ``torch.cuda.Stream``; None lets the lattice create its own stream.
    """

    def __init__(self, nx: int, ny: int, tau: float, theta: float = 1.0 / 3.0,
                 equilibrium: str = "guided", storage: str = "f64", collision: str = "oreg",
                 boundary_x: str = "periodic", rho0: float = 1.0, stream=None,
                 device: int = -1, check_nonfinite: bool = False, fuse_steps: int = 0):
        o = lb_options()
        lb_options_init(ctypes.byref(o))
        o.nx, o.ny, o.tau, o.theta = int(nx), int(ny), float(tau), float(theta)
        o.equilibrium = EQUILIBRIA[equilibrium]
        o.storage = STORAGES[storage]
        o.collision = COLLISIONS[collision]
        o.boundary_x = BOUNDARIES[boundary_x]
        o.rho0 = float(rho0)
        if stream is not None:
            if hasattr(stream, "cuda_stream"):
                stream = stream.cuda_stream
            o.stream = int(stream) or None
            o.use_stream = 1
        o.device = int(device)
        o.check_nonfinite = int(bool(check_nonfinite))
        o.fuse_steps = int(fuse_steps)
        h = _H()
        check(lb_create_ex(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.nx, self.ny = int(nx), int(ny)
        self.options = o

    # -- lifecycle --------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_h", None):
            lb_destroy(self._h)
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
        return int(lb_time(self._h))

    @property
    def device_bytes(self) -> int:
        return int(lb_device_bytes(self._h))

    # -- state ------------------------------------------------------------
    def init(self, rho, ux, uy) -> None:
        """f(x, 0) = f^eq(rho, u): numpy arrays or float64 device tensors [ny, nx]."""
        shape = (self.ny, self.nx)
        if _is_device_tensor(rho):
            ptrs = [_device_ptr(a, shape) for a in (rho, ux, uy)]
            _ready([rho, ux, uy])
            check(lb_init_device(self._h, *ptrs), self._h)
            return
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (rho, ux, uy)]
        for a in arrs:
            if a.shape != shape:
                raise ValueError(f"field shape {a.shape} != {shape}")
        check(lb_init(self._h, *[_ptr(a) for a in arrs]), self._h)

    def step(self, n: int = 1) -> None:
        check(lb_step(self._h, int(n)), self._h)

    def sync(self) -> None:
        check(lb_sync(self._h), self._h)

    def moments(self, out=None):
        """rho, ux, uy of the pre-collision state, [3, ny, nx] float64.

        With ``out`` a float64 device tensor the gather is enqueued
        asynchronously into it; otherwise a numpy array is returned."""
        if out is not None and _is_device_tensor(out):
            ptr = _device_ptr(out, (3, self.ny, self.nx))
            _ready([out])
            check(lb_moments_device(self._h, ptr), self._h)
            return out
        res = np.empty((3, self.ny, self.nx))
        check(lb_moments(self._h, _ptr(res)), self._h)
        return res

    def populations(self) -> np.ndarray:
        res = np.empty((9, self.ny, self.nx))
        check(lb_populations(self._h, _ptr(res)), self._h)
        return res

    def set_populations(self, f) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64)
        if f.shape != (9, self.ny, self.nx):
            raise ValueError(f"populations shape {f.shape} != {(9, self.ny, self.nx)}")
        check(lb_set_populations(self._h, _ptr(f)), self._h)

    def diagnostics(self) -> np.ndarray:
        """[mass, jx, jy, kinetic energy, total energy, non-finite node count]."""
        res = np.empty(6)
        check(lb_diagnostics(self._h, _ptr(res)), self._h)
        return res

    def diagnostics_device_noalloc(self, out):
        """``lb_diagnostics_device_noalloc``: the six sums of ``diagnostics``
        enqueued into ``out`` (a float64 device tensor of 6 elements) on the
        lattice's stream, with no allocation and no synchronization."""
        ptr = _device_ptr(out, (6,))
        _ready([out])
        check(lb_diagnostics_device_noalloc(self._h, ptr), self._h)
        return out

    def density_profile(self) -> np.ndarray:
        res = np.empty(self.nx)
        check(lb_density_profile(self._h, _ptr(res)), self._h)
        return res

"""FP64 CPU oracle of the Onsager-regularized method on the D3Q27 lattice.

TEST INFRASTRUCTURE ONLY (the test suite and the CPU baseline of
``bench.py``).  The arithmetic lives in ``oreg_oracle3.c``: Eq. (11) with a
third axis factor, Eq. (6) with D = 3, Eqs. (7) and (1) on a periodic box.
This module only builds it with gcc and marshals numpy arrays: fields
``[nz, ny, nx]``, populations ``[27, nz, ny, nx]`` with velocity index
``i = 9 (c_z + 1) + 3 (c_y + 1) + (c_x + 1)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oreg_oracle3.c")
_LIB = os.path.join(_HERE, "liboreg_oracle3.so")
# A different build (the mutation tests load deliberately broken copies).
_LIB_OVERRIDE = os.environ.get("OREG_ORACLE3_LIB")

_EQ = {"guided": 0, "poly2": 1}
_COLL = {"oreg": 0, "bgk": 1}


def build() -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-fopenmp", "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _LIB_OVERRIDE:
        path = _LIB_OVERRIDE
    else:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        path = _LIB
    lib = ctypes.CDLL(path)
    d, i = ctypes.c_double, ctypes.c_int
    P = ctypes.POINTER(ctypes.c_double)
    lib.orc3_velocities.argtypes = [ctypes.POINTER(ctypes.c_int)]
    lib.orc3_equilibrium.argtypes = [i, d, d, P, P]
    lib.orc3_moments_cell.argtypes = [P, P, P]
    lib.orc3_stress.argtypes = [P, P]
    lib.orc3_oreg_cell.argtypes = [i, d, P, P]
    lib.orc3_collide_cell.argtypes = [i, i, d, d, P, P]
    lib.orc3_init.argtypes = [i, i, i, i, d, P, P, P, P, P]
    lib.orc3_run.argtypes = [i, i, i, i, i, d, d, ctypes.c_int64, P, P, i]
    lib.orc3_moments.argtypes = [i, i, i, P, P]
    lib.orc3_diagnostics.argtypes = [i, i, i, d, P, P]
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def velocities() -> np.ndarray:
    c = np.zeros((27, 3), dtype=np.int32)
    _load().orc3_velocities(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return c


def equilibrium(eq: str, theta: float, rho: float, u) -> np.ndarray:
    u = _f64(u)
    out = np.zeros(27)
    _load().orc3_equilibrium(_EQ[eq], theta, rho, _p(u), _p(out))
    return out


def moments_cell(f):
    f = _f64(f)
    r = ctypes.c_double()
    u = np.zeros(3)
    _load().orc3_moments_cell(_p(f), ctypes.byref(r), _p(u))
    return r.value, u


def stress(fneq) -> np.ndarray:
    fneq = _f64(fneq)
    S = np.zeros((3, 3))
    _load().orc3_stress(_p(fneq), _p(S))
    return S


def oreg_cell(eq: str, theta: float, f) -> np.ndarray:
    f = _f64(f)
    out = np.zeros(27)
    _load().orc3_oreg_cell(_EQ[eq], theta, _p(f), _p(out))
    return out


def collide_cell(eq: str, tau: float, theta: float, f, collision: str = "oreg") -> np.ndarray:
    f = _f64(f)
    out = np.zeros(27)
    _load().orc3_collide_cell(_EQ[eq], _COLL[collision], tau, theta, _p(f), _p(out))
    return out


def init(eq: str, theta: float, rho, ux, uy, uz) -> np.ndarray:
    """f(x, 0) = f^eq(rho(x), u(x)); returns [27, nz, ny, nx]."""
    rho, ux, uy, uz = _f64(rho), _f64(ux), _f64(uy), _f64(uz)
    nz, ny, nx = rho.shape
    f = np.zeros((27, nz, ny, nx))
    _load().orc3_init(nx, ny, nz, _EQ[eq], theta, _p(rho), _p(ux), _p(uy), _p(uz), _p(f))
    return f


def run(f, nsteps: int, tau: float, theta: float, eq: str = "guided",
        collision: str = "oreg", nthreads: int = 0) -> np.ndarray:
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    _, nz, ny, nx = f.shape
    tmp = np.empty_like(f)
    _load().orc3_run(nx, ny, nz, _EQ[eq], _COLL[collision], tau, theta, int(nsteps),
                     _p(f), _p(tmp), int(nthreads))
    return f


def moments(f) -> np.ndarray:
    """rho, ux, uy, uz of every cell: [4, nz, ny, nx]."""
    f = _f64(f)
    _, nz, ny, nx = f.shape
    out = np.zeros((4, nz, ny, nx))
    _load().orc3_moments(nx, ny, nz, _p(f), _p(out))
    return out


def diagnostics(f, theta: float) -> np.ndarray:
    """[mass, jx, jy, jz, kinetic energy, total energy, non-finite cell count]."""
    f = _f64(f)
    _, nz, ny, nx = f.shape
    out = np.zeros(7)
    _load().orc3_diagnostics(nx, ny, nz, theta, _p(f), _p(out))
    return out

"""FP64 CPU oracle of the Onsager-regularized D2Q9 lattice Boltzmann method.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU
baseline of ``bench.py`` are the only users; the GPU library and its Python
binding never import this package, and it imports nothing from them.

The arithmetic lives in ``oreg_oracle.c`` (plain C, FP64, the paper's formulas
as printed: Eqs. (1), (6), (7), (11) and the Sec. III.D polynomial
equilibrium).  This module only builds it with gcc and marshals numpy arrays.
Arrays are ``float64`` C-contiguous: fields ``[ny, nx]``, populations
``[9, ny, nx]`` in the velocity order

    0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oreg_oracle.c")
_LIB = os.path.join(_HERE, "liboreg_oracle.so")
# A different build of the oracle (the mutation tests load deliberately broken
# copies this way to show that the pins catch them).
_LIB_OVERRIDE = os.environ.get("OREG_ORACLE_LIB")

EQ_GUIDED, EQ_POLY2 = 0, 1
COLL_OREG, COLL_BGK = 0, 1
BC_PERIODIC, BC_BOUNCEBACK = 0, 1

_EQ = {"guided": EQ_GUIDED, "poly2": EQ_POLY2}
_COLL = {"oreg": COLL_OREG, "bgk": COLL_BGK}
_BC = {"periodic": BC_PERIODIC, "bounceback": BC_BOUNCEBACK}


def build() -> str:
    """Compile the oracles with gcc (-O2, no fast-math, OpenMP): this D2Q9 one
    and the D3Q27 one of ``oracle.d3q27``."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-fopenmp", "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    from . import d3q27
    d3q27.build()
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
    d = ctypes.c_double
    i = ctypes.c_int
    P = ctypes.POINTER(ctypes.c_double)
    lib.orc_equilibrium.argtypes = [i, d, d, d, d, P]
    lib.orc_moments_cell.argtypes = [P, P, P, P]
    lib.orc_stress.argtypes = [P, P]
    lib.orc_oreg_cell.argtypes = [i, d, P, P]
    lib.orc_collide_cell.argtypes = [i, i, d, d, P, P]
    lib.orc_init.argtypes = [i, i, i, d, P, P, P, P]
    lib.orc_run.argtypes = [i, i, i, i, i, d, d, ctypes.c_int64, P, P, i]
    lib.orc_moments.argtypes = [i, i, P, P]
    lib.orc_diagnostics.argtypes = [i, i, d, P, P]
    lib.orc_velocities.argtypes = [ctypes.POINTER(ctypes.c_int)]
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def velocities() -> np.ndarray:
    """The D2Q9 velocity table c[i, alpha] (int)."""
    c = np.zeros((9, 2), dtype=np.int32)
    _load().orc_velocities(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return c


def equilibrium(eq: str, theta: float, rho: float, ux: float, uy: float) -> np.ndarray:
    """f^eq of one cell (Eq. (11) or the Sec. III.D polynomial form)."""
    out = np.zeros(9)
    _load().orc_equilibrium(_EQ[eq], theta, rho, ux, uy, _p(out))
    return out


def moments_cell(f) -> tuple[float, float, float]:
    f = _f64(f)
    r, ux, uy = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _load().orc_moments_cell(_p(f), ctypes.byref(r), ctypes.byref(ux), ctypes.byref(uy))
    return r.value, ux.value, uy.value


def stress(fneq) -> np.ndarray:
    """Inner trace-free sum S[a, b] of Eq. (6)."""
    fneq = _f64(fneq)
    S = np.zeros((2, 2))
    _load().orc_stress(_p(fneq), _p(S))
    return S


def oreg_cell(eq: str, theta: float, f) -> np.ndarray:
    """Eq. (6): f^OReg of one cell."""
    f = _f64(f)
    out = np.zeros(9)
    _load().orc_oreg_cell(_EQ[eq], theta, _p(f), _p(out))
    return out


def collide_cell(eq: str, tau: float, theta: float, f, collision: str = "oreg") -> np.ndarray:
    """Post-collision populations of one cell (Eq. (7), or Eq. (1) for 'bgk')."""
    f = _f64(f)
    out = np.zeros(9)
    _load().orc_collide_cell(_EQ[eq], _COLL[collision], tau, theta, _p(f), _p(out))
    return out


def init(eq: str, theta: float, rho, ux, uy) -> np.ndarray:
    """f(x, 0) = f^eq(rho(x), u(x)); returns [9, ny, nx]."""
    rho, ux, uy = _f64(rho), _f64(ux), _f64(uy)
    ny, nx = rho.shape
    f = np.zeros((9, ny, nx))
    _load().orc_init(nx, ny, _EQ[eq], theta, _p(rho), _p(ux), _p(uy), _p(f))
    return f


def run(f, nsteps: int, tau: float, theta: float, eq: str = "guided",
        collision: str = "oreg", bc_x: str = "periodic", nthreads: int = 0) -> np.ndarray:
    """Apply ``nsteps`` time steps to populations ``f`` [9, ny, nx]; returns a new array."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    _, ny, nx = f.shape
    tmp = np.empty_like(f)
    _load().orc_run(nx, ny, _EQ[eq], _COLL[collision], _BC[bc_x], tau, theta,
                    int(nsteps), _p(f), _p(tmp), int(nthreads))
    return f


def moments(f) -> np.ndarray:
    """rho, ux, uy of every cell: [3, ny, nx]."""
    f = _f64(f)
    _, ny, nx = f.shape
    out = np.zeros((3, ny, nx))
    _load().orc_moments(nx, ny, _p(f), _p(out))
    return out


def diagnostics(f, theta: float) -> np.ndarray:
    """[mass, jx, jy, kinetic energy, total energy, non-finite cell count]."""
    f = _f64(f)
    _, ny, nx = f.shape
    out = np.zeros(6)
    _load().orc_diagnostics(nx, ny, theta, _p(f), _p(out))
    return out

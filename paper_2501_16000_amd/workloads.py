"""Seeded synthetic inputs for the OReg D2Q9 lattice.

This module holds no arithmetic of the lattice Boltzmann method: it only
builds initial macroscopic fields (density and velocity on the nodes), plain
random noise and request schedules.  The GPU library and the CPU oracle both
take these arrays as inputs.  Fields are float64 arrays of shape ``[ny, nx]``
with nodes at integer coordinates ``(x, y)``, x fastest.

Workloads (the paper's benchmarks of Sec. IV, restated on periodic grids):

* ``shear_wave``: a decaying shear wave whose fronts are rotated by
  atan(1/2) from the axes.  The phase is ``s = (2x + y)/N`` so the wave vector
  ``k = (2 pi / N) (2, 1)`` is periodic on an ``N x N`` grid and ``|k|^2 =
  5 (2 pi / N)^2``; the velocity ``u0 sin(2 pi s)`` points along
  ``(-1, 2)/sqrt(5)``, parallel to the fronts (divergence free).
* ``paper_shear_wave``: the axis-aligned and pi/4-rotated waves of Eq. (18)
  with a mean flow ``Ma sqrt(theta)`` along y.
* ``shocktube``: a density step (1.5 | 0.75 by default) at rest.
* ``smooth_random_velocity``: a divergence-free field from a stream function
  with 8 x 8 Fourier modes and random phases (numpy PCG64, seeded), scaled to
  a given maximum speed.
* ``serving_requests``: the request stream of the serving benchmark.
* ``shear_wave3``: the 3D shear wave of the D3Q27 lattice, fronts normal to
  the body diagonal: phase ``s = (x + y + z)/N``, ``|k|^2 = 3 (2 pi / N)^2``,
  velocity along ``(1, -1, 0)/sqrt(2)``; 3D fields are ``[nz, ny, nx]``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "shear_wave", "shear_wave_k2", "paper_shear_wave", "shocktube",
    "shear_wave3", "shear_wave3_k2", "shear_wave3_projection", "shear_wave_at",
    "shear_wave3_at",
    "smooth_random_velocity", "noise", "ServingRequest", "serving_requests",
]


def _grid(nx: int, ny: int):
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                       indexing="ij")
    return x, y


def shear_wave(n: int, u0: float, rho: float = 1.0, mode: int = 1):
    """Rotated (atan(1/2)) shear wave on an ``n x n`` periodic grid.

    Returns ``(rho, ux, uy)``, each ``[n, n]`` float64.
    """
    x, y = _grid(n, n)
    s = mode * (2.0 * x + y) / n
    amp = u0 * np.sin(2.0 * np.pi * s)
    e_perp = np.array([-1.0, 2.0]) / math.sqrt(5.0)
    return (np.full((n, n), float(rho)), amp * e_perp[0], amp * e_perp[1])


def shear_wave_at(x, y, n: int, u0: float, xp=np):
    """Fields of ``shear_wave(n, u0)`` at nodes (x, y) (arrays of any shape);
    ``xp`` is the array namespace (numpy, or torch for fields built on the
    device).  Returns ``(rho, ux, uy)``."""
    s = (2.0 * x + y) / n
    amp = u0 * xp.sin(2.0 * math.pi * s)
    rho = xp.ones_like(amp)
    return rho, amp * (-1.0 / math.sqrt(5.0)), amp * (2.0 / math.sqrt(5.0))


def shear_wave3_at(x, y, z, n: int, u0: float, xp=np):
    """Fields of ``shear_wave3(n, u0)`` (cube) at nodes (x, y, z)."""
    s = (x + y + z) / n
    amp = u0 * xp.sin(2.0 * math.pi * s)
    return xp.ones_like(amp), amp * _E3[0], amp * _E3[1], amp * 0.0


def shear_wave_k2(n: int, mode: int = 1) -> float:
    """|k|^2 of ``shear_wave(n, ..., mode)``."""
    return 5.0 * (2.0 * math.pi * mode / n) ** 2


def shear_wave_projection(n: int, mode: int = 1):
    """Unit vector e_perp and the complex phase exp(-2 pi i s) of the wave, used
    to project a velocity field onto the wave's Fourier mode."""
    x, y = _grid(n, n)
    s = mode * (2.0 * x + y) / n
    return np.array([-1.0, 2.0]) / math.sqrt(5.0), np.exp(-2j * np.pi * s)


def _grid3(nx: int, ny: int, nz: int):
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


_E3 = np.array([1.0, -1.0, 0.0]) / math.sqrt(2.0)


def shear_wave3(n: int, u0: float, rho: float = 1.0, nz: int | None = None):
    """Shear wave on an ``n x n x nz`` periodic box (``nz = n`` by default),
    wave vector ``(2 pi / n) (1, 1, 1)`` when ``nz = n``; returns
    ``(rho, ux, uy, uz)``, each ``[nz, n, n]`` float64.  With ``nz != n`` the
    phase is ``(x + y)/n + z/nz`` (still periodic)."""
    nz = n if nz is None else nz
    x, y, z = _grid3(n, n, nz)
    s = (x + y) / n + z / nz
    amp = u0 * np.sin(2.0 * np.pi * s)
    return (np.full(x.shape, float(rho)), amp * _E3[0], amp * _E3[1], amp * _E3[2])


def shear_wave3_k2(n: int, nz: int | None = None) -> float:
    nz = n if nz is None else nz
    return 2.0 * (2.0 * math.pi / n) ** 2 + (2.0 * math.pi / nz) ** 2


def shear_wave3_projection(n: int, nz: int | None = None):
    """Unit vector e_perp and the phase exp(-2 pi i s) of ``shear_wave3``."""
    nz = n if nz is None else nz
    x, y, z = _grid3(n, n, nz)
    return _E3, np.exp(-2j * np.pi * ((x + y) / n + z / nz))


def paper_shear_wave(ly: int, a0: float, ma: float, theta: float, rotated: bool, lx: int = 1):
    """Initial fields of Eq. (18) on an ``lx x ly`` grid (unit density).

    Axis-aligned: ``ux = a0 sin(2 pi y / ly)``, ``uy = Ma sqrt(theta)``.
    Rotated: the same profile in the phase ``2 pi (-x + y) / (ly sqrt 2)``
    added to both components.  The rotated phase is periodic only when the
    grid is square and the phase is taken as ``2 pi (-x + y) / ly``; this
    function uses that periodic form (see the design notes on Eq. (18)).
    """
    x, y = _grid(lx, ly)
    uy0 = ma * math.sqrt(theta)
    if not rotated:
        ux = a0 * np.sin(2.0 * np.pi * y / ly)
        uy = np.full_like(ux, uy0)
    else:
        ph = a0 * np.sin(2.0 * np.pi * (-x + y) / ly)
        ux = ph.copy()
        uy = uy0 + ph
    return np.ones((ly, lx)), ux, uy


def shocktube(nx: int, ny: int, rho_left: float = 1.5, rho_right: float = 0.75,
              split: int | None = None):
    """Density step at rest: ``rho_left`` for ``x < split`` (default nx/2)."""
    split = nx // 2 if split is None else split
    x, _ = _grid(nx, ny)
    rho = np.where(x < split, rho_left, rho_right).astype(np.float64)
    return rho, np.zeros((ny, nx)), np.zeros((ny, nx))


def smooth_random_velocity(n: int, umax: float = 0.03, modes: int = 8, seed: int = 2501,
                           rho: float = 1.0):
    """Divergence-free random velocity from a stream function.

    psi = sum_{m,l=1..modes} A_ml sin(2 pi m x/n + a_ml) sin(2 pi l y/n + b_ml),
    A_ml ~ N(0,1)/(m^2 + l^2), a, b ~ U[0, 2 pi); u = (d psi/dy, -d psi/dx)
    evaluated analytically, then scaled so that max |u| = umax.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.standard_normal((modes, modes))
    al = rng.uniform(0.0, 2.0 * np.pi, (modes, modes))
    be = rng.uniform(0.0, 2.0 * np.pi, (modes, modes))
    xs = np.arange(n, dtype=np.float64)
    kk = 2.0 * np.pi / n
    m = np.arange(1, modes + 1, dtype=np.float64)
    a = A / (m[:, None] ** 2 + m[None, :] ** 2)          # [m, l]
    # sin(kk m x + al) = sin(kk m x) cos(al) + cos(kk m x) sin(al): every term
    # is a product of a function of y and a function of x, so both velocity
    # components are one [n, 2 modes^2] x [2 modes^2, n] product.
    ph_x = kk * m[:, None] * xs[None, :]                  # [m, x]
    sxm, cxm = np.sin(ph_x), np.cos(ph_x)
    ph_y = kk * m[None, :, None] * xs[None, None, :] + be[:, :, None]   # [m, l, y]
    sy, cy = np.sin(ph_y), np.cos(ph_y)
    # u_x = d psi / dy = sum a (kk l) cos(kk l y + be) sin(kk m x + al)
    wx = (a * kk * m[None, :])[:, :, None] * cy           # [m, l, y]
    left_x = np.concatenate([(wx * np.cos(al)[:, :, None]).sum(1),
                             (wx * np.sin(al)[:, :, None]).sum(1)])   # [2m, y]
    ux = left_x.T @ np.concatenate([sxm, cxm])           # [y, x]
    # u_y = -d psi / dx = -sum a (kk m) sin(kk l y + be) cos(kk m x + al),
    # cos(kk m x + al) = cos(kk m x) cos(al) - sin(kk m x) sin(al)
    wy = (a * kk * m[:, None])[:, :, None] * sy
    left_y = np.concatenate([(wy * np.cos(al)[:, :, None]).sum(1),
                             -(wy * np.sin(al)[:, :, None]).sum(1)])
    uy = -(left_y.T @ np.concatenate([cxm, sxm]))
    speed = np.sqrt(ux * ux + uy * uy).max()
    scale = umax / speed
    return np.full((n, n), float(rho)), ux * scale, uy * scale


def noise(shape, seed: int, amplitude: float = 1.0) -> np.ndarray:
    """Uniform noise in [-amplitude, amplitude] (numpy PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return amplitude * rng.uniform(-1.0, 1.0, size=shape)


@dataclass
class ServingRequest:
    """One independent shear-wave simulation of the serving stream."""
    rid: int
    arrival_s: float
    n: int
    tau: float
    u0: float
    steps: int


def serving_requests(count: int = 2000, seed: int = 16000, rate_hz: float = 100.0,
                     n_min: int = 32, n_max: int = 1024, tau_range=(0.52, 1.2),
                     u0_range=(0.005, 0.05), steps_range=(200, 5000)):
    """Request stream: ln N ~ U[ln n_min, ln n_max] (rounded to an integer),
    tau, u0 uniform, steps uniform integers, Poisson arrivals at ``rate_hz``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), count))).astype(int)
    tau = rng.uniform(tau_range[0], tau_range[1], count)
    u0 = rng.uniform(u0_range[0], u0_range[1], count)
    steps = rng.integers(steps_range[0], steps_range[1] + 1, count)
    gaps = rng.exponential(1.0 / rate_hz, count)
    arrivals = np.cumsum(gaps) - gaps[0]
    return [ServingRequest(i, float(arrivals[i]), int(n[i]), float(tau[i]), float(u0[i]),
                           int(steps[i])) for i in range(count)]

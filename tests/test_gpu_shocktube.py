"""The walled shocktube of Sec. IV on the GPU (full-way bounce-back columns,
guided equilibrium, 800 x 1, 500 steps) against the FP64 oracle, for OReg and
lattice BGK at theta = 0.35, nu = 1e-5 and theta = 0.4, nu = 1e-9 (tau - 1/2
down to 2.5e-9, the least damped settings of the paper).  The density profiles
agree to 1e-12 (measured 1.5e-13 at worst), and so do the accuracies against
the exact Riemann solution (about 99.2 % and 98.5 % for OReg, 94 % for BGK)."""
import math
import sys

import numpy as np
import pytest

import oracle
from test_oracle_pins import isothermal_riemann_density, walled_shocktube

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("collision", ["oreg", "bgk"])
@pytest.mark.parametrize("theta,nu", [(0.35, 1e-5), (0.4, 1e-9)])
def test_walled_shocktube_gpu_matches_oracle(collision, theta, nu):
    from paper_2501_16000_amd import oreg
    nx, steps = 800, 500
    print(f"[shocktube] {collision} theta={theta} nu={nu}", flush=True)
    acc_ref, tv_ref, r_ref = walled_shocktube(collision, theta, nu, nx, steps)
    tau = nu / theta + 0.5
    x = np.arange(nx)
    rho = np.where(x < nx // 2, 1.5, 0.75)[None, :].astype(float)
    with oreg.Lattice(nx, 1, tau, theta, collision=collision, boundary_x="bounceback") as L:
        L.init(rho, 0 * rho, 0 * rho)
        L.step(steps)
        r = L.moments()[0, 0]
    ref = isothermal_riemann_density(x.astype(float), steps, 1.5, 0.75, math.sqrt(theta),
                                     (nx - 1) / 2)
    fl = slice(1, nx - 1)
    acc = 1 - np.linalg.norm(r[fl] - ref[fl]) / np.linalg.norm(ref[fl])
    print(f"  accuracy GPU {acc * 100:.3f} % oracle {acc_ref * 100:.3f} %; "
          f"max |rho - rho_oracle| {np.abs(r - r_ref).max():.2e}", flush=True)
    assert np.abs(r - r_ref).max() < 1e-12
    assert abs(acc - acc_ref) < 1e-12

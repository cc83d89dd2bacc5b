"""Shifted reduced-precision storage (FP32 / FP16 / BF16 of f_i - w_i rho0,
FP32 collision) against the FP64 oracle.

These are not bit-parity tests: the stored values are rounded to nearest even
on every step.  Each test states the error of a physical result against the
oracle and asserts the bound measured for it (with margin):
  * the rotated shear wave (128^2, theta = 1/3, tau = 0.8, u0 = 0.01, 500
    steps): decay rate nu~ relative to the oracle's;
  * the periodic shocktube (16384 x 4, rho 1.5 | 0.75, tau = 0.55, 4000
    steps, rho0 = 1.125): y-averaged density profile, L2 and Linf;
  * the polynomial-equilibrium random smooth flow (512^2 stand-in of the
    8192^2 workload, tau = 0.7, 500 steps): kinetic energy history; and the
    8192^2 workload itself against the GPU FP64 run.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2501_16000_amd import workloads

pytestmark = pytest.mark.gpu

STORAGES = ["f32s", "f16s", "bf16s"]


def lib():
    from paper_2501_16000_amd import oreg
    return oreg


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def amplitude(m, n):
    e_perp, phase = workloads.shear_wave_projection(n)
    up = e_perp[0] * m[1] + e_perp[1] * m[2]
    return 2.0 / (n * n) * abs((up * phase).sum())


def decay_rate(amps, ts):
    sel = ts >= 20
    return -np.polyfit(ts[sel], np.log(amps[sel]), 1)[0]


_SHEAR = {}


def shear_reference():
    if "ref" not in _SHEAR:
        n, tau, theta = 128, 0.8, 1 / 3
        rho, ux, uy = workloads.shear_wave(n, 0.01)
        f = oracle.init("guided", theta, rho, ux, uy)
        amps, ts = [amplitude(oracle.moments(f), n)], [0]
        for t in range(25, 501, 25):
            f = oracle.run(f, 25, tau, theta)
            amps.append(amplitude(oracle.moments(f), n))
            ts.append(t)
        _SHEAR["ref"] = (np.array(amps), np.array(ts), oracle.moments(f))
    return _SHEAR["ref"]


# decay-rate error bounds (relative to the oracle's nu~), measured with margin
# (measured: 7.2e-6, 1.1e-3, 1.4e-2).  In FP16 the stored non-equilibrium part
# of this small wave (u0 = 0.01) is a few units of the last place, so the
# error is rounding noise that moves with the FP32 evaluation order of the
# collision: CPU runs of two orders of the same collision on six waves
# (N 64-192, tau 0.6-0.9, u0 0.01-0.03) gave 9e-5 to 4e-3 for both, and 1e-4
# or 9e-4 on this one.
SHEAR_BOUND = {"f32s": 3e-5, "f16s": 2e-3, "bf16s": 3e-2}


@pytest.mark.parametrize("storage", STORAGES)
def test_shear_wave_decay_rate(storage):
    oreg = lib()
    n, tau, theta = 128, 0.8, 1 / 3
    say(f"[precision] shear wave 128^2 {storage}")
    amps_ref, ts, m_ref = shear_reference()
    rho, ux, uy = workloads.shear_wave(n, 0.01)
    with oreg.Lattice(n, n, tau, theta, storage=storage, rho0=1.0) as L:
        L.init(rho, ux, uy)
        amps = [amplitude(L.moments(), n)]
        for _ in range(20):
            L.step(25)
            amps.append(amplitude(L.moments(), n))
        m = L.moments()
        d = L.diagnostics()
    k_ref = decay_rate(amps_ref, ts)
    k = decay_rate(np.array(amps), ts)
    err = abs(k / k_ref - 1)
    du = np.max(np.abs(m[1:] - m_ref[1:])) / 0.01
    say(f"  decay-rate rel error {err:.3e}; max |u - u_ref|/u0 at step 500 {du:.3e}; "
        f"mass drift {abs(d[0] - n * n) / (n * n):.3e}")
    assert err < SHEAR_BOUND[storage]


_TUBE = {}


def tube_reference():
    if "ref" not in _TUBE:
        nx, ny, tau, theta, steps = 16384, 4, 0.55, 1 / 3, 4000
        rho, ux, uy = workloads.shocktube(nx, ny)
        f = oracle.run(oracle.init("guided", theta, rho, ux, uy), steps, tau, theta)
        _TUBE["ref"] = oracle.moments(f)[0].mean(axis=0)
    return _TUBE["ref"]


# FP64: 4000 steps across a shock, so the parity bound of 100 steps is widened.
# Measured: F32S 8.3e-6 / 5.2e-4, F16S 2.4e-3 / 2.4e-2, BF16S 1.5e-2 / 5.0e-2.
TUBE_BOUND = {"f64": (1e-12, 2e-11), "f32s": (2e-5, 1e-3), "f16s": (4e-3, 4e-2),
              "bf16s": (5e-2, 1.2e-1)}


@pytest.mark.parametrize("storage", ["f64"] + STORAGES)
def test_shocktube_density_profile(storage):
    oreg = lib()
    nx, ny, tau, theta, steps = 16384, 4, 0.55, 1 / 3, 4000
    say(f"[precision] shocktube 16384x4 {storage}, {steps} steps")
    ref = tube_reference()
    rho, ux, uy = workloads.shocktube(nx, ny)
    with oreg.Lattice(nx, ny, tau, theta, storage=storage, rho0=1.125) as L:
        L.init(rho, ux, uy)
        L.step(steps)
        prof = L.density_profile()
        m = L.moments()
    # the state stays independent of y (symmetry of the initial data)
    assert np.max(np.abs(m[0] - m[0][0:1])) <= (0.0 if storage == "f64" else 1e-2)
    l2 = np.linalg.norm(prof - ref) / np.linalg.norm(ref)
    linf = np.max(np.abs(prof - ref))
    say(f"  density profile rel L2 {l2:.3e}, Linf {linf:.3e}")
    b2, binf = TUBE_BOUND[storage]
    assert l2 < b2 and linf < binf


KE_BOUND = {"f32s": 2e-4, "f16s": 3e-4, "bf16s": 3e-2}


@pytest.mark.parametrize("storage", STORAGES)
def test_polynomial_random_flow_kinetic_energy(storage):
    oreg = lib()
    n, tau, theta, steps = 512, 0.7, 1 / 3, 500
    say(f"[precision] poly2 random smooth flow 512^2 {storage}")
    rho, ux, uy = workloads.smooth_random_velocity(n, umax=0.03, seed=2501)
    f = oracle.init("poly2", theta, rho, ux, uy)
    ke_ref = [oracle.diagnostics(f, theta)[3]]
    for _ in range(5):
        f = oracle.run(f, steps // 5, tau, theta, "poly2")
        ke_ref.append(oracle.diagnostics(f, theta)[3])
    with oreg.Lattice(n, n, tau, theta, equilibrium="poly2", storage=storage) as L:
        L.init(rho, ux, uy)
        ke = [L.diagnostics()[3]]
        for _ in range(5):
            L.step(steps // 5)
            ke.append(L.diagnostics()[3])
    ke, ke_ref = np.array(ke), np.array(ke_ref)
    err = np.max(np.abs(ke - ke_ref)) / ke_ref[0]
    decay_err = abs((ke[-1] - ke[0]) / (ke_ref[-1] - ke_ref[0]) - 1)
    say(f"  max |KE - KE_ref| / KE(0) {err:.3e}; relative error of the KE decay {decay_err:.3e}")
    assert err < KE_BOUND[storage]


def test_f64_kinetic_energy_matches_oracle():
    oreg = lib()
    n, tau, theta = 256, 0.7, 1 / 3
    rho, ux, uy = workloads.smooth_random_velocity(n, umax=0.03, seed=7)
    f = oracle.run(oracle.init("poly2", theta, rho, ux, uy), 100, tau, theta, "poly2")
    with oreg.Lattice(n, n, tau, theta, equilibrium="poly2") as L:
        L.init(rho, ux, uy)
        L.step(100)
        d = L.diagnostics()
    np.testing.assert_allclose(d[3], oracle.diagnostics(f, theta)[3], rtol=1e-12)


# The full-size polynomial workload: 8192^2, tau = 0.7, 500 steps.  The
# oracle cannot run it (33.6 G node updates), so the GPU FP64 run stands in
# for it: the FP64 sweep equals the oracle element by element in the parity
# tests (within 1e-12 after 100 steps, sampled at 4096^2 and 32768^2) and in
# the kinetic energy above.  Over 500 steps the modes (at most 8 per axis on
# 8192) lose only about 2e-3 of their energy, so the decay itself is an
# ill-conditioned difference; both errors are reported.
KE_BOUND_8192 = {"f32s": 3e-4, "f16s": 1e-3, "bf16s": 2e-3}


def test_polynomial_random_flow_8192_full_size():
    oreg = lib()
    n, tau, theta, steps = 8192, 0.7, 1 / 3, 500
    rho, ux, uy = workloads.smooth_random_velocity(n, umax=0.03, seed=2501)
    ke = {}
    for storage in ["f64"] + STORAGES:
        say(f"[precision] poly2 random smooth flow 8192^2 {storage}")
        with oreg.Lattice(n, n, tau, theta, equilibrium="poly2", storage=storage) as L:
            L.init(rho, ux, uy)
            h = [L.diagnostics()[3]]
            for _ in range(5):
                L.step(steps // 5)
                h.append(L.diagnostics()[3])
        ke[storage] = np.array(h)
    ref = ke["f64"]
    say(f"  FP64 kinetic energy {ref[0]:.6e} -> {ref[-1]:.6e} (decay {1 - ref[-1] / ref[0]:.3e})")
    errs = {}
    for storage in STORAGES:
        errs[storage] = np.max(np.abs(ke[storage] - ref)) / ref[0]
        decay_err = abs((ke[storage][-1] - ke[storage][0]) / (ref[-1] - ref[0]) - 1)
        say(f"  {storage}: max |KE - KE_f64| / KE(0) {errs[storage]:.3e}; "
            f"relative error of the KE decay {decay_err:.3e}")
    for storage in STORAGES:
        assert errs[storage] < KE_BOUND_8192[storage], storage

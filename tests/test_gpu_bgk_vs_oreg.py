"""Lattice BGK (Eq. 1) against OReg (Eqs. 6, 7) on the shear waves of Sec. IV.

Eq. (18): a wave of amplitude A0 = 1e-3 (Sec. IV) on a 32 x 32 periodic grid with a mean
flow u_y = Ma sqrt(theta), theta = 1/3, nu = 0.01 (tau = 0.53), either
axis-aligned (wave vector along y, perturbation u_x) or rotated by pi/4
(wave vector along (-1, 1), perturbation along (1, 1)).  The measured
viscosity nu~ comes from the decay of the wave's Fourier amplitude.

Asserted:
  * the GPU library's nu~ equals the FP64 oracle's for every case (both
    schemes, both waves, Ma in {0, 0.2, 0.4});
  * Fig. 2a: on the axis-aligned wave both schemes give nu~/nu = 1 within
    0.5 % at every Mach number;
  * at Ma = 0 both schemes give nu~/nu = 1 within 0.5 % on the rotated wave.
Reported, not asserted against the paper: with a mean flow the rotated wave
gives nu~/nu away from 1 for both schemes (OReg 1.21 and 1.65, BGK 0.97 and
0.88 at Ma = 0.2 and 0.4), so this implementation of Eqs. (6), (7) does not
reproduce the statement of Fig. 2b that only OReg recovers nu there; see the
design notes for the reading.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2501_16000_amd import workloads

pytestmark = pytest.mark.gpu

N, TAU, THETA, STEPS, EVERY = 32, 0.53, 1 / 3, 2000, 50


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def wave(rotated, ma):
    return workloads.paper_shear_wave(N, 1e-3, ma, THETA, rotated=rotated, lx=N)


def projector(rotated, ma):
    y, x = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    u0 = ma * math.sqrt(THETA)
    if rotated:
        return (np.exp(-2j * np.pi * (-x + y) / N), 2 * (2 * np.pi / N) ** 2,
                lambda m: (m[1] + (m[2] - u0)) / math.sqrt(2))
    return np.exp(-2j * np.pi * y / N), (2 * np.pi / N) ** 2, lambda m: m[1]


def nu_ratio(amps):
    ts = np.arange(0, STEPS + 1, EVERY)
    sel = ts >= 200
    return -np.polyfit(ts[sel], np.log(amps[sel]), 1)[0]


def oracle_amps(collision, rotated, ma):
    ph, k2, comp = projector(rotated, ma)
    f = oracle.init("guided", THETA, *wave(rotated, ma))
    amps = []
    for t in range(0, STEPS + 1, EVERY):
        if t:
            f = oracle.run(f, EVERY, TAU, THETA, collision=collision)
        amps.append(abs((comp(oracle.moments(f)) * ph).sum()))
    return np.array(amps), k2


def gpu_amps(collision, rotated, ma):
    from paper_2501_16000_amd import oreg
    ph, k2, comp = projector(rotated, ma)
    amps = []
    with oreg.Lattice(N, N, TAU, THETA, collision=collision) as L:
        L.init(*wave(rotated, ma))
        for t in range(0, STEPS + 1, EVERY):
            if t:
                L.step(EVERY)
            amps.append(abs((comp(L.moments()) * ph).sum()))
    return np.array(amps)


@pytest.mark.parametrize("rotated", [False, True])
@pytest.mark.parametrize("ma", [0.0, 0.2, 0.4])
def test_viscosity_bgk_and_oreg(rotated, ma):
    nu = THETA * (TAU - 0.5)
    out = {}
    for coll in ("oreg", "bgk"):
        ref, k2 = oracle_amps(coll, rotated, ma)
        got = gpu_amps(coll, rotated, ma)
        r_ref = nu_ratio(ref) / k2 / nu
        r_gpu = nu_ratio(got) / k2 / nu
        assert abs(r_gpu - r_ref) < 1e-6 * r_ref
        out[coll] = r_gpu
    say(f"[bgk vs oreg] {'rotated' if rotated else 'axis'} Ma={ma}: "
        f"nu~/nu OReg {out['oreg']:.4f}  BGK {out['bgk']:.4f}")
    if not rotated or ma == 0.0:
        assert abs(out["oreg"] - 1) < 5e-3
        assert abs(out["bgk"] - 1) < 5e-3

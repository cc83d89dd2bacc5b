"""The shear-wave viscosities of Fig. 2 (Sec. IV) from the spectrum of the
discrete update linearized about the mean flow, against the decay the
oracle's time evolution shows.

For a small wave on a uniform state (rho = 1, u = (0, Ma sqrt(theta))) one
time step multiplies each Fourier mode by M(k) = diag(exp(-i k.c_i)) J, with
J the Jacobian of one collision (Eq. (7) with Eq. (6), or Eq. (1)) at the
state's equilibrium.  The shear eigenvalue lambda gives nu~ = -ln|lambda| /
|k|^2; the test checks that it equals the rate fitted to the oracle's
decaying wave (so the numbers reported for Fig. 2 are what the discrete
equations do, not an artefact of the fit), and records them: on the
axis-aligned wave both schemes give nu~/nu = 1.002-1.003 at every Mach
number; on the pi/4-rotated wave OReg gives 1.205 and 1.651 and BGK 0.970
and 0.881 at Ma = 0.2 and 0.4 (tau = 0.53, theta = 1/3, nu = 0.01, N = 32).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2501_16000_amd import workloads

C = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)],
             dtype=float)
N, TAU, THETA = 32, 0.53, 1 / 3
NU = THETA * (TAU - 0.5)


def jacobian(collision, u, tau=TAU):
    f0 = oracle.equilibrium("guided", THETA, 1.0, u[0], u[1])
    J = np.zeros((9, 9))
    h = 1e-7
    for j in range(9):
        e = np.zeros(9)
        e[j] = h
        J[:, j] = (oracle.collide_cell("guided", tau, THETA, f0 + e, collision)
                   - oracle.collide_cell("guided", tau, THETA, f0 - e, collision)) / (2 * h)
    return J


def wave_vector(rotated, n=N):
    return 2 * math.pi / n * (np.array([-1.0, 1.0]) if rotated else np.array([0.0, 1.0]))


def spectral_ratio(collision, rotated, ma, tau=TAU, n=N):
    nu = THETA * (tau - 0.5)
    u = np.array([0.0, ma * math.sqrt(THETA)])
    k = wave_vector(rotated, n)
    ev = np.linalg.eigvals(np.diag(np.exp(-1j * (C @ k))) @ jacobian(collision, u, tau))
    target = np.exp(-1j * (k @ u) - nu * (k @ k))   # advected shear mode at nu
    lam = ev[np.argmin(np.abs(ev - target))]
    return -math.log(abs(lam)) / (k @ k) / nu


def fitted_ratio(collision, rotated, ma, steps=1200, every=50):
    fields = workloads.paper_shear_wave(N, 1e-3, ma, THETA, rotated=rotated, lx=N)
    y, x = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    k = wave_vector(rotated)
    phase = np.exp(-1j * (k[0] * x + k[1] * y))
    u0 = ma * math.sqrt(THETA)
    if rotated:
        comp = lambda m: (m[1] + (m[2] - u0)) / math.sqrt(2)
    else:
        comp = lambda m: m[1]
    f = oracle.init("guided", THETA, *fields)
    ts, amps = [], []
    for t in range(0, steps + 1, every):
        if t:
            f = oracle.run(f, every, TAU, THETA, collision=collision)
        amps.append(abs((comp(oracle.moments(f)) * phase).sum()))
        ts.append(t)
    ts, amps = np.array(ts), np.array(amps)
    sel = ts >= 200
    return -np.polyfit(ts[sel], np.log(amps[sel]), 1)[0] / (k @ k) / NU


@pytest.mark.parametrize("rotated,ma", [(False, 0.2), (True, 0.0), (True, 0.2), (True, 0.4)])
@pytest.mark.parametrize("collision", ["oreg", "bgk"])
def test_fitted_decay_equals_linear_spectrum(collision, rotated, ma):
    s = spectral_ratio(collision, rotated, ma)
    f = fitted_ratio(collision, rotated, ma)
    assert abs(f - s) < 2e-3 * s


def test_recorded_fig2_values():
    got = {(c, r, m): round(spectral_ratio(c, r, m), 3) for c in ("oreg", "bgk")
           for r in (False, True) for m in (0.0, 0.2, 0.4)}
    for m in (0.0, 0.2, 0.4):
        assert abs(got[("oreg", False, m)] - 1) < 5e-3 and abs(got[("bgk", False, m)] - 1) < 5e-3
    assert abs(got[("oreg", True, 0.0)] - 1) < 1e-3 and abs(got[("bgk", True, 0.0)] - 1) < 1e-3
    assert got[("oreg", True, 0.2)] == pytest.approx(1.205, abs=2e-3)
    assert got[("oreg", True, 0.4)] == pytest.approx(1.651, abs=2e-3)
    assert got[("bgk", True, 0.2)] == pytest.approx(0.970, abs=2e-3)
    assert got[("bgk", True, 0.4)] == pytest.approx(0.881, abs=2e-3)


# Where Fig. 2b's claim holds.  nu~/nu on the pi/4-rotated wave with mean flow
# u_y = Ma sqrt(theta), theta = 1/3, from the linearized update (OReg / BGK):
#
#   tau    Ma=0.1          Ma=0.2          Ma=0.3          Ma=0.4
#   0.51   1.177 / 0.993   1.678 / 0.970   2.408 / 0.933   3.211 / 0.881
#   0.53   1.054 / 0.993   1.205 / 0.970   1.422 / 0.933   1.651 / 0.881
#   0.6    1.010 / 0.993   1.038 / 0.971   1.073 / 0.933   1.100 / 0.881
#   0.7    1.000 / 0.993   0.999 / 0.971   0.993 / 0.934   0.975 / 0.881
#   0.8    0.997 / 0.994   0.985 / 0.971   0.964 / 0.934   0.928 / 0.882
#   1.0    0.996 / 0.996   0.973 / 0.973   0.935 / 0.935   0.882 / 0.882
#
# BGK's error depends on Ma and hardly on tau (its stress relaxes at 1/tau whatever the
# flow); OReg's grows as tau -> 1/2, where the factor of Eq. (12b) acting on
# the diagonal stress times (1 - 1/tau) shifts the effective relaxation
# time.  OReg is the closer one from a crossover tau_c = 0.59-0.62 up to
# tau = 1 (where 1 - 1/tau = 0 and both updates stream the equilibrium), and
# BGK below it: the paper's nu = 0.01 at theta = 1/3 (tau = 0.53) lies in the
# regime where the claim does not hold for this reading of Eqs. (6), (7).
# The ratios do not depend on the wave length (long-wave limit).
TAUS_MAP = [0.51, 0.53, 0.6, 0.7, 0.8, 1.0]
MAS_MAP = [0.1, 0.2, 0.3, 0.4]


def crossover_tau(ma, lo=0.52, hi=0.7):
    """tau where |OReg - 1| = |BGK - 1| on the rotated wave (bisection)."""
    def d(t):
        return abs(spectral_ratio("oreg", True, ma, t) - 1) - abs(spectral_ratio("bgk", True, ma, t) - 1)
    assert d(lo) > 0 > d(hi)
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        if d(mid) > 0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def test_fig2b_regime_map():
    grid = {(t, m): (spectral_ratio("oreg", True, m, t), spectral_ratio("bgk", True, m, t))
            for t in TAUS_MAP for m in MAS_MAP}
    for m in MAS_MAP:
        for t in TAUS_MAP:
            o, b = grid[(t, m)]
            if t <= 0.53:
                assert abs(b - 1) < abs(o - 1), (t, m, o, b)  # BGK closer near tau = 1/2
            elif t in (0.7, 0.8):
                assert abs(o - 1) < abs(b - 1), (t, m, o, b)  # OReg closer: Fig. 2b's claim
            elif t == 1.0:
                assert o == pytest.approx(b, abs=1e-6)         # 1 - 1/tau = 0: same update
        tc = crossover_tau(m)
        assert 0.58 < tc < 0.63, (m, tc)
    # BGK's ratio is independent of tau; OReg's is monotone in tau at fixed Ma
    for m in MAS_MAP:
        bs = [grid[(t, m)][1] for t in TAUS_MAP]
        assert max(bs) - min(bs) < 5e-3
        os_ = [grid[(t, m)][0] for t in TAUS_MAP]
        assert all(a > c for a, c in zip(os_, os_[1:]))
    # the pinned values of the table above
    assert grid[(0.7, 0.4)][0] == pytest.approx(0.975, abs=2e-3)
    assert grid[(0.6, 0.2)][0] == pytest.approx(1.038, abs=2e-3)
    assert grid[(0.51, 0.4)][0] == pytest.approx(3.211, abs=5e-3)


def test_fig2b_ratios_independent_of_wavelength():
    for coll in ("oreg", "bgk"):
        for ma in (0.2, 0.4):
            a = spectral_ratio(coll, True, ma, 0.53, n=32)
            b = spectral_ratio(coll, True, ma, 0.53, n=200)
            assert abs(a - b) < 2e-3 * a


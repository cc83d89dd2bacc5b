"""GPU-vs-oracle parity of the D3Q27 sweep (lb3_* entry points of liboreg.so).

Both sides start from the same seeded inputs and advance the same number of
steps; the comparison is element by element on the pre-collision populations.
Tolerance: 1e-12 relative per population after 100 steps in FP64 (only the
rounding order differs).  At the 256^3 benchmark size the oracle recomputes
sampled nodes one by one on the (2n+1)^3 periodic patch that determines them
after n steps.  Reduced-precision storage is checked by the error of the
shear-wave decay rate against the FP64 oracle.
"""
import itertools
import sys

import numpy as np
import pytest

from oracle import d3q27 as o3
from paper_2501_16000_amd import workloads

pytestmark = pytest.mark.gpu

RTOL = 1e-12


def lib():
    from paper_2501_16000_amd import oreg3
    return oreg3


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(got, ref):
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)))


def random_populations(eq, theta, shape, seed, amp=0.02, u=0.05):
    rho = 1.0 + 0.1 * workloads.noise(shape, seed)
    us = [u * workloads.noise(shape, seed + k) for k in (1, 2, 3)]
    f = o3.init(eq, theta, rho, *us)
    return f * (1.0 + workloads.noise(f.shape, seed + 4, amp))


CASES = [
    # (nx, ny, nz, eq, theta, tau, collision)
    (8, 8, 8, "guided", 1 / 3, 0.8, "oreg"),
    (70, 9, 7, "guided", 1 / 3, 0.8, "oreg"),     # two 64-node segments, ragged tail of 6
    (70, 9, 7, "guided", 0.35, 0.51, "oreg"),
    (70, 9, 7, "guided", 0.4, 1.0, "oreg"),
    (70, 9, 7, "poly2", 1 / 3, 0.51, "oreg"),
    (33, 5, 4, "guided", 0.35, 0.7, "bgk"),
    (33, 5, 4, "poly2", 1 / 3, 0.9, "bgk"),
    (130, 3, 2, "guided", 1 / 3, 0.6, "oreg"),    # three segments
    (1, 1, 1, "guided", 1 / 3, 0.8, "oreg"),
    (1, 6, 5, "guided", 1 / 3, 0.7, "oreg"),
    (5, 1, 1, "guided", 0.4, 0.7, "oreg"),
    (1, 1, 40, "guided", 1 / 3, 0.55, "oreg"),
    (64, 1, 3, "guided", 1 / 3, 0.75, "oreg"),    # exactly one segment
]


@pytest.mark.parametrize("nx,ny,nz,eq,theta,tau,coll", CASES)
def test_parity_random_populations(nx, ny, nz, eq, theta, tau, coll):
    oreg3 = lib()
    shape = (nz, ny, nx)
    f0 = random_populations(eq, theta, shape, 1000 + nx + 7 * ny + 31 * nz)
    say(f"[d3q27] {nx}x{ny}x{nz} {eq} theta={theta:.4f} tau={tau} {coll}: 100 steps")
    ref = o3.run(f0, 100, tau, theta, eq, collision=coll)
    with oreg3.Lattice3(nx, ny, nz, tau, theta, equilibrium=eq, collision=coll) as L:
        L.set_populations(f0)
        np.testing.assert_allclose(L.populations(), f0, rtol=0, atol=0)
        L.step(100)
        assert L.time == 100
        got = L.populations()
        err = rel_err(got, ref)
        say(f"  max relative error {err:.3e}")
        assert err <= RTOL
        np.testing.assert_allclose(L.moments(), o3.moments(ref), rtol=0, atol=1e-13)
        d, dref = L.diagnostics(), o3.diagnostics(ref, theta if eq == "guided" else 1 / 3)
        np.testing.assert_allclose(d[:6], dref[:6], rtol=1e-12, atol=1e-12)
        assert d[6] == 0


def test_parity_shear_wave_from_fields():
    oreg3 = lib()
    n, tau, theta = 32, 0.8, 1 / 3
    fields = workloads.shear_wave3(n, 0.05)
    say("[d3q27] 32^3 shear wave from fields, 100 steps")
    ref = o3.run(o3.init("guided", theta, *fields), 100, tau, theta)
    with oreg3.Lattice3(n, n, n, tau, theta) as L:
        L.init(*fields)
        L.step(100)
        assert rel_err(L.populations(), ref) <= RTOL
        np.testing.assert_allclose(L.moments(), o3.moments(ref), rtol=0, atol=1e-13)


def patch(a, x0, y0, z0, h):
    nz, ny, nx = a.shape[-3:]
    zs = np.arange(z0 - h, z0 + h + 1) % nz
    ys = np.arange(y0 - h, y0 + h + 1) % ny
    xs = np.arange(x0 - h, x0 + h + 1) % nx
    return a[..., zs[:, None, None], ys[None, :, None], xs[None, None, :]]


@pytest.mark.parametrize("tau", [0.51, 0.6, 1.0])
def test_parity_sampled_256_fp64(tau):
    """The 256^3 FP64 throughput box (shear wave normal to (1, 1, 1), u0 = 0.05):
    corners, faces (periodic wrap), segment boundaries and random interior nodes
    after 20 steps, each recomputed by the oracle on its 41^3 dependency patch."""
    oreg3 = lib()
    n, theta, steps = 256, 1 / 3, 20
    say(f"[d3q27] 256^3 FP64 tau={tau}: sampled nodes after {steps} steps")
    fields = workloads.shear_wave3(n, 0.05)
    with oreg3.Lattice3(n, n, n, tau, theta) as L:
        L.init(*fields)
        L.step(steps)
        m = L.moments()
        d = L.diagnostics()
    rng = np.random.default_rng(8)
    samples = [(x, y, z) for x, y, z in itertools.product((0, n - 1), repeat=3)]
    samples += [(63, 64, 17), (64, 0, 255), (n // 2, n // 2, 0)]
    samples += [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(4)]
    F = np.stack(fields)
    worst = 0.0
    for (x0, y0, z0) in samples:
        pf = patch(F, x0, y0, z0, steps)
        fp = o3.run(o3.init("guided", theta, *pf), steps, tau, theta)
        mp = o3.moments(fp)[:, steps, steps, steps]
        worst = max(worst, float(np.max(np.abs(m[:, z0, y0, x0] - mp))))
    say(f"  max |moment difference| over {len(samples)} nodes: {worst:.3e}")
    assert worst < 1e-13
    assert abs(d[0] - n ** 3) < 1e-9 * n ** 3
    assert d[6] == 0


def test_fixed_point_at_full_size():
    oreg3 = lib()
    n = 256
    say("[d3q27] uniform state fixed point, 256^3, 10 steps")
    with oreg3.Lattice3(n, n, n, 0.6, 0.35) as L:
        full = lambda v: np.full((n, n, n), v)
        L.init(full(1.2), full(0.04), full(-0.02), full(0.03))
        L.step(10)
        m = L.moments()
    for k, v in enumerate((1.2, 0.04, -0.02, 0.03)):
        assert np.max(np.abs(m[k] - v)) < 1e-14


def test_determinism_and_checkpoint_resume():
    oreg3 = lib()
    shape, tau, theta = (11, 13, 70), 0.7, 1 / 3
    f0 = random_populations("guided", theta, shape, 11)
    say("[d3q27] determinism and checkpoint/resume 70x13x11")
    with oreg3.Lattice3(70, 13, 11, tau, theta) as A, oreg3.Lattice3(70, 13, 11, tau, theta) as B:
        A.set_populations(f0)
        A.step(40)
        fa = A.populations()
        B.set_populations(f0)
        B.step(40)
        np.testing.assert_array_equal(B.populations(), fa)
        B.set_populations(f0)
        B.step(20)
        B.set_populations(B.populations())
        B.step(20)
        np.testing.assert_array_equal(B.populations(), fa)
        np.testing.assert_array_equal(A.diagnostics(), B.diagnostics())


def test_axis_permutation_commutes():
    """Swapping the x and y axes of the initial state commutes with the sweep
    (to rounding: the kernel sums populations line by line along x)."""
    oreg3 = lib()
    n, nz, tau, theta = 24, 10, 0.62, 1 / 3
    f0 = random_populations("guided", theta, (nz, n, n), 21)
    c = o3.velocities()
    idx = {tuple(v): i for i, v in enumerate(c)}

    def swap(f):
        g = np.empty_like(f)
        for i, v in enumerate(c):
            g[idx[(v[1], v[0], v[2])]] = np.swapaxes(f[i], 1, 2)
        return g

    say("[d3q27] x <-> y permutation, 24x24x10, 30 steps")
    with oreg3.Lattice3(n, n, nz, tau, theta) as L:
        L.set_populations(f0)
        L.step(30)
        a = L.populations()
        L.set_populations(swap(f0))
        L.step(30)
        b = L.populations()
    assert rel_err(b, swap(a)) < 1e-13


@pytest.mark.parametrize("storage,bound", [("f32s", 5e-5), ("f16s", 1e-3), ("bf16s", 5e-3)])
def test_reduced_precision_decay_rate(storage, bound):
    """Shifted FP32/FP16/BF16 storage: the decay rate of the 3D shear wave
    (u0 = 0.01, 32^3, tau = 0.8) stays within the stated relative error of the
    FP64 oracle's; mass is conserved to the storage's rounding."""
    oreg3 = lib()
    n, tau, theta, every, steps = 32, 0.8, 1 / 3, 40, 320
    fields = workloads.shear_wave3(n, 0.01)
    e, phase = workloads.shear_wave3_projection(n)
    amp = lambda m: abs(((e[0] * m[1] + e[1] * m[2] + e[2] * m[3]) * phase).sum())
    f = o3.init("guided", theta, *fields)
    ts, ref, got = [0], [amp(o3.moments(f))], []
    with oreg3.Lattice3(n, n, n, tau, theta, storage=storage) as L:
        L.init(*fields)
        got.append(amp(L.moments()))
        for t in range(every, steps + 1, every):
            f = o3.run(f, every, tau, theta)
            L.step(every)
            ts.append(t)
            ref.append(amp(o3.moments(f)))
            got.append(amp(L.moments()))
        d = L.diagnostics()
    k_ref = -np.polyfit(ts[1:], np.log(ref[1:]), 1)[0]
    k_got = -np.polyfit(ts[1:], np.log(got[1:]), 1)[0]
    err = abs(k_got / k_ref - 1)
    say(f"[d3q27] {storage}: decay-rate relative error {err:.2e}, "
        f"mass error {abs(d[0] - n ** 3) / n ** 3:.2e}")
    assert err < bound
    assert abs(d[0] - n ** 3) < {"f32s": 1e-5, "f16s": 1e-3, "bf16s": 1e-2}[storage] * n ** 3


def test_viscosity_gpu_equals_oracle():
    """nu~ of the 3D shear wave from the GPU equals the oracle's (16^3, 160 steps)."""
    oreg3 = lib()
    n, tau, theta = 16, 0.8, 1 / 3
    fields = workloads.shear_wave3(n, 1e-3)
    e, phase = workloads.shear_wave3_projection(n)
    amp = lambda m: abs(((e[0] * m[1] + e[1] * m[2] + e[2] * m[3]) * phase).sum())
    f = o3.init("guided", theta, *fields)
    ref, got = [], []
    with oreg3.Lattice3(n, n, n, tau, theta) as L:
        L.init(*fields)
        for _ in range(8):
            f = o3.run(f, 20, tau, theta)
            L.step(20)
            ref.append(amp(o3.moments(f)))
            got.append(amp(L.moments()))
    ts = np.arange(1, 9) * 20
    k_ref = np.polyfit(ts, np.log(ref), 1)[0]
    k_got = np.polyfit(ts, np.log(got), 1)[0]
    assert abs(k_got / k_ref - 1) < 1e-9


def test_error_paths_on_device():
    oreg3 = lib()
    from paper_2501_16000_amd import oreg
    with oreg3.Lattice3(6, 5, 4, 0.8) as L:
        with pytest.raises(oreg.LBError) as e:
            L.step(1)
        assert e.value.status == oreg.LB_ESTATE
        bad = np.ones((4, 5, 6))
        bad[1, 2, 3] = np.nan
        z = np.zeros((4, 5, 6))
        with pytest.raises(oreg.LBError) as e:
            L.init(bad, z, z, z)
        assert e.value.status == oreg.LB_EINVAL
        with pytest.raises(oreg.LBError) as e:
            L.init(-np.ones((4, 5, 6)), z, z, z)
        assert e.value.status == oreg.LB_EINVAL
        L.init(np.ones((4, 5, 6)), z, z, z)
        with pytest.raises(oreg.LBError) as e:
            L.step(-1)
        assert e.value.status == oreg.LB_EINVAL
        f = L.populations()
        f[3, 0, 0, 0] = np.inf
        with pytest.raises(oreg.LBError):
            L.set_populations(f)
        L.step(0)
        assert L.time == 0


def test_device_init_and_moments_with_torch():
    import torch
    oreg3 = lib()
    n, tau, theta = 20, 0.7, 1 / 3
    fields = workloads.shear_wave3(n, 0.03)
    say("[d3q27] init and moments through torch device tensors")
    s = torch.cuda.Stream()
    with oreg3.Lattice3(n, n, n, tau, theta, stream=s) as A, oreg3.Lattice3(n, n, n, tau, theta) as B:
        dev = [torch.from_numpy(a).cuda() for a in fields]
        torch.cuda.synchronize()
        A.init(*dev)
        B.init(*fields)
        A.step(10)
        B.step(10)
        out = torch.empty((4, n, n, n), dtype=torch.float64, device="cuda")
        A.moments(out=out)
        A.sync()
        np.testing.assert_array_equal(out.cpu().numpy(), B.moments())
        bad = dev[0].clone()
        bad[0, 0, 0] = float("nan")
        from paper_2501_16000_amd import oreg
        with pytest.raises(oreg.LBError) as e:
            A.init(bad, *dev[1:])
        assert e.value.status == oreg.LB_EINVAL


@pytest.mark.parametrize("storage,bound", [("f32s", 1e-7), ("f16s", 1e-5), ("bf16s", 1e-4)])
def test_reduced_precision_ragged_box(storage, bound):
    """Shifted storage on a box with several 128-node row segments, a ragged
    tail and periodic x edges (the 16-bit formats take two nodes per lane):
    moments after 50 steps stay within the storage's rounding of the FP64
    oracle's."""
    oreg3 = lib()
    nx, ny, nz, tau, theta = 301, 9, 7, 0.7, 1 / 3
    shape = (nz, ny, nx)
    rho = 1.0 + 0.02 * workloads.noise(shape, 61)
    us = [0.02 * workloads.noise(shape, 62 + k) for k in range(3)]
    ref = o3.moments(o3.run(o3.init("guided", theta, rho, *us), 50, tau, theta))
    with oreg3.Lattice3(nx, ny, nz, tau, theta, storage=storage) as L:
        L.init(rho, *us)
        L.step(50)
        m = L.moments()
    err = float(np.max(np.abs(m - ref)))
    say(f"[d3q27] {storage} ragged 301x9x7: max |moment error| {err:.2e}")
    assert err < bound

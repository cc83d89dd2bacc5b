"""GPU-vs-oracle parity of the FP64 sweep (through the C ABI of liboreg.so).

Both sides start from the same seeded inputs (``paper_2501_16000_amd.workloads``
or oracle-built populations) and advance the same number of steps; the
comparison is element by element on the pre-collision populations f(x, t).
Tolerance: 1e-12 relative per population after 100 steps (FP64 on both sides;
the kernel evaluates the same equations in a different algebraic order, so
only rounding differs, and the update does not amplify rounding in stable
regimes).  At the full 4096^2 size the oracle computes sampled nodes one by
one on the (2n+1)^2 periodic patch that determines them after n steps.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2501_16000_amd import workloads

pytestmark = pytest.mark.gpu

RTOL = 1e-12


def lib():
    from paper_2501_16000_amd import oreg
    return oreg


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(got, ref):
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)))


def random_populations(eq, theta, ny, nx, seed, amp=0.02, u=0.05):
    rho = 1.0 + 0.1 * workloads.noise((ny, nx), seed)
    ux = u * workloads.noise((ny, nx), seed + 1)
    uy = u * workloads.noise((ny, nx), seed + 2)
    f = oracle.init(eq, theta, rho, ux, uy)
    return f * (1.0 + workloads.noise(f.shape, seed + 3, amp))


CASES = [
    # (nx, ny, eq, theta, tau, collision, bc)
    (8, 8, "guided", 1 / 3, 0.8, "oreg", "periodic"),
    (37, 53, "guided", 1 / 3, 0.8, "oreg", "periodic"),
    (37, 53, "guided", 0.35, 0.51, "oreg", "periodic"),
    (37, 53, "guided", 0.4, 1.0, "oreg", "periodic"),
    (37, 53, "poly2", 1 / 3, 0.51, "oreg", "periodic"),
    (37, 53, "poly2", 1 / 3, 1.0, "oreg", "periodic"),
    (128, 128, "guided", 1 / 3, 0.8, "oreg", "periodic"),
    (1, 200, "guided", 1 / 3, 0.53, "oreg", "periodic"),
    (800, 1, "guided", 0.35, 0.6, "oreg", "periodic"),
    (300, 7, "guided", 1 / 3, 0.7, "oreg", "periodic"),   # ragged: 2 segments, tail of 44
    (16384, 4, "guided", 1 / 3, 0.55, "oreg", "periodic"),
    (1, 1, "guided", 1 / 3, 0.9, "oreg", "periodic"),
    (37, 53, "guided", 1 / 3, 0.8, "bgk", "periodic"),
    (37, 53, "poly2", 1 / 3, 0.6, "bgk", "periodic"),
    (40, 3, "guided", 0.35, 0.7, "oreg", "bounceback"),
    (800, 1, "guided", 0.4, 0.6, "oreg", "bounceback"),
    # the default lb_step path fuses several steps per launch from 48^2 nodes up,
    # with the row block chosen per lattice: both sides of the threshold,
    # narrow-tall and wide-short strips, every collision and boundary
    (48, 48, "guided", 1 / 3, 0.8, "oreg", "periodic"),
    (47, 49, "guided", 1 / 3, 0.8, "oreg", "periodic"),
    (52, 700, "guided", 0.35, 0.6, "oreg", "periodic"),
    (3000, 49, "guided", 1 / 3, 0.51, "oreg", "periodic"),
    (200, 200, "poly2", 1 / 3, 0.7, "oreg", "periodic"),
    (64, 64, "guided", 0.4, 0.9, "bgk", "periodic"),
    (100, 60, "guided", 1 / 3, 0.6, "oreg", "bounceback"),
]


@pytest.mark.parametrize("nx,ny,eq,theta,tau,coll,bc", CASES)
def test_parity_random_populations(nx, ny, eq, theta, tau, coll, bc):
    oreg = lib()
    steps = 100
    say(f"[parity] {nx}x{ny} {eq} theta={theta:.4g} tau={tau} {coll} {bc} steps={steps}")
    f0 = random_populations(eq, theta, ny, nx, seed=nx * 1000 + ny)
    ref = oracle.run(f0, steps, tau, theta, eq, collision=coll, bc_x=bc)
    with oreg.Lattice(nx, ny, tau, theta, equilibrium=eq, collision=coll, boundary_x=bc) as L:
        L.set_populations(f0)
        np.testing.assert_array_equal(L.populations(), f0)  # FP64 round trip is exact
        L.step(steps)
        got = L.populations()
        assert L.time == steps
    err = rel_err(got, ref)
    say(f"  max relative error {err:.3e}")
    assert err <= RTOL


def test_parity_shear_wave_128_from_fields():
    """The 128^2 rotated shear-wave workload (theta = 1/3, tau = 0.8, u0 = 0.01):
    parity at 100 steps, moments at 500 steps."""
    oreg = lib()
    n, tau, theta = 128, 0.8, 1 / 3
    rho, ux, uy = workloads.shear_wave(n, 0.01)
    say("[parity] shear wave 128^2 from fields")
    f0 = oracle.init("guided", theta, rho, ux, uy)
    with oreg.Lattice(n, n, tau, theta) as L:
        L.init(rho, ux, uy)
        np.testing.assert_allclose(L.populations(), f0, rtol=1e-15, atol=0)
        L.step(100)
        f100 = oracle.run(f0, 100, tau, theta)
        err = rel_err(L.populations(), f100)
        say(f"  step 100 max relative error {err:.3e}")
        assert err <= RTOL
        L.step(400)
        f500 = oracle.run(f100, 400, tau, theta)
        m_ref = oracle.moments(f500)
        m = L.moments()
        assert np.max(np.abs(m[0] - m_ref[0])) < 1e-12
        assert np.max(np.abs(m[1:] - m_ref[1:])) < 1e-13
        np.testing.assert_allclose(L.diagnostics()[:5], oracle.diagnostics(f500, theta)[:5],
                                   rtol=1e-12, atol=1e-12)


def patch(f, x0, y0, h):
    """(2h+1)^2 periodic patch of f centred at (x0, y0)."""
    ny, nx = f.shape[-2:]
    ys = (np.arange(y0 - h, y0 + h + 1)) % ny
    xs = (np.arange(x0 - h, x0 + h + 1)) % nx
    return f[..., ys[:, None], xs[None, :]]


@pytest.mark.parametrize("tau", [0.51, 0.6, 1.0])
def test_parity_sampled_4096_fp64(tau):
    """The 4096^2 FP64 throughput workload (rotated shear wave, u0 = 0.05):
    sampled nodes -- corners, edges (periodic wrap) and interior -- after 100
    steps, each recomputed by the oracle on its 201^2 dependency patch."""
    oreg = lib()
    n, theta, steps = 4096, 1 / 3, 100
    say(f"[parity] 4096^2 FP64 tau={tau} sampled nodes, {steps} steps")
    rho, ux, uy = workloads.shear_wave(n, 0.05)
    with oreg.Lattice(n, n, tau, theta) as L:
        L.init(rho, ux, uy)
        L.step(steps)
        m = L.moments()
        d = L.diagnostics()
    rng = np.random.default_rng(7)
    samples = [(0, 0), (n - 1, 0), (0, n - 1), (n - 1, n - 1), (n // 2, 0), (0, n // 2),
               (255, 17), (256, 4000)] + [tuple(rng.integers(0, n, 2)) for _ in range(4)]
    fields = np.stack([rho, ux, uy])
    worst = 0.0
    for (x0, y0) in samples:
        pf = patch(fields, x0, y0, steps)
        fp = oracle.run(oracle.init("guided", theta, pf[0], pf[1], pf[2]), steps, tau, theta)
        mp = oracle.moments(fp)[:, steps, steps]
        worst = max(worst, float(np.max(np.abs(m[:, y0, x0] - mp))))
    say(f"  max |moment difference| over {len(samples)} nodes: {worst:.3e}")
    assert worst < 1e-13
    # mass is conserved to roundoff at any size (Sec. III.C, Eq. 13a)
    assert abs(d[0] - n * n) < 1e-9 * n * n
    assert d[5] == 0


@pytest.mark.parametrize("storage,bound", [("f32s", 3e-7), ("f16s", 5e-5), ("bf16s", 1.5e-3)])
def test_sampled_4096_reduced_precision(storage, bound):
    """The 4096^2 workload in shifted reduced-precision storage, in the launch
    configuration the benchmark times (fused six-step launches): sampled
    nodes after 100 steps against the FP64 oracle on their dependency
    patches, within the storage's rounding."""
    oreg = lib()
    n, tau, theta, steps = 4096, 0.6, 1 / 3, 100
    say(f"[parity] 4096^2 {storage} sampled nodes, {steps} steps")
    rho, ux, uy = workloads.shear_wave(n, 0.05)
    with oreg.Lattice(n, n, tau, theta, storage=storage) as L:
        L.init(rho, ux, uy)
        L.step(steps)
        m = L.moments()
    rng = np.random.default_rng(9)
    samples = [(0, 0), (n - 1, n - 1), (51, 63), (52, 64), (2000, 4095)] + \
        [tuple(rng.integers(0, n, 2)) for _ in range(3)]
    fields = np.stack([rho, ux, uy])
    worst = 0.0
    for (x0, y0) in samples:
        pf = patch(fields, x0, y0, steps)
        fp = oracle.run(oracle.init("guided", theta, pf[0], pf[1], pf[2]), steps, tau, theta)
        mp = oracle.moments(fp)[:, steps, steps]
        worst = max(worst, float(np.max(np.abs(m[:, y0, x0] - mp))))
    say(f"  max |moment difference| over {len(samples)} nodes: {worst:.3e}")
    assert worst < bound


def test_fixed_point_and_mass_at_full_size():
    oreg = lib()
    n = 4096
    say("[gpu] uniform state fixed point, 4096^2, 20 steps")
    with oreg.Lattice(n, n, 0.6, 0.35) as L:
        rho = np.full((n, n), 1.2)
        ux = np.full((n, n), 0.04)
        uy = np.full((n, n), -0.02)
        L.init(rho, ux, uy)
        L.step(20)
        m = L.moments()
    assert np.max(np.abs(m[0] - 1.2)) < 1e-14
    assert np.max(np.abs(m[1] - 0.04)) < 1e-14
    assert np.max(np.abs(m[2] + 0.02)) < 1e-14


def test_determinism_and_checkpoint_resume():
    """Two runs are bitwise identical; 100 steps == 50 + export/import + 50."""
    oreg = lib()
    nx, ny, tau, theta = 97, 61, 0.7, 1 / 3
    f0 = random_populations("guided", theta, ny, nx, 11)
    say("[gpu] determinism and checkpoint/resume 97x61")
    with oreg.Lattice(nx, ny, tau, theta) as A, oreg.Lattice(nx, ny, tau, theta) as B:
        A.set_populations(f0)
        A.step(100)
        fa = A.populations()
        B.set_populations(f0)
        B.step(100)
        np.testing.assert_array_equal(B.populations(), fa)
        B.set_populations(f0)
        B.step(50)
        mid = B.populations()
        B.set_populations(mid)
        B.step(50)
        np.testing.assert_array_equal(B.populations(), fa)
        da, db = A.diagnostics(), B.diagnostics()
        np.testing.assert_array_equal(da, db)


def test_symmetry_on_gpu():
    """A 90-degree rotation of the initial state commutes with the sweep."""
    oreg = lib()
    n, tau, theta = 64, 0.62, 1 / 3
    f0 = random_populations("guided", theta, n, n, 21)
    c = oracle.velocities()

    def rot(f):
        g = np.empty_like(f)
        for i in range(9):
            j = [k for k in range(9) if c[k, 0] == -c[i, 1] and c[k, 1] == c[i, 0]][0]
            # g_j(x' = n-1-y, y' = x) = f_i(x, y)
            g[j] = f[i][::-1, :].T
        return g

    say("[gpu] rotation symmetry 64x64")
    with oreg.Lattice(n, n, tau, theta) as L:
        L.set_populations(f0)
        L.step(40)
        a = L.populations()
        L.set_populations(rot(f0))
        L.step(40)
        b = L.populations()
    np.testing.assert_allclose(b, rot(a), rtol=1e-13, atol=1e-16)


def test_density_profile_and_diagnostics_shocktube():
    oreg = lib()
    nx, ny, tau, theta, steps = 2048, 4, 0.55, 1 / 3, 300
    rho, ux, uy = workloads.shocktube(nx, ny)
    say("[gpu] shocktube 2048x4 profile vs oracle")
    f = oracle.run(oracle.init("guided", theta, rho, ux, uy), steps, tau, theta)
    with oreg.Lattice(nx, ny, tau, theta) as L:
        L.init(rho, ux, uy)
        L.step(steps)
        prof = L.density_profile()
        d = L.diagnostics()
    ref = oracle.moments(f)[0].mean(axis=0)
    assert np.max(np.abs(prof - ref)) < 1e-13
    dref = oracle.diagnostics(f, theta)
    np.testing.assert_allclose(d[:5], dref[:5], rtol=1e-12, atol=1e-11)


def test_error_paths_on_device():
    oreg = lib()
    say("[gpu] error paths")
    L = oreg.Lattice(16, 16, 0.8)
    with pytest.raises(oreg.LBError) as e:
        L.step(1)
    assert e.value.status == oreg.LB_ESTATE
    with pytest.raises(oreg.LBError) as e:
        L.moments()
    assert e.value.status == oreg.LB_ESTATE
    bad = np.ones((16, 16))
    bad[3, 4] = np.nan
    with pytest.raises(oreg.LBError) as e:
        L.init(bad, np.zeros((16, 16)), np.zeros((16, 16)))
    assert e.value.status == oreg.LB_EINVAL
    f = np.full((9, 16, 16), 1.0 / 9)
    f[2, 5, 5] = np.inf
    with pytest.raises(oreg.LBError) as e:
        L.set_populations(f)
    assert e.value.status == oreg.LB_EINVAL
    L.init(np.ones((16, 16)), np.zeros((16, 16)), np.zeros((16, 16)))
    with pytest.raises(oreg.LBError) as e:
        L.step(-1)
    assert e.value.status == oreg.LB_EINVAL
    L.step(0)
    assert L.time == 0
    L.close()


def test_nonfinite_check_reports():
    """check_nonfinite turns a blow-up into LB_ENONFINITE instead of silent NaN."""
    oreg = lib()
    say("[gpu] non-finite detection")
    n = 16
    f = random_populations("guided", 0.35, n, n, 5)
    # one node carries an enormous momentum: u far beyond the scheme's range
    f[1, 7, 7] = 50.0
    with oreg.Lattice(n, n, 0.5000001, 0.35, check_nonfinite=True) as L:
        L.set_populations(f)
        status = None
        for _ in range(200):
            try:
                L.step(10)
            except oreg.LBError as e:
                status = e.status
                break
        assert status == oreg.LB_ENONFINITE
        assert L.diagnostics()[5] > 0


def test_device_init_and_moments_with_torch():
    """torch supplies device memory and the stream; the library does the work."""
    import torch
    oreg = lib()
    n, tau, theta = 64, 0.8, 1 / 3
    say("[gpu] torch device pointers and stream")
    rho, ux, uy = workloads.shear_wave(n, 0.02)
    dev = torch.device("cuda:0")
    s = torch.cuda.current_stream()
    fields = [torch.from_numpy(a.copy()).to(dev) for a in (rho, ux, uy)]
    out = torch.empty((3, n, n), dtype=torch.float64, device=dev)
    with oreg.Lattice(n, n, tau, theta, stream=s) as L:
        L.init(*fields)
        L.step(30)
        L.moments(out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        host = L.moments()
    np.testing.assert_array_equal(got, host)
    ref = oracle.moments(oracle.run(oracle.init("guided", theta, rho, ux, uy), 30, tau, theta))
    assert np.max(np.abs(got - ref)) < 1e-13


FUSED_CASES = [
    # (nx, ny, eq, theta, tau, collision, bc, storage)
    (300, 77, "guided", 1 / 3, 0.8, "oreg", "periodic", "f64"),
    (64, 64, "guided", 0.35, 0.51, "oreg", "periodic", "f64"),
    (37, 5, "poly2", 1 / 3, 0.6, "oreg", "periodic", "f64"),
    (1, 200, "guided", 1 / 3, 0.53, "oreg", "periodic", "f64"),
    (800, 1, "guided", 0.4, 0.6, "oreg", "bounceback", "f64"),
    (53, 71, "guided", 1 / 3, 0.9, "bgk", "periodic", "f64"),
    (130, 3, "poly2", 1 / 3, 0.7, "bgk", "bounceback", "f64"),
    (52, 128, "guided", 1 / 3, 0.75, "oreg", "periodic", "f64"),    # exactly one strip, two row blocks
    (104, 65, "guided", 0.35, 0.6, "oreg", "bounceback", "f64"),   # two strips, one row past a block
    (513, 130, "guided", 1 / 3, 0.6, "oreg", "periodic", "f32s"),
    (200, 40, "poly2", 1 / 3, 0.7, "oreg", "periodic", "f16s"),
    (1000, 130, "guided", 1 / 3, 0.6, "oreg", "periodic", "f16s"),
    (301, 67, "guided", 0.4, 0.55, "bgk", "bounceback", "f16s"),
    (97, 33, "guided", 0.35, 0.8, "oreg", "bounceback", "bf16s"),
    (640, 96, "poly2", 1 / 3, 0.9, "oreg", "periodic", "bf16s"),
    # several 66-row blocks per strip: ragged last block, exact multiple
    (52, 300, "guided", 1 / 3, 0.7, "oreg", "periodic", "f64"),
    (52, 198, "guided", 0.35, 0.6, "oreg", "periodic", "f32s"),
    (60, 500, "guided", 1 / 3, 0.55, "oreg", "periodic", "bf16s"),
    # F32S: strip edges across the periodic wrap, walls, BGK, degenerate shapes
    (117, 40, "guided", 1 / 3, 0.6, "oreg", "periodic", "f32s"),
    (116, 70, "guided", 0.35, 0.7, "oreg", "bounceback", "f32s"),
    (233, 35, "poly2", 1 / 3, 0.8, "bgk", "periodic", "f32s"),
    (1, 200, "guided", 1 / 3, 0.53, "oreg", "periodic", "f32s"),
    (801, 1, "guided", 0.4, 0.6, "oreg", "bounceback", "f32s"),
    (245, 40, "guided", 1 / 3, 0.7, "oreg", "periodic", "f32s"),    # one 244-column strip and one column
    (700, 130, "guided", 0.35, 0.6, "bgk", "bounceback", "f32s"),
]


@pytest.mark.parametrize("nx,ny,eq,theta,tau,coll,bc,storage", FUSED_CASES)
def test_fused_steps_equal_single_steps(nx, ny, eq, theta, tau, coll, bc, storage):
    """Fused launches (fuse_steps = 2 forces them at any size) give bit for
    bit the result of one sweep launch per step (fuse_steps = 1)."""
    oreg = lib()
    say(f"[fused] {nx}x{ny} {eq} {coll} {bc} {storage}")
    f0 = random_populations(eq, theta, ny, nx, seed=7 * nx + ny)
    out = []
    for fuse in (2, 1):
        with oreg.Lattice(nx, ny, tau, theta, equilibrium=eq, collision=coll, boundary_x=bc,
                          storage=storage, rho0=1.0, fuse_steps=fuse) as L:
            L.set_populations(f0)
            L.step(37)
            out.append(L.populations())
    np.testing.assert_array_equal(out[0], out[1])
    if storage == "f64":
        ref = oracle.run(f0, 37, tau, theta, eq, collision=coll, bc_x=bc)
        assert rel_err(out[0], ref) <= RTOL


@pytest.mark.parametrize("nbytes", [16, 4096 + 48, (1 << 26) + 16 * 7])
def test_copy_device_copies_every_byte(nbytes):
    """lb_copy_device (the bandwidth reference of the benchmark) copies the
    bytes it is given and nothing past them."""
    import torch
    oreg = lib()
    say(f"[copy] {nbytes} bytes")
    g = torch.Generator(device="cpu").manual_seed(nbytes)
    host = torch.randint(0, 256, (nbytes + 64,), dtype=torch.uint8, generator=g)
    src = host.to("cuda")
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    oreg.copy_device(src.data_ptr(), dst.data_ptr(), nbytes, stream)
    torch.cuda.synchronize()
    out = dst.cpu()
    assert torch.equal(out[:nbytes], host[:nbytes])
    assert int(out[nbytes:].count_nonzero()) == 0


SHORT_FUSED_CASES = [
    # (nx, ny, eq, tau, storage, steps): periodic OReg lattices advance a
    # remainder of 2 .. K-1 steps in one shorter fused launch (K = 7 in FP64,
    # 6 in the shifted formats)
    (300, 77, "guided", 0.8, "f64", 2),
    (300, 77, "guided", 0.8, "f64", 9),     # 7 + 2
    (64, 64, "poly2", 0.51, "f64", 20),     # 7 + 7 + 6
    (1, 200, "guided", 0.53, "f64", 5),
    (801, 3, "guided", 0.6, "f64", 11),     # 7 + 4
    (513, 130, "guided", 0.6, "f32s", 10),  # 6 + 4
    (245, 40, "poly2", 0.7, "f32s", 3),
    (1000, 130, "guided", 0.6, "f16s", 8),  # 6 + 2
    (97, 33, "guided", 0.8, "bf16s", 17),   # 6 + 6 + 5
]


@pytest.mark.parametrize("nx,ny,eq,tau,storage,steps", SHORT_FUSED_CASES)
def test_short_fused_launches_equal_single_steps(nx, ny, eq, tau, storage, steps):
    """Fused launches of fewer than K steps give bit for bit the result of
    one sweep launch per step (and, in FP64, the oracle's)."""
    oreg = lib()
    theta = 1 / 3
    say(f"[fused short] {nx}x{ny} {eq} {storage} steps={steps}")
    f0 = random_populations(eq, theta, ny, nx, seed=11 * nx + ny + steps)
    out = []
    for fuse in (2, 1):
        with oreg.Lattice(nx, ny, tau, theta, equilibrium=eq, storage=storage, rho0=1.0,
                          fuse_steps=fuse) as L:
            L.set_populations(f0)
            L.step(steps)
            assert L.time == steps
            out.append(L.populations())
    np.testing.assert_array_equal(out[0], out[1])
    if storage == "f64":
        ref = oracle.run(f0, steps, tau, theta, eq)
        assert rel_err(out[0], ref) <= RTOL

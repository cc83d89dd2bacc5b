"""Continuous-batching server (lb_server_*) on the GPU.

* Every result of a mixed stream equals, bit for bit, the same request run
  alone on a server and the same lattice run through lb_step: the batched
  launch does the per-node arithmetic of a lattice on its own.
* Admission by footprint and by slots: with a budget that holds two lattices,
  the rest wait (submit answers no room) and run as lattices retire.
* Results agree with the FP64 oracle to the FP32-storage error, and the
  decay rate of a served shear wave is within 1e-3 of the oracle's, also on
  the corner of the stream's distribution where FP32 storage is least
  accurate (tau near 1/2, waves that decay by 5-10 % over the run).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2501_16000_amd import workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mods():
    from paper_2501_16000_amd import oreg, serve
    return oreg, serve


def small_requests(count=14, seed=3):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        n = int(rng.choice([8, 17, 32, 45, 64, 100, 128]))
        reqs.append(workloads.ServingRequest(i, 0.0, n, float(rng.uniform(0.52, 1.2)),
                                             float(rng.uniform(0.005, 0.05)),
                                             int(rng.integers(20, 300))))
    return reqs


def serve_all(server, reqs, steps_per_call=3):
    """Submit in order (waiting when there is no room), step, collect (results
    of lattices submitted earlier are collected too)."""
    out, queue = {}, list(reqs)
    want = {r.rid for r in reqs}
    while not want <= set(out):
        while queue:
            r = queue[0]
            rho, ux, uy = workloads.shear_wave(r.n, r.u0)
            if not server.submit(r.rid, rho, ux, uy, r.tau, r.steps):
                break
            queue.pop(0)
        server.step(steps_per_call)
        while True:
            res = server.poll()
            if res is None:
                break
            out[res.tag] = server.fetch(res)
    return out


def test_mix_equals_alone_and_single_lattice_path():
    oreg, serve = mods()
    reqs = small_requests()
    say(f"[serve] {len(reqs)} requests in one mix")
    with serve.Server(memory_budget=1 << 30, max_active=64) as srv:
        mixed = serve_all(srv, reqs)
    assert sorted(mixed) == [r.rid for r in reqs]
    for r in reqs[:6]:
        say(f"  request {r.rid}: {r.n}^2 tau={r.tau:.3f} steps={r.steps} alone")
        with serve.Server(memory_budget=1 << 28, max_active=4) as srv:
            alone = serve_all(srv, [r])[r.rid]
        np.testing.assert_array_equal(mixed[r.rid], alone)
        with oreg.Lattice(r.n, r.n, r.tau, storage="f32s") as L:
            L.init(*workloads.shear_wave(r.n, r.u0))
            L.step(r.steps)
            np.testing.assert_array_equal(mixed[r.rid], L.moments())


def test_admission_by_footprint_and_slots():
    oreg, serve = mods()
    reqs = [workloads.ServingRequest(i, 0.0, 64, 0.8, 0.02, 40 + 10 * i) for i in range(6)]
    footprint = 2 * 9 * 4 * 64 * 64 + 3 * 8 * 64 * 64
    say("[serve] admission: arena for two lattices, then one slot")
    with serve.Server(memory_budget=2 * footprint + 512, max_active=8) as srv:
        rho, ux, uy = workloads.shear_wave(64, 0.02)
        assert srv.submit(0, rho, ux, uy, 0.8, 40)
        assert srv.submit(1, rho, ux, uy, 0.8, 50)
        assert not srv.submit(2, rho, ux, uy, 0.8, 60)   # arena full
        assert srv.stats().active == 2
        got = serve_all(srv, reqs[2:])
        while len(got) < 6:
            srv.step(10)
            srv.sync()
            while (res := srv.poll()) is not None:
                got[res.tag] = srv.fetch(res)
    assert sorted(got) == list(range(6))
    with serve.Server(memory_budget=1 << 28, max_active=1) as srv:
        rho, ux, uy = workloads.shear_wave(32, 0.02)
        assert srv.submit(0, rho, ux, uy, 0.8, 5)
        assert not srv.submit(1, rho, ux, uy, 0.8, 5)     # no slot
        srv.step(5)
        srv.sync()
        assert srv.submit(1, rho, ux, uy, 0.8, 5)


def test_results_match_oracle_and_decay_rate():
    oreg, serve = mods()
    n, tau, u0 = 64, 0.7, 0.03
    rho, ux, uy = workloads.shear_wave(n, u0)
    say("[serve] served shear wave vs FP64 oracle")
    checkpoints = [0, 100, 200, 300, 400]
    with serve.Server(memory_budget=1 << 28) as srv:
        got = {}
        for k, steps in enumerate(checkpoints[1:]):
            assert srv.submit(k, rho, ux, uy, tau, steps)
        srv.step(400)
        srv.sync()
        while (res := srv.poll()) is not None:
            got[res.steps] = srv.fetch(res)
    f = oracle.init("guided", 1 / 3, rho, ux, uy)
    e_perp, phase = workloads.shear_wave_projection(n)

    def amp(m):
        return abs(((e_perp[0] * m[1] + e_perp[1] * m[2]) * phase).sum())

    a_ref, a_gpu = [amp(oracle.moments(f))], [amp(np.stack([rho, ux, uy]))]
    for t0, t1 in zip(checkpoints, checkpoints[1:]):
        f = oracle.run(f, t1 - t0, tau, 1 / 3)
        m_ref = oracle.moments(f)
        assert np.max(np.abs(got[t1] - m_ref)) < 1e-6
        a_ref.append(amp(m_ref))
        a_gpu.append(amp(got[t1]))
    k_ref = -np.polyfit(checkpoints, np.log(a_ref), 1)[0]
    k_gpu = -np.polyfit(checkpoints, np.log(a_gpu), 1)[0]
    err = abs(k_gpu / k_ref - 1)
    say(f"  decay-rate relative error {err:.2e}")
    assert err < 1e-3


def test_pinned_result_space_exhausted_falls_back():
    oreg, serve = mods()
    n = 48
    rho, ux, uy = workloads.shear_wave(n, 0.02)
    one = 3 * 8 * n * n
    say("[serve] results larger than the pinned space in flight")
    with serve.Server(memory_budget=1 << 28, pinned_bytes=one + 256) as srv:
        for k in range(3):
            assert srv.submit(k, rho, ux, uy, 0.8, 10)
        srv.step(10)
        srv.sync()
        res = []
        while (r := srv.poll()) is not None:
            res.append(srv.fetch(r))
    assert len(res) == 3
    for m in res[1:]:
        np.testing.assert_array_equal(m, res[0])


def test_invalid_requests():
    oreg, serve = mods()
    with serve.Server(memory_budget=1 << 26) as srv:
        rho, ux, uy = workloads.shear_wave(16, 0.01)
        for tau, steps in ((0.5, 10), (0.8, 0)):
            with pytest.raises(oreg.LBError) as e:
                srv.submit(0, rho, ux, uy, tau, steps)
            assert e.value.status == oreg.LB_EINVAL
        bad = rho.copy()
        bad[2, 3] = np.nan
        with pytest.raises(oreg.LBError):
            srv.submit(0, bad, ux, uy, 0.8, 5)
        big = workloads.shear_wave(2048, 0.01)
        with pytest.raises(oreg.LBError) as e:
            srv.submit(1, *big, 0.8, 5)   # larger than the whole arena
        assert e.value.status == oreg.LB_EINVAL


@pytest.mark.parametrize("storage", ["f64", "f16s"])
def test_other_storages_equal_single_lattice_path(storage):
    """F64 and F16S serving (batched fused launches) equal lb_step on one
    lattice bit for bit, also when a lattice's steps are not a multiple of the
    fused step count."""
    oreg, serve = mods()
    reqs = [workloads.ServingRequest(0, 0.0, 40, 0.7, 0.03, 31),
            workloads.ServingRequest(1, 0.0, 70, 0.9, 0.02, 12),
            workloads.ServingRequest(2, 0.0, 17, 0.55, 0.04, 5)]
    say(f"[serve] {storage} mix vs lb_step")
    with serve.Server(memory_budget=1 << 28, storage=storage) as srv:
        got = serve_all(srv, reqs, steps_per_call=2)
    for r in reqs:
        with oreg.Lattice(r.n, r.n, r.tau, storage=storage) as L:
            L.init(*workloads.shear_wave(r.n, r.u0))
            L.step(r.steps)
            np.testing.assert_array_equal(got[r.rid], L.moments())


@pytest.mark.parametrize("storage", ["f32s", "f64", "bf16s"])
def test_degenerate_and_non_square_lattices(storage):
    """Rows and columns of one node, odd and non-square sizes, in one mix:
    each result equals lb_step on the same lattice bit for bit."""
    oreg, serve = mods()
    shapes = [(1, 7), (5, 1), (1, 1), (64, 3), (3, 64), (129, 65), (33, 200)]
    rng = np.random.default_rng(17)
    cases = []
    for k, (nx, ny) in enumerate(shapes):
        rho = 1.0 + 0.05 * rng.uniform(-1, 1, (ny, nx))
        ux = 0.03 * rng.uniform(-1, 1, (ny, nx))
        uy = 0.03 * rng.uniform(-1, 1, (ny, nx))
        cases.append((k, rho, ux, uy, float(rng.uniform(0.55, 1.1)), int(rng.integers(1, 40))))
    say(f"[serve] {storage}: degenerate and non-square lattices")
    got = {}
    with serve.Server(memory_budget=1 << 28, storage=storage) as srv:
        for k, rho, ux, uy, tau, steps in cases:
            assert srv.submit(k, rho, ux, uy, tau, steps)
        while len(got) < len(cases):
            srv.step(4)
            srv.sync()
            while (res := srv.poll()) is not None:
                got[res.tag] = srv.fetch(res)
    for k, rho, ux, uy, tau, steps in cases:
        ny, nx = rho.shape
        with oreg.Lattice(nx, ny, tau, storage=storage) as L:
            L.init(rho, ux, uy)
            L.step(steps)
            np.testing.assert_array_equal(got[k], L.moments())


# The corner of the serving stream's distribution where shifted FP32 storage
# is least accurate: tau near 1/2 and waves that decay by only 5-10 % over the
# run (the lower edge of the window 0.05 <= ln(a0/aT) <= ln 1e4 in which the
# stream's decay rates are compared), N up to 969, up to 5000 steps.  The first
# two are the stream's worst requests; the others sit at the same edge with
# tau = 0.52-0.53 and u0 from 0.005 to 0.05.
CORNER = [(342, 0.5312, 0.0248, 3679), (969, 0.6996, 0.0274, 4256), (300, 0.52, 0.005, 5000),
          (256, 0.52, 0.05, 5000), (420, 0.53, 0.01, 5000), (180, 0.52, 0.005, 2000)]


def test_worst_case_corner_decay_rate():
    """Served F32S results against the FP64 lb_step path on the corner
    requests: the decay rate within 1e-3 (the serving accuracy target)."""
    oreg, serve = mods()
    reqs = [workloads.ServingRequest(i, 0.0, n, tau, u0, steps)
            for i, (n, tau, u0, steps) in enumerate(CORNER)]
    say(f"[serve] {len(reqs)} corner requests, F32S server vs FP64 lb_step")
    with serve.Server(memory_budget=1 << 32, storage="f32s") as srv:
        got = serve_all(srv, reqs, steps_per_call=50)
    for r in reqs:
        rho, ux, uy = workloads.shear_wave(r.n, r.u0)
        with oreg.Lattice(r.n, r.n, r.tau, 1 / 3) as L:
            L.init(rho, ux, uy)
            L.step(r.steps)
            ref = L.moments()
        e_perp, phase = workloads.shear_wave_projection(r.n)

        def amp(m):
            return abs(((e_perp[0] * m[1] + e_perp[1] * m[2]) * phase).sum())

        a0 = amp(np.stack([rho, ux, uy]))
        l64 = np.log(a0 / amp(ref))
        err = abs(np.log(a0 / amp(got[r.rid])) / l64 - 1)
        say(f"  N={r.n} tau={r.tau} u0={r.u0} steps={r.steps}: ln(a0/aT) {l64:.4f}, "
            f"decay-rate error {err:.2e}")
        assert 0.05 <= l64 <= np.log(1e4)
        assert err < 1e-3

"""The largest boxes that fit one MI355X, to exercise 64-bit indexing: every
population plane offset and row offset beyond 2^31 elements.

* D2Q9 32768^2 FP64: 1.07e9 nodes, 9.7e9 stored populations per buffer
  (155 GB for the two buffers), one fused launch (6 steps) and one single
  step;
* D3Q27 512^3 FP64: 1.34e8 nodes, 3.6e9 populations per buffer (58 GB).

Fields are built on the device with the same generator formula the oracle
uses for its patches (workloads.shear_wave_at); sampled nodes (corners, the
last row and column, offsets past 2^31) are recomputed by the oracle on the
periodic patch that determines them.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import d3q27 as o3
from paper_2501_16000_amd import workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_d2q9_32768_fp64_sampled():
    import torch
    from paper_2501_16000_amd import oreg
    n, tau, theta, u0 = 32768, 0.6, 1 / 3, 0.05
    if torch.cuda.get_device_properties(0).total_memory < 200 * 2 ** 30:
        pytest.skip("needs a GPU with 200 GiB")
    say(f"[large] D2Q9 {n}^2 FP64: device fields, 7 + 1 steps")
    with oreg.Lattice(n, n, tau, theta) as L:
        ys = torch.arange(n, dtype=torch.float64, device="cuda")
        y, x = torch.meshgrid(ys, ys, indexing="ij")
        fields = workloads.shear_wave_at(x, y, n, u0, xp=torch)
        del x, y
        L.init(*[f.contiguous() for f in fields])
        del fields
        torch.cuda.synchronize()
        L.step(8)          # one fused launch of 7 steps, then one single step
        out = torch.empty((3, n, n), dtype=torch.float64, device="cuda")
        L.moments(out=out)
        L.sync()
        samples = [(0, 0), (n - 1, n - 1), (n - 1, 0), (0, n - 1), (12345, 23456),
                   (n // 2, n - 2), (7, 30001)]
        got = {s: out[:, s[1], s[0]].cpu().numpy() for s in samples}
        d = L.diagnostics()
    del out
    torch.cuda.empty_cache()
    steps, h = 8, 8
    worst = 0.0
    for (x0, y0) in samples:
        xs = (np.arange(x0 - h, x0 + h + 1) % n).astype(np.float64)
        ysv = (np.arange(y0 - h, y0 + h + 1) % n).astype(np.float64)
        py, px = np.meshgrid(ysv, xs, indexing="ij")
        pf = workloads.shear_wave_at(px, py, n, u0)
        fp = oracle.run(oracle.init("guided", theta, *pf), steps, tau, theta)
        ref = oracle.moments(fp)[:, h, h]
        worst = max(worst, float(np.max(np.abs(got[(x0, y0)] - ref))))
    say(f"  max |moment difference| over {len(samples)} nodes: {worst:.3e}")
    assert worst < 1e-14
    assert abs(d[0] - float(n) * n) < 1e-6 * n * n
    assert d[5] == 0


def test_d3q27_512_fp64_sampled():
    import torch
    from paper_2501_16000_amd import oreg3
    n, tau, theta, u0, steps = 512, 0.6, 1 / 3, 0.05, 2
    say(f"[large] D3Q27 {n}^3 FP64: device fields, {steps} steps")
    with oreg3.Lattice3(n, n, n, tau, theta) as L:
        r = torch.arange(n, dtype=torch.float64, device="cuda")
        z, y, x = torch.meshgrid(r, r, r, indexing="ij")
        fields = workloads.shear_wave3_at(x, y, z, n, u0, xp=torch)
        del x, y, z
        L.init(*[f.contiguous() for f in fields])
        del fields
        torch.cuda.synchronize()
        L.step(steps)
        out = torch.empty((4, n, n, n), dtype=torch.float64, device="cuda")
        L.moments(out=out)
        L.sync()
        samples = [(0, 0, 0), (n - 1, n - 1, n - 1), (n - 1, 0, n - 1), (63, 64, 500),
                   (300, 511, 7), (n // 2, n // 3, n - 2)]
        got = {s: out[:, s[2], s[1], s[0]].cpu().numpy() for s in samples}
        d = L.diagnostics()
    del out
    torch.cuda.empty_cache()
    h = steps
    worst = 0.0
    for (x0, y0, z0) in samples:
        ax = [(np.arange(c - h, c + h + 1) % n).astype(np.float64) for c in (z0, y0, x0)]
        pz, py, px = np.meshgrid(*ax, indexing="ij")
        pf = workloads.shear_wave3_at(px, py, pz, n, u0)
        fp = o3.run(o3.init("guided", theta, *pf), steps, tau, theta)
        ref = o3.moments(fp)[:, h, h, h]
        worst = max(worst, float(np.max(np.abs(got[(x0, y0, z0)] - ref))))
    say(f"  max |moment difference| over {len(samples)} nodes: {worst:.3e}")
    assert worst < 1e-14
    assert abs(d[0] - float(n) ** 3) < 1e-6 * n ** 3
    assert d[6] == 0

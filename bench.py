#!/usr/bin/env python3
"""Throughput of the fused OReg D2Q9 sweep on one MI355X.

One step = one sweep (pull streaming + moments + equilibrium + OReg
reconstruction + relaxation + store) over the whole lattice.  Workload: the
4096 x 4096 periodic lattice with the rotated (atan(1/2)) shear wave,
u0 = 0.05, guided equilibrium, theta = 1/3, tau = 0.6, FP64 storage, one
lattice per launch.  Populations are resident in HBM before timing starts.

Prints one JSON line (rank 0):
  value      MLUPS = nx * ny * steps / seconds / 1e6 (FP64 storage)
  roofline   the sweep kernel's algorithmic bytes (2 * 9 * 8 per node) per
             launch over its average launch time (HIP events on the lattice's
             stream), against 8 TB/s; traffic from rocprofv3 counters when
             profiles/ holds them for this kernel
  variants   the same workload with shifted FP32 / FP16 / BF16 storage
  d3q27      the D3Q27 sweep on a 256^3 periodic box (shear wave normal to
             (1, 1, 1)), every storage, against the HBM roofline
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the workload
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (FP64 vs FP32/BF16 storage) at % HBM roofline; p50/p99 latency batched"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector
FP32_PEAK_TFLOPS = 157.3    # MI355X FP32 vector
VALU_PEAK = 256 * 4 * 16 * 2.4e9  # lane-instructions/s: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
BYTES_PER_NODE = {"f64": 144, "f32s": 72, "f16s": 36, "bf16s": 36}
STORAGE_BYTES = {"f64": 8, "f32s": 4, "f16s": 2, "bf16s": 2}
# Time steps per fused launch (dispatch.hpp FusedLevels) and the algorithmic
# flops of one guided-equilibrium OReg node update as implemented in
# d2q9.hpp::collide for FP64 (FMA = 2, the one division = 1): moments, 1/rho,
# u and u^2 22; axis factors and rho X 17; stress and kappa S 9; bracket
# factors 32; the nine updates 45.
FUSED_K = {"f64": 7, "f32s": 6, "f16s": 6, "bf16s": 6}
FLOPS_PER_UPDATE = 125
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_traffic_4096.json")


def parse():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1000)
    p.add_argument("--warmup", type=int, default=50)
    p.add_argument("--n", type=int, default=4096, help="lattice side")
    p.add_argument("--tau", type=float, default=0.6)
    p.add_argument("--storage", default="f64", choices=sorted(BYTES_PER_NODE))
    p.add_argument("--variants", default="f32s,f16s,bf16s",
                   help="other storages to time on the same workload ('' for none)")
    p.add_argument("--variant-steps", type=int, default=600)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-steps", type=int, default=60,
                   help="oracle steps on the full lattice for the CPU baseline")
    p.add_argument("--serving-requests", type=int, default=2000,
                   help="requests of the serving stream (0 skips the serving measurement)")
    p.add_argument("--serving-plain-requests", type=int, default=0,
                   help="requests of the stream that the plain FP64 path also runs and the "
                        "decay-rate errors cover (0: all)")
    p.add_argument("--d3q27-n", type=int, default=256,
                   help="side of the D3Q27 box timed per storage (0 skips it)")
    p.add_argument("--d3q27-steps", type=int, default=100)
    p.add_argument("--pmc-workload", action="store_true",
                   help="only run a few sweeps per storage plus a 1 GiB device copy "
                        "(the workload profiled with rocprofv3 --pmc)")
    p.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                   help="turn two rocprofv3 --pmc counter CSVs (FETCH_SIZE, WRITE_SIZE) of "
                        "--pmc-workload into " + os.path.relpath(TRAFFIC_FILE, ROOT))
    p.add_argument("--summarize-counters", nargs="+", metavar="CSV",
                   help="print per-launch SQ / TCP counter figures of the 4096^2 sweep kernels "
                        "from rocprofv3 --pmc CSVs of --pmc-workload (markdown)")
    return p.parse_args()


def time_lattice(oreg, torch, n, tau, storage, steps, warmup, fields, fuse_steps=0, split=None):
    """Return (elapsed_ms, diagnostics) of `steps` time steps timed with HIP
    events on the stream the sweeps are launched on.  With `split`, the timed
    region is issued as `split` steps and then the rest, with an event between
    them, and the elapsed ms of the first part is returned third."""
    stream = torch.cuda.Stream()  # default priority
    rho0 = 1.0
    with torch.cuda.stream(stream), \
            oreg.Lattice(n, n, tau, 1.0 / 3.0, storage=storage, rho0=rho0, stream=stream,
                         fuse_steps=fuse_steps) as lat:
        lat.init(*fields)
        lat.step(warmup)
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        if split is None:
            lat.step(steps)
        else:
            mid = torch.cuda.Event(enable_timing=True)
            lat.step(split)
            mid.record(stream)
            lat.step(steps - split)
        end.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(end)
        diag = lat.diagnostics()
        if split is not None:
            return ms, diag, start.elapsed_time(mid)
    return ms, diag


SOURCES_2D = ("kernels.hip", "d2q9.hpp", "dispatch.hpp", "fused_impl.hpp", "fused_f64.hip",
              "fused_f32s.hip", "fused_f16s.hip", "fused_bf16s.hip")
SOURCES_3D = ("kernels3.hip", "d3q27.hpp", "d2q9.hpp")


def load_traffic(storage, n, nbytes_alg, fused=False, d3=False):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    covers this kernel build; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    key = ("d3q27_" if d3 else "") + ("fused_" if fused else "") + storage
    entry = t.get("kernels", {}).get(key)
    sha = kernel_source_sha(SOURCES_3D if d3 else SOURCES_2D)
    if not entry or entry.get("n") != n or entry.get("kernel_source_sha") != sha:
        return None
    return entry.get("hbm_bytes_per_launch")


def kernel_source_sha(files=SOURCES_2D):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2501_16000_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def time_box(oreg3, torch, n, tau, storage, steps, warmup, fields):
    """Elapsed ms of `steps` D3Q27 sweeps (HIP events on the sweeps' stream)."""
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream), \
            oreg3.Lattice3(n, n, n, tau, 1.0 / 3.0, storage=storage, stream=stream) as box:
        box.init(*fields)
        box.step(warmup)
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        box.step(steps)
        end.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(end)
        diag = box.diagnostics()
    return ms, diag


def hbm_side(traffic, alg_bytes, launch_s):
    """HBM view of a fused launch: the algorithmic bytes (the state read and
    written once per K-step launch: 2 * 9 * sizeof(storage) per node) and the
    counter bytes of the committed rocprofv3 summary, each over the launch
    time, against 8 TB/s."""
    out = {"bytes_model": "2*9*sizeof(storage) per node per K-step launch",
           "algorithmic_GBs": round(alg_bytes / launch_s / 1e9, 1),
           "algorithmic_frac_of_peak": round(alg_bytes / launch_s / 1e9 / HBM_PEAK_GBS, 4),
           "counter_GBs": None, "counter_frac_of_peak": None}
    if traffic:
        gbs = traffic / launch_s / 1e9
        out["counter_GBs"] = round(gbs, 1)
        out["counter_frac_of_peak"] = round(gbs / HBM_PEAK_GBS, 4)
    return out


def add_copy_fraction(hbm, copy_gbs):
    hbm["algorithmic_frac_of_copy"] = round(hbm["algorithmic_GBs"] / copy_gbs, 4)
    hbm["counter_frac_of_copy"] = (round(hbm["counter_GBs"] / copy_gbs, 4)
                                   if hbm["counter_GBs"] else None)


def copy_ceiling(oreg, torch, nbytes, reps=20):
    """GB/s of the library's plain streaming copy (lb_copy_device: every byte
    read once and written once) between two device buffers of nbytes, timed
    with HIP events on its stream: the practical HBM ceiling."""
    stream = torch.cuda.Stream()  # default priority
    src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    h = stream.cuda_stream
    for _ in range(3):
        oreg.copy_device(src.data_ptr(), dst.data_ptr(), nbytes, h)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        oreg.copy_device(src.data_ptr(), dst.data_ptr(), nbytes, h)
    end.record(stream)
    torch.cuda.synchronize()
    if not bool((dst[:: max(1, nbytes // 4096)] == 1).all()):
        raise RuntimeError("lb_copy_device did not copy")
    gbs = 2.0 * nbytes * reps / (start.elapsed_time(end) / 1e3) / 1e9
    del src, dst
    return gbs


def d3q27_bench(torch, n, tau, steps, copy_gbs=None):
    """The D3Q27 sweep (one launch per step) on an n^3 box, every storage."""
    from paper_2501_16000_amd import oreg3, workloads
    fields = workloads.shear_wave3(n, 0.05)
    out = {"workload": f"D3Q27 periodic {n}^3 OReg sweep, shear wave u0=0.05 normal to "
                       f"(1,1,1), guided equilibrium, theta=1/3, tau={tau}, one box per launch",
           "kernel": "sweep3_kernel<guided, OReg, storage>", "steps": steps}
    for st in ("f64", "f32s", "f16s", "bf16s"):
        ms, diag = time_box(oreg3, torch, n, tau, st, steps, 10, fields)
        if diag[6] != 0:
            raise RuntimeError(f"non-finite populations in the D3Q27 {st} run")
        launch_s = ms / 1e3 / steps
        alg = 2 * 27 * STORAGE_BYTES[st] * n ** 3
        ach = alg / launch_s / 1e9
        out[st] = {"value": round(n ** 3 / launch_s / 1e6, 1), "unit": "MLUPS",
                   "ms_per_step": round(launch_s * 1e3, 5),
                   "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                                "traffic": load_traffic(st, n, alg, d3=True),
                                "algorithmic_bytes_per_launch": alg}}
        if copy_gbs:
            out[st]["roofline"]["frac_of_copy"] = round(ach / copy_gbs, 4)
    return out


COPY_BYTES = 1 << 30
D3_PMC_N = 256


def workloads_shear_wave3(n):
    from paper_2501_16000_amd import workloads
    return workloads.shear_wave3(n, 0.05)


def pmc_workload(oreg, torch, n, tau, fields):
    """A few sweeps per storage and one plain 1 GiB device-to-device copy, the
    calibration of the HBM counters."""
    for st in ("f64", "f32s", "f16s", "bf16s"):
        time_lattice(oreg, torch, n, tau, st, 2 * FUSED_K[st], 0, fields)  # two full fused launches
        time_lattice(oreg, torch, n, tau, st, 5, 2, fields, fuse_steps=1)  # single steps
    from paper_2501_16000_amd import oreg3
    f3 = workloads_shear_wave3(D3_PMC_N)
    for st in ("f64", "f32s", "f16s", "bf16s"):
        time_box(oreg3, torch, D3_PMC_N, tau, st, 5, 2, f3)
    src = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()


def summarize_counters(paths, n):
    """Per-launch means of SQ / TCP counters for the D2Q9 sweep kernels, and
    the figures derived from them, as markdown tables."""
    import csv
    import re
    from collections import defaultdict
    vals = defaultdict(lambda: defaultdict(list))
    for path in paths:
        with open(path) as fh:
            for row in csv.DictReader(fh):
                m = re.search(r"((?:fused_)?sweep_kernel<[^>]*>)", row["Kernel_Name"])
                if m:
                    vals[m.group(1)][row["Counter_Name"]].append(float(row["Counter_Value"]))
    mean = {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in vals.items()}
    names = {"0": "F64", "1": "F32S", "2": "F16S", "3": "BF16S"}
    out = ["| kernel | node updates / launch | waves | VALU instr (wave) | VALU lane-instr / "
           "update | FP64 FMA / MUL / ADD per update | wave-cycles waiting to issue | "
           "wave-cycles in s_waitcnt | L2 read latency (cycles) | UTCL1 misses |",
           "|---|---|---|---|---|---|---|---|---|---|"]
    for k in sorted(mean):
        c = mean[k]
        args = [a.strip() for a in k.split("<")[1].rstrip(">").split(",")]
        fused = k.startswith("fused")
        st = names.get(args[4 if fused else 3], "?")  # <K, eq, coll, bc, storage[, buf]>
        steps = int(args[0]) if fused else 1
        upd = steps * n * n

        def g(name):
            return c.get(name)

        def per(name):
            v = g(name)
            return f"{v * 64 / upd:.1f}" if v is not None else "-"

        def frac(a, b):
            return f"{100 * g(a) / g(b):.0f} %" if g(a) is not None and g(b) else "-"

        lat = (f"{g('TCP_TCC_READ_REQ_LATENCY') / g('TCP_TCC_READ_REQ'):.0f}"
               if g("TCP_TCC_READ_REQ") else "-")
        kind = f"fused, {steps} steps" if k.startswith("fused") else "one step"
        out.append(f"| `{k}` ({st}, {kind}) | {upd:,} | {g('SQ_WAVES') or 0:.0f} | "
                   f"{g('SQ_INSTS_VALU') or 0:.4g} | {per('SQ_INSTS_VALU')} | "
                   f"{per('SQ_INSTS_VALU_FMA_F64')} / {per('SQ_INSTS_VALU_MUL_F64')} / "
                   f"{per('SQ_INSTS_VALU_ADD_F64')} | {frac('SQ_WAIT_INST_ANY', 'SQ_WAVE_CYCLES')} | "
                   f"{frac('SQ_WAIT_ANY', 'SQ_WAVE_CYCLES')} | {lat} | "
                   f"{g('TCP_UTCL1_TRANSLATION_MISS') or 0:.0f} |")
    print("\n".join(out))


def summarize_pmc(fetch_csv, write_csv, n):
    """HBM bytes per sweep launch from FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch), each scaled by the ratio of known bytes to the counter's
    reading for the plain copy."""
    import csv
    import re
    from collections import defaultdict

    def read(path, counter):
        """Mean counter value per kernel name, and the largest single dispatch
        of the runtime's copy kernel (the 1 GiB calibration copy)."""
        vals, copy = defaultdict(list), 0.0
        with open(path) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                v = float(row["Counter_Value"])
                vals[row["Kernel_Name"]].append(v)
                if "copyBuffer" in row["Kernel_Name"]:
                    copy = max(copy, v)
        return {k: sum(v) / len(v) for k, v in vals.items()}, copy

    fetch, copy_f = read(fetch_csv, "FETCH_SIZE")
    write, copy_w = read(write_csv, "WRITE_SIZE")
    f_scale = COPY_BYTES / (copy_f * 1024.0)
    w_scale = COPY_BYTES / (copy_w * 1024.0)
    out = {"source": "rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE of "
                     "`bench.py --pmc-workload`, scaled by a 1 GiB device copy",
           "copy_fetch_scale": f_scale, "copy_write_scale": w_scale,
           "kernel_source_sha": kernel_source_sha(), "kernels": {}}
    sts = {"Storage<0>": "f64", "Storage<1>": "f32s", "Storage<2>": "f16s", "Storage<3>": "bf16s"}
    for k, v in fetch.items():
        if "sweep" not in k or "batched" in k:
            continue
        st = next((name for tag, name in sts.items() if tag in k), None)
        if st is None or k not in write:
            continue
        fb = v * 1024.0 * f_scale
        wb = write[k] * 1024.0 * w_scale
        d3 = "sweep3_kernel" in k
        key = ("d3q27_" if d3 else "") + ("fused_" if "fused_sweep_kernel" in k else "") + st
        side = D3_PMC_N if d3 else n
        alg = (2 * 27 * STORAGE_BYTES[st] * side ** 3) if d3 else BYTES_PER_NODE[st] * n * n
        out["kernels"][key] = {"n": side,
                               "kernel_source_sha": kernel_source_sha(SOURCES_3D if d3 else SOURCES_2D),
                               "kernel": (re.search(r"\w+_kernel<[^>]*>", k) or re.search(".*", k)).group(0),
                               "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                               "hbm_bytes_per_launch": fb + wb,
                               "algorithmic_bytes_per_launch": alg,
                               "fetch_kib_raw": v, "write_kib_raw": write[k]}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def serving_bench(oreg, count, plain_count=0):
    """The serving stream: rotated shear waves, N log-uniform in 32..1024,
    tau ~ U[0.52, 1.2], u0 ~ U[0.005, 0.05], steps ~ U{200..5000}, FP32S.

    1. capacity: every request available at once (saturated server);
    2. Poisson arrivals at 0.8 x that capacity: p50 / p99 latency (arrival ->
       moments in host memory) and aggregate MLUPS over the run;
    3. the plain path on the same requests: one FP64 lattice per request,
       lb_step over all its steps, one lattice at a time; its results are the
       reference of the decay-rate errors;
    4. the saturated stream on an FP64 server (its results equal lb_step's
       bit for bit).
    Decay-rate errors of the served results are taken over every request of
    the stream whose FP64 wave decays by 0.05 <= ln(a0/aT) <= ln(1e4)."""
    import math

    import numpy as np

    from paper_2501_16000_amd import serve, workloads
    base = workloads.serving_requests(count=count, seed=16000, rate_hz=1.0)
    by_id = {r.rid: r for r in base}
    lup = np.array([r.n * r.n * r.steps for r in base], dtype=float)

    def amplitude(tag, m):
        """|Fourier coefficient| of u . e_perp on the wave's mode; the phase
        exp(-2 pi i (2x + y)/N) factors into an x and a y vector."""
        n = by_id[tag].n
        e_perp, _ = workloads.shear_wave_projection(1)
        k = np.arange(n)
        v = e_perp[0] * m[1] + e_perp[1] * m[2]
        return abs(np.exp(-2j * np.pi * k / n) @ (v @ np.exp(-4j * np.pi * k / n)))

    # throughput: no per-result work on the host beyond fetching the moments
    with serve.Server(memory_budget=16 << 30, max_active=256, storage="f32s") as srv:
        sat = serve.run_stream(srv, base, realtime=False)
    capacity = sat.node_updates / sat.wall_s
    rate = 0.8 * capacity / lup.mean()
    stream = workloads.serving_requests(count=count, seed=16000, rate_hz=rate)
    with serve.Server(memory_budget=16 << 30, max_active=256, storage="f32s") as srv:
        rep = serve.run_stream(srv, stream, realtime=True, keep_results=False)
    with serve.Server(memory_budget=64 << 30, max_active=256, storage="f64") as srv:
        sat64 = serve.run_stream(srv, base, realtime=False)
    # accuracy: the same streams again (untimed), keeping each result's wave
    # amplitude
    with serve.Server(memory_budget=16 << 30, max_active=256, storage="f32s") as srv:
        acc = serve.run_stream(srv, base, realtime=False, on_result=amplitude).results
    with serve.Server(memory_budget=64 << 30, max_active=256, storage="f64") as srv:
        acc64 = serve.run_stream(srv, base, realtime=False, on_result=amplitude).results
    # the plain one-lattice-per-launch FP64 path on the same requests (timed:
    # create, init, steps and moments in host memory, as a served result)
    checked = base[:plain_count] if plain_count > 0 else base
    plain_s, plain_lup, plain = 0.0, 0, {}
    for r in checked:
        fields = workloads.shear_wave(r.n, r.u0)
        t0 = time.perf_counter()
        with oreg.Lattice(r.n, r.n, r.tau, 1.0 / 3.0) as lat:
            lat.init(*fields)
            lat.step(r.steps)
            m = lat.moments()
        plain_s += time.perf_counter() - t0
        plain[r.rid] = amplitude(r.rid, m)
        plain_lup += r.n * r.n * r.steps
    errs, errs64, worst = [], [], None
    for r in checked:
        a0 = amplitude(r.rid, np.stack(workloads.shear_wave(r.n, r.u0)))
        ln_ref = math.log(a0 / plain[r.rid])
        # well-conditioned decays only: at least 5 % and the wave still at
        # 1e-4 of its start (below that the FP32 storage noise floor decides)
        if 0.05 <= ln_ref <= math.log(1e4):
            e = abs(math.log(a0 / acc[r.rid]) / ln_ref - 1)
            errs.append(e)
            errs64.append(abs(math.log(a0 / acc64[r.rid]) / ln_ref - 1))
            if worst is None or e > worst[0]:
                worst = (e, r)
    out = {
        "workload": f"{count} rotated shear-wave requests, N log-uniform 32..1024, "
                    "tau U[0.52,1.2], u0 U[0.005,0.05], steps U{200..5000}, FP32S storage, "
                    "guided equilibrium, Poisson arrivals at 0.8 x measured capacity",
        "rate_hz": round(rate, 2),
        "p50_latency_s": round(rep.percentile(50), 4),
        "p99_latency_s": round(rep.percentile(99), 4),
        "aggregate_mlups": round(rep.mlups, 1),
        "wall_s": round(rep.wall_s, 2),
        "saturated_mlups": round(sat.mlups, 1),
        "launches": rep.launches,
        "plain_f64_one_lattice_per_launch_mlups": round(plain_lup / plain_s / 1e6, 1),
        "plain_sample": (f"all {len(base)} requests of the stream" if len(checked) == len(base)
                         else f"first {len(checked)} requests of the stream"),
        "served_vs_plain_decay_rate_error": {
            "window": "0.05 <= ln(a0/aT) <= ln(1e4) of the FP64 run",
            "samples": len(errs),
            "max": float(max(errs)) if errs else None,
            "p50": float(np.median(errs)) if errs else None,
            "p99": float(np.percentile(errs, 99)) if errs else None},
        "f64_server": {
            "saturated_mlups": round(sat64.mlups, 1),
            "decay_rate_error_max_same_window": float(max(errs64)) if errs64 else None,
            "note": "FP64 storage, same stream and window; results equal lb_step bit for bit"},
    }
    if worst is not None:
        e, r = worst
        out["served_vs_plain_decay_rate_error"]["worst_request"] = {
            "rid": r.rid, "n": r.n, "tau": round(r.tau, 4), "u0": round(r.u0, 4),
            "steps": r.steps, "error": float(e)}
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n, tau, steps, fields, single_steps=2):
    import numpy as np

    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    f0 = oracle.init("guided", 1.0 / 3.0, *fields)
    t0 = time.perf_counter()
    f = oracle.run(f0, steps, tau, 1.0 / 3.0, "guided", nthreads=threads)
    dt = time.perf_counter() - t0
    assert np.isfinite(f[0, 0, 0])
    t0 = time.perf_counter()
    f = oracle.run(f0, single_steps, tau, 1.0 / 3.0, "guided", nthreads=1)
    dt1 = time.perf_counter() - t0
    assert np.isfinite(f[0, 0, 0])
    return {"value": n * n * steps / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{n}x{n} rotated shear wave, FP64, guided, tau={tau}, {steps} steps "
                      f"({dt:.1f} s, OpenMP over nodes, gcc -O2)",
            "cpu_model": cpu_model(),
            "single_thread": {"value": round(n * n * single_steps / dt1 / 1e6, 2), "unit": "MLUPS",
                              "sample": f"{single_steps} steps of the same lattice ({dt1:.1f} s)"}}


def main():
    args = parse()
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.n)
        return 0
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, args.n)
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the sweep's multi-GPU slab decomposition is design-only).", file=sys.stderr)
        return 2
    import torch

    from paper_2501_16000_amd import oreg, workloads

    torch.cuda.set_device(0)
    n, tau = args.n, args.tau
    fields = workloads.shear_wave(n, 0.05)
    if args.pmc_workload:
        pmc_workload(oreg, torch, n, tau, fields)
        return 0
    K = FUSED_K[args.storage]
    # The timed region is issued as its whole K-step launches and then the
    # remainder, with an event between: the first part times the dominant
    # kernel's launches alone, inside the same timed region.
    nl = args.steps // K if K > 1 else 0
    ms, diag, fms = time_lattice(oreg, torch, n, tau, args.storage, args.steps, args.warmup,
                                 fields, split=nl * K)
    if diag[5] != 0:
        raise RuntimeError("non-finite populations after the timed run")
    cells = n * n
    sec = ms / 1e3
    mlups = cells * args.steps / sec / 1e6
    alg_bytes = BYTES_PER_NODE[args.storage] * cells
    if nl > 0:
        # the dominant kernel: K steps per launch
        per_launch_s = fms / 1e3 / nl
        flops = FLOPS_PER_UPDATE * K * cells
        peak = FP64_PEAK_TFLOPS if args.storage == "f64" else FP32_PEAK_TFLOPS
        achieved = flops / per_launch_s / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": peak,
                    "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                    "traffic": load_traffic(args.storage, n, alg_bytes, fused=True),
                    "kernel": f"fused_sweep_kernel<K={K}, guided, OReg, periodic, {args.storage}>",
                    "launch_ms": round(per_launch_s * 1e3, 4),
                    "node_updates_per_launch": K * cells,
                    "flops_per_node_update": FLOPS_PER_UPDATE}
        roofline["hbm"] = hbm_side(roofline["traffic"], alg_bytes, per_launch_s)
    else:
        per_launch_s = sec / args.steps
        achieved = alg_bytes / per_launch_s / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": load_traffic(args.storage, n, alg_bytes),
                    "kernel": f"sweep_kernel<guided, OReg, periodic, {args.storage}>",
                    "algorithmic_bytes_per_launch": alg_bytes}
    # the single-step sweep of the same workload (one launch per step)
    sms, _ = time_lattice(oreg, torch, n, tau, args.storage, min(args.steps, 300), 10, fields,
                          fuse_steps=1)
    s_launch = sms / 1e3 / min(args.steps, 300)
    s_ach = alg_bytes / s_launch / 1e9
    single = {"value": round(cells / s_launch / 1e6, 1), "unit": "MLUPS",
              "kernel": f"sweep_kernel<guided, OReg, periodic, {args.storage}>",
              "roofline": {"bound": "hbm", "achieved": round(s_ach, 1), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(s_ach / HBM_PEAK_GBS, 4),
                           "traffic": load_traffic(args.storage, n, alg_bytes),
                           "algorithmic_bytes_per_launch": alg_bytes}}
    # the practical ceiling: a plain copy of one population buffer of this
    # lattice (each byte read once and written once, as one sweep step does)
    copy_bytes = alg_bytes // 2 // 16 * 16
    copy_gbs = copy_ceiling(oreg, torch, copy_bytes)
    copy = {"value": round(copy_gbs, 1), "unit": "GB/s", "kernel": "copy_kernel (lb_copy_device)",
            "bytes_per_copy": copy_bytes, "copies": 20}
    single["roofline"]["frac_of_copy"] = round(s_ach / copy_gbs, 4)
    if "hbm" in roofline:
        add_copy_fraction(roofline["hbm"], copy_gbs)

    # spread: five more timed runs of 300 steps each
    reps = []
    for _ in range(5):
        rms, _ = time_lattice(oreg, torch, n, tau, args.storage, 300, args.warmup, fields)
        reps.append(cells * 300 / (rms / 1e3) / 1e6)
    reps.sort()
    repeats = {"n": 5, "steps": 300, "median": round(reps[2], 1), "min": round(reps[0], 1),
               "max": round(reps[-1], 1), "unit": "MLUPS"}

    # the other relaxation times of the workload (same kernels, same work,
    # the same step count), in FP64 and in shifted FP32 storage
    tau_sweep = {}
    for st in dict.fromkeys((args.storage, "f32s")):
        tau_sweep[st] = {}
        for t_other in (0.51, 0.6, 1.0):
            if st == args.storage and t_other == tau:
                continue
            tms, tdiag = time_lattice(oreg, torch, n, t_other, st, args.steps, args.warmup,
                                      fields)
            if tdiag[5] != 0:
                raise RuntimeError(f"non-finite populations at tau={t_other} ({st})")
            tau_sweep[st][str(t_other)] = {
                "value": round(cells * args.steps / (tms / 1e3) / 1e6, 1), "unit": "MLUPS",
                "steps": args.steps}

    variants = {}
    for st in [s for s in args.variants.split(",") if s and s != args.storage]:
        vms, vdiag = time_lattice(oreg, torch, n, tau, st, args.variant_steps,
                                  min(args.warmup, 20), fields)
        vsec = vms / 1e3
        v_ach = BYTES_PER_NODE[st] * cells / (vsec / args.variant_steps) / 1e9
        entry = {"value": round(cells * args.variant_steps / vsec / 1e6, 1),
                 "unit": "MLUPS", "steps": args.variant_steps,
                 "ms_per_step": round(vms / args.variant_steps, 5),
                 "mass_drift_rel": float(abs(vdiag[0] - diag[0]) / diag[0])}
        if FUSED_K[st] > 1:
            # K steps per launch: bounded by VALU issue, not by HBM
            tf = FLOPS_PER_UPDATE * cells * args.variant_steps / vsec / 1e12
            traffic = load_traffic(st, n, BYTES_PER_NODE[st] * cells, fused=True)
            entry["roofline"] = {"bound": "alu", "achieved": round(tf, 2),
                                 "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                                 "frac": round(tf / FP32_PEAK_TFLOPS, 4),
                                 "kernel": f"fused_sweep_kernel<K={FUSED_K[st]}, {st}>",
                                 "traffic": traffic}
            entry["roofline"]["hbm"] = hbm_side(traffic, BYTES_PER_NODE[st] * cells,
                                                vsec / args.variant_steps * FUSED_K[st])
            add_copy_fraction(entry["roofline"]["hbm"], copy_gbs)
        else:
            entry["roofline"] = {"bound": "hbm", "achieved": round(v_ach, 1),
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": round(v_ach / HBM_PEAK_GBS, 4),
                                 "kernel": f"sweep_kernel<{st}>",
                                 "traffic": load_traffic(st, n, BYTES_PER_NODE[st] * cells)}
        variants[st] = entry

    line = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.storage == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"D2Q9 periodic {n}x{n} OReg sweep, rotated shear wave u0=0.05 "
                               f"along atan(1/2), guided equilibrium, theta=1/3, tau={tau}, "
                               f"{args.storage} storage, one lattice per launch",
                   "nx": n, "ny": n, "tau": tau, "storage": args.storage},
        "roofline": roofline,
        "repeats": repeats,
        "single_step": single,
        "copy_ceiling": copy,
        "tau_sweep": tau_sweep,
        "variants": variants,
    }
    if args.d3q27_n > 0:
        line["d3q27"] = d3q27_bench(torch, args.d3q27_n, tau, args.d3q27_steps, copy_gbs)
    if args.serving_requests > 0:
        line["serving"] = serving_bench(oreg, args.serving_requests, args.serving_plain_requests)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(n, tau, args.cpu_steps, fields)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

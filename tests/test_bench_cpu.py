"""Host logic of bench.py, without a GPU: the refusal of more than one GPU,
the rocprofv3 counter summaries (kernel names as the profiler prints them,
the 1 GiB copy calibration) and the staleness check of the committed HBM
traffic summary."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

FUSED = ("oreg::(anonymous namespace)::fused_sweep_kernel<7, 0, 0, 0, 0, true>"
         "(oreg::Storage<0>::T const*, oreg::Storage<0>::T*, oreg::Geometry, oreg::Coef64, int, int, int)")
SINGLE = ("oreg::(anonymous namespace)::sweep_kernel<0, 0, 0, 1>"
          "(oreg::Storage<1>::T const*, oreg::Storage<1>::T*, oreg::Geometry, oreg::Coef64, int)")
COPY = "__amd_rocclr_copyBuffer"


def write_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": counter, "Counter_Value": v})


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_summarize_pmc_scales_by_the_copy_and_keys_by_storage(tmp_path, monkeypatch):
    n = 4096
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    # FETCH_SIZE of the copy reads half the bytes (in KiB), WRITE_SIZE all of them
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    write_csv(fetch, "FETCH_SIZE", [(COPY, 524288.0), (FUSED, 700000.0), (FUSED, 710000.0),
                                    (SINGLE, 300000.0)])
    write_csv(write, "WRITE_SIZE", [(COPY, 1048576.0), (FUSED, 1200000.0), (FUSED, 1200000.0),
                                    (SINGLE, 590000.0)])
    bench.summarize_pmc(str(fetch), str(write), n)
    t = json.loads(out.read_text())
    assert t["copy_fetch_scale"] == pytest.approx(2.0)
    assert t["copy_write_scale"] == pytest.approx(1.0)
    f = t["kernels"]["fused_f64"]
    assert f["kernel"] == "fused_sweep_kernel<7, 0, 0, 0, 0, true>"
    assert f["fetch_bytes_per_launch"] == pytest.approx(705000.0 * 1024 * 2)
    assert f["write_bytes_per_launch"] == pytest.approx(1200000.0 * 1024)
    assert f["algorithmic_bytes_per_launch"] == 144 * n * n
    s = t["kernels"]["f32s"]
    assert s["kernel"] == "sweep_kernel<0, 0, 0, 1>"
    assert s["hbm_bytes_per_launch"] == pytest.approx((300000.0 * 2 + 590000.0) * 1024)
    # the entries carry the kernel sources' hash: load_traffic finds them for
    # this n and source tree, and not for another n
    assert bench.load_traffic("f64", n, 0, fused=True) == pytest.approx(f["hbm_bytes_per_launch"])
    assert bench.load_traffic("f64", 2048, 0, fused=True) is None


def test_load_traffic_rejects_a_summary_of_other_sources(tmp_path, monkeypatch):
    out = tmp_path / "traffic.json"
    out.write_text(json.dumps({"kernels": {"fused_f64": {
        "n": 4096, "kernel_source_sha": "0000000000000000", "hbm_bytes_per_launch": 1.0}}}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    assert bench.load_traffic("f64", 4096, 0, fused=True) is None


def test_summarize_counters_names_storage_and_steps(tmp_path, capsys):
    path = tmp_path / "sq.csv"
    rows = []
    for k, waves, valu in ((FUSED, 3036, 2.5e8), (SINGLE, 262144, 4.5e7)):
        rows += [(k, "SQ_WAVES", waves), (k, "SQ_INSTS_VALU", valu)]
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})
    bench.summarize_counters([str(path)], 4096)
    text = capsys.readouterr().out
    assert "`fused_sweep_kernel<7, 0, 0, 0, 0, true>` (F64, fused, 7 steps)" in text
    assert "`sweep_kernel<0, 0, 0, 1>` (F32S, one step)" in text
    # VALU lane-instructions per node update: 2.5e8 x 64 / (7 x 4096^2)
    assert f"{2.5e8 * 64 / (7 * 4096 * 4096):.1f}" in text


def test_hbm_side_reports_both_views():
    h = bench.hbm_side(2.0e9, 1.0e9, 1e-3)
    assert h["algorithmic_GBs"] == pytest.approx(1000.0)
    assert h["counter_GBs"] == pytest.approx(2000.0)
    assert h["counter_frac_of_peak"] == pytest.approx(2000.0 / bench.HBM_PEAK_GBS, abs=1e-4)
    assert bench.hbm_side(None, 1.0e9, 1e-3)["counter_GBs"] is None

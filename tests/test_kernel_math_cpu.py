"""The device collision of csrc/d2q9.hpp, compiled for the host CPU, against
the oracle one node at a time (no GPU needed).

FP64: the kernel's algebraic rearrangements of Eqs. (6), (7) and (11) agree
with the printed forms to a few ulp.  Shifted FP32: the absolute error per
population stays at FP32 rounding of the shifted values.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def output(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("collide")
    obj = d / "orc.o"
    subprocess.run(["gcc", "-O2", "-c", os.path.join(ROOT, "oracle", "oreg_oracle.c"), "-o",
                    str(obj)], check=True)
    hobj = d / "check.o"
    subprocess.run([hipcc, "-std=c++17", "-O2", "-x", "hip", "--offload-arch=gfx950",
                    "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2501_16000_amd", "csrc"),
                    "-c", os.path.join(ROOT, "tests", "host", "collide_check.cpp"),
                    "-o", str(hobj)], check=True, capture_output=True)
    exe = d / "check"
    subprocess.run([hipcc, "--offload-arch=gfx950", str(hobj), str(obj), "-o", str(exe)],
                   check=True, capture_output=True)
    return subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout


def test_collision_matches_oracle_on_host(output):
    rows = re.findall(r"f64_rel=(\S+) f32s_abs=(\S+)", output)
    assert len(rows) == 6, output
    for f64_rel, f32_abs in rows:
        assert float(f64_rel) < 5e-15, output
        assert float(f32_abs) < 1e-7, output  # ~7 ulp of the largest shifted value

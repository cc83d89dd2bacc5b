"""The device collisions of csrc/d2q9.hpp and csrc/d3q27.hpp, compiled for the
host CPU, against the oracles one node at a time (no GPU needed).

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


def build_and_run(d, oracle_src, check_src):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    obj = d / "orc.o"
    subprocess.run(["gcc", "-O2", "-c", os.path.join(ROOT, "oracle", oracle_src), "-o",
                    str(obj)], check=True)
    hobj = d / "check.o"
    subprocess.run([hipcc, "-std=c++17", "-O2", "-x", "hip", "--offload-arch=gfx950",
                    "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2501_16000_amd", "csrc"),
                    "-c", os.path.join(ROOT, "tests", "host", check_src),
                    "-o", str(hobj)], check=True, capture_output=True)
    exe = d / "check"
    subprocess.run([hipcc, "--offload-arch=gfx950", str(hobj), str(obj), "-o", str(exe)],
                   check=True, capture_output=True)
    return subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout


@pytest.fixture(scope="module")
def output(tmp_path_factory):
    return build_and_run(tmp_path_factory.mktemp("collide"), "oreg_oracle.c", "collide_check.cpp")


@pytest.fixture(scope="module")
def output3(tmp_path_factory):
    return build_and_run(tmp_path_factory.mktemp("collide3"), "oreg_oracle3.c",
                         "collide3_check.cpp")


def test_collision_matches_oracle_on_host(output):
    rows = re.findall(r"f64_rel=(\S+) f32s_abs=(\S+) f32u_abs=(\S+)", output)
    assert len(rows) == 6, output
    for f64_rel, f32_abs, f32u_abs in rows:
        assert float(f64_rel) < 5e-15, output
        assert float(f32_abs) < 1e-7, output  # ~7 ulp of the largest shifted value
        assert float(f32u_abs) < 1e-7, output  # u from drho / rho (F32S)


def test_d3q27_collision_matches_oracle_on_host(output3):
    rows = re.findall(r"f64_rel=(\S+) f32s_abs=(\S+)", output3)
    assert len(rows) == 6, output3
    for f64_rel, f32_abs in rows:
        assert float(f64_rel) < 1e-14, output3
        assert float(f32_abs) < 5e-8, output3  # the largest shifted value is ~0.3

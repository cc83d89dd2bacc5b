"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the CPU-side
code: both oracles (driven over small and degenerate shapes, every
equilibrium, collision and boundary) and the host-compiled device collisions
of csrc/d2q9.hpp and csrc/d3q27.hpp with their oracle checks.  The sanitizers
apply to host code only; the collision headers are compiled for the host
alone.  A run passes when it exits 0 and prints no sanitizer report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def check_clean(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert "runtime error" not in out and "AddressSanitizer" not in out, out
    return out


def test_oracles_under_asan_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_driver")
    run(["gcc", "-O1", "-g", "-std=c11", *SAN, "-I", os.path.join(ROOT, "oracle"),
         os.path.join(ROOT, "tests", "host", "oracle_driver.c"),
         os.path.join(ROOT, "oracle", "oreg_oracle.c"),
         os.path.join(ROOT, "oracle", "oreg_oracle3.c"), "-lm", "-o", exe])
    assert "oracle driver: ok" in check_clean(exe)


@pytest.mark.parametrize("check,oracle_src", [("collide_check.cpp", "oreg_oracle.c"),
                                               ("collide3_check.cpp", "oreg_oracle3.c")])
def test_host_collisions_under_asan_ubsan(tmp_path, check, oracle_src):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    clangxx = "/opt/rocm/llvm/bin/clang++"
    if not (os.path.exists(hipcc) and os.path.exists(clangxx) and shutil.which("gcc")):
        pytest.skip("hipcc / clang++ / gcc not available")
    orc = str(tmp_path / "orc.o")
    run(["gcc", "-O1", "-g", "-std=c11", *SAN, "-c", os.path.join(ROOT, "oracle", oracle_src),
         "-o", orc])
    obj = str(tmp_path / "check.o")
    # host-only compilation of the HIP source; each sanitizer flag for the host side
    host_san = [a for f in SAN for a in ("-Xarch_host", f)]
    run([hipcc, "-std=c++17", "-O1", "-g", "-x", "hip", "--cuda-host-only", *host_san,
         "-I", os.path.join(ROOT, "include"),
         "-I", os.path.join(ROOT, "paper_2501_16000_amd", "csrc"),
         "-c", os.path.join(ROOT, "tests", "host", check), "-o", obj])
    exe = str(tmp_path / "check")
    run([clangxx, *SAN, obj, orc, "-L/opt/rocm/lib", "-lamdhip64",
         "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    out = check_clean(exe)
    assert "f64_rel=" in out

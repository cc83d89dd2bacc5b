"""Host-side checks of the C ABI (no kernel launches): the library loads,
exports every entry point that include/oreg.h and include/oreg3.h declare,
and validates its arguments before it touches a device."""
import ctypes
import glob
import math
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def oreg():
    from paper_2501_16000_amd import oreg as m
    return m


def declared_functions():
    names = set()
    for path in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
        names |= set(re.findall(r"\b(lb3?_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("lb_create", "lb_init", "lb_step", "lb_moments"):
        assert required in names


def test_library_exports_every_declared_symbol():
    m = oreg()
    out = subprocess.run(["nm", "-D", "--defined-only", m.LIBRARY_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (lb3?_[a-z_0-9]+)$", out, flags=re.M))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, f"declared but not exported: {missing}"
    from paper_2501_16000_amd import oreg3, serve
    assert sorted(m.EXPORTED + serve.EXPORTED + oreg3.EXPORTED) == declared_functions()


def test_options_defaults_and_struct_layout():
    m = oreg()
    o = m.lb_options()
    m.lb_options_init(ctypes.byref(o))
    assert (o.nx, o.ny) == (0, 0)
    assert o.tau == 1.0 and abs(o.theta - 1 / 3) < 1e-16
    assert o.equilibrium == m.LB_EQ_GUIDED and o.storage == m.LB_F64
    assert o.collision == m.LB_COLL_OREG and o.boundary_x == m.LB_BC_PERIODIC
    assert o.rho0 == 1.0 and o.device == -1 and not o.stream and o.check_nonfinite == 0
    assert o.use_stream == 0 and o.fuse_steps == 0
    # C layout of lb_options: 2 ints, 2 doubles, 4 enums, double, pointer, 4 ints
    assert ctypes.sizeof(m.lb_options) == 4 * 2 + 8 * 2 + 4 * 4 + 8 + 8 + 4 * 4


INVALID = [
    dict(nx=0, ny=8), dict(nx=8, ny=-1), dict(tau=0.5), dict(tau=0.3), dict(tau=math.nan),
    dict(tau=math.inf), dict(theta=0.0), dict(theta=1.0), dict(theta=math.nan),
    dict(equilibrium=1, theta=0.35), dict(equilibrium=7), dict(storage=9), dict(collision=3),
    dict(boundary_x=5), dict(storage=1, rho0=0.0), dict(storage=2, rho0=-1.0),
    dict(storage=3, rho0=math.inf), dict(nx=1, ny=20_000_000), dict(fuse_steps=3),
    dict(fuse_steps=-1),
]


@pytest.mark.parametrize("bad", INVALID)
def test_create_rejects_invalid_options(bad):
    m = oreg()
    o = m.lb_options()
    m.lb_options_init(ctypes.byref(o))
    o.nx, o.ny, o.tau = 8, 8, 0.8
    for k, v in bad.items():
        setattr(o, k, v)
    h = ctypes.c_void_p(123)
    st = m.lb_create_ex(ctypes.byref(o), ctypes.byref(h))
    assert st == m.LB_EINVAL
    assert h.value is None
    assert m.lb_last_error(None).decode()


@pytest.mark.parametrize("storage,launchable", [(0, True), (1, False), (2, True), (3, True)])
def test_launch_size_limit_uses_each_storages_sweep_tile(storage, launchable):
    """The single-step sweep launches one thread per node on 256-node tiles
    (FP64: nx = 600 -> 768 threads per row) and on 512-node tiles (F32S: 1024
    threads per row), and one thread per two nodes on 512-node tiles (FP16S,
    BF16S: 512 threads per row).  With ny = 4.2e6 only the F32S launch exceeds
    2^32 work-items, which lb_create must refuse up front (not the first
    lb_step)."""
    import torch
    m = oreg()
    o = m.lb_options()
    m.lb_options_init(ctypes.byref(o))
    o.nx, o.ny, o.tau, o.storage = 600, 4_200_000, 0.8, storage
    h = ctypes.c_void_p()
    st = m.lb_create_ex(ctypes.byref(o), ctypes.byref(h))
    if not launchable:
        assert st == m.LB_EINVAL
        assert "too large" in m.lb_last_error(None).decode()
    else:
        assert st != m.LB_EINVAL  # passes validation: no device here, or too little memory
        if torch.cuda.device_count() == 0:
            assert st == m.LB_EDEVICE
        elif st == m.LB_OK:
            m.lb_destroy(h)


def test_null_arguments():
    m = oreg()
    assert m.lb_create(8, 8, 0.8, 1 / 3, 0, None) == m.LB_EINVAL
    assert m.lb_create_ex(None, ctypes.byref(ctypes.c_void_p())) == m.LB_EINVAL
    assert m.lb_step(None, 1) == m.LB_EINVAL
    assert m.lb_init(None, None, None, None) == m.LB_EINVAL
    assert m.lb_moments(None, None) == m.LB_EINVAL
    assert m.lb_sync(None) == m.LB_EINVAL
    assert m.lb_destroy(None) == m.LB_OK
    assert m.lb_time(None) == -1
    assert m.lb_device_bytes(None) == 0


def test_copy_device_validates_before_any_device_call():
    """The measurement copy rejects bad arguments on the host (no buffer is
    touched: the addresses below are never dereferenced)."""
    m = oreg()
    a, b = 1 << 20, 1 << 24
    assert m.lb_copy_device(None, b, 16, None) == m.LB_EINVAL
    assert m.lb_copy_device(a, None, 16, None) == m.LB_EINVAL
    assert m.lb_copy_device(a, b, -16, None) == m.LB_EINVAL
    assert m.lb_copy_device(a, b, 24, None) == m.LB_EINVAL          # not a multiple of 16
    assert m.lb_copy_device(a + 8, b, 16, None) == m.LB_EINVAL      # misaligned
    assert m.lb_copy_device(a, a + 64, 128, None) == m.LB_EINVAL    # overlapping
    assert "overlap" in m.lb_last_error(None).decode()
    assert m.lb_copy_device(a, b, 0, None) == m.LB_OK               # nothing to do


def test_status_strings():
    m = oreg()
    for code in (m.LB_OK, m.LB_EINVAL, m.LB_ENOMEM, m.LB_EDEVICE, m.LB_ESTATE, m.LB_ENONFINITE,
                 m.LB_EAGAIN):
        assert m.lb_status_string(code).decode().startswith("LB_")
    assert m.lb_status_string(42) == b"unknown lb_status"


def test_valid_create_without_device_reports_edevice():
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible; device creation is covered by the gpu tests")
    m = oreg()
    h = ctypes.c_void_p()
    assert m.lb_create(8, 8, 0.8, 1 / 3, m.LB_EQ_GUIDED, ctypes.byref(h)) == m.LB_EDEVICE
    assert h.value is None
    assert "device" in m.lb_last_error(None).decode()


def test_server_options_defaults_and_validation():
    from paper_2501_16000_amd import serve
    m = oreg()
    o = serve.lb_server_options()
    serve.lb_server_options_init(ctypes.byref(o))
    assert o.memory_budget == 16 << 30 and o.pinned_bytes == 1 << 30 and o.max_active == 256
    assert o.storage == m.LB_F32S and o.equilibrium == m.LB_EQ_GUIDED and o.device == -1
    h = ctypes.c_void_p()
    for field, bad in (("memory_budget", 0), ("max_active", 0), ("max_active", 70000),
                       ("storage", 7), ("theta", 1.5), ("rho0", -1.0)):
        o2 = serve.lb_server_options()
        serve.lb_server_options_init(ctypes.byref(o2))
        setattr(o2, field, bad)
        assert serve.lb_server_create(ctypes.byref(o2), ctypes.byref(h)) == m.LB_EINVAL
        assert serve.lb_server_last_error(None).decode()
    assert serve.lb_server_destroy(None) == m.LB_OK
    assert serve.lb_server_step(None, 1) == m.LB_EINVAL


def test_lb3_options_defaults_and_struct_layout():
    from paper_2501_16000_amd import oreg3
    m = oreg()
    o = oreg3.lb3_options()
    oreg3.lb3_options_init(ctypes.byref(o))
    assert (o.nx, o.ny, o.nz) == (0, 0, 0)
    assert o.tau == 1.0 and abs(o.theta - 1 / 3) < 1e-16 and o.rho0 == 1.0
    assert o.equilibrium == m.LB_EQ_GUIDED and o.storage == m.LB_F64
    assert o.collision == m.LB_COLL_OREG and o.device == -1 and o.use_stream == 0
    # 3 ints (+4 padding), 2 doubles, 3 enums (+4), double, pointer, 2 ints
    assert ctypes.sizeof(oreg3.lb3_options) == 16 + 16 + 16 + 8 + 8 + 8


INVALID3 = [
    dict(nx=0), dict(ny=-2), dict(nz=0), dict(tau=0.5), dict(tau=math.nan), dict(theta=0.0),
    dict(theta=1.0), dict(equilibrium=1, theta=0.4), dict(equilibrium=3), dict(storage=4),
    dict(collision=2), dict(storage=1, rho0=0.0), dict(storage=3, rho0=math.nan),
    dict(nx=64, ny=1 << 16, nz=1 << 16),
]


@pytest.mark.parametrize("bad", INVALID3)
def test_lb3_create_rejects_invalid_options(bad):
    from paper_2501_16000_amd import oreg3
    m = oreg()
    o = oreg3.lb3_options()
    oreg3.lb3_options_init(ctypes.byref(o))
    o.nx, o.ny, o.nz, o.tau = 8, 8, 8, 0.8
    for k, v in bad.items():
        setattr(o, k, v)
    h = ctypes.c_void_p(123)
    assert oreg3.lb3_create(ctypes.byref(o), ctypes.byref(h)) == m.LB_EINVAL
    assert h.value is None
    assert oreg3.lb3_last_error(None).decode()


def test_lb3_null_arguments_and_no_device():
    import torch
    from paper_2501_16000_amd import oreg3
    m = oreg()
    assert oreg3.lb3_create(None, ctypes.byref(ctypes.c_void_p())) == m.LB_EINVAL
    assert oreg3.lb3_step(None, 1) == m.LB_EINVAL
    assert oreg3.lb3_init(None, None, None, None, None) == m.LB_EINVAL
    assert oreg3.lb3_moments(None, None) == m.LB_EINVAL
    assert oreg3.lb3_diagnostics(None, None) == m.LB_EINVAL
    assert oreg3.lb3_sync(None) == m.LB_EINVAL
    assert oreg3.lb3_destroy(None) == m.LB_OK
    assert oreg3.lb3_time(None) == -1 and oreg3.lb3_device_bytes(None) == 0
    if torch.cuda.device_count() == 0:
        o = oreg3.lb3_options()
        oreg3.lb3_options_init(ctypes.byref(o))
        o.nx = o.ny = o.nz = 8
        h = ctypes.c_void_p()
        assert oreg3.lb3_create(ctypes.byref(o), ctypes.byref(h)) == m.LB_EDEVICE
        assert h.value is None


def test_binding_fails_loudly_without_the_library(tmp_path):
    """A copy of the package without liboreg.so cannot be imported: there is no
    other implementation to fall back to."""
    import shutil
    import sys
    pkg = os.path.join(ROOT, "paper_2501_16000_amd")
    dst = tmp_path / "paper_2501_16000_amd"
    shutil.copytree(pkg, dst, ignore=shutil.ignore_patterns("*.so", "__pycache__", "csrc"))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "try:\n"
            "    from paper_2501_16000_amd import oreg\n"
            "except ImportError as e:\n"
            "    print('IMPORTERROR', e)\n"
            "else:\n"
            "    print('LOADED', oreg.LIBRARY_PATH)\n") % str(tmp_path)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert "IMPORTERROR" in r.stdout and "liboreg.so" in r.stdout, r.stdout + r.stderr

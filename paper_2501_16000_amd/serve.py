"""Continuous-batching serving of independent OReg lattices (ctypes binding
of the ``lb_server_*`` entry points of ``liboreg.so``) and a request-stream
driver.

The server (native, ``csrc/serve.hip``) keeps every admitted lattice resident
in a device arena, advances all of them with one batched launch per time step
and retires each one after its own number of steps.  Python keeps only the
arrival clock and the queue of requests that did not fit yet:
``submit`` either admits a request at once or answers ``False`` (no slot or
arena space now), and the driver retries after the next steps.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field

import numpy as np

from . import oreg

_lib = oreg._lib
_VP = ctypes.c_void_p


class lb_server_options(ctypes.Structure):
    _fields_ = [
        ("memory_budget", ctypes.c_int64), ("pinned_bytes", ctypes.c_int64),
        ("max_active", ctypes.c_int), ("equilibrium", ctypes.c_int), ("storage", ctypes.c_int),
        ("theta", ctypes.c_double), ("rho0", ctypes.c_double), ("device", ctypes.c_int),
    ]


class lb_request(ctypes.Structure):
    _fields_ = [
        ("tag", ctypes.c_int64), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("tau", ctypes.c_double), ("steps", ctypes.c_int64),
        ("rho", _VP), ("ux", _VP), ("uy", _VP),
    ]


class lb_result(ctypes.Structure):
    _fields_ = [
        ("tag", ctypes.c_int64), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("steps", ctypes.c_int64), ("t_submit", ctypes.c_double), ("t_done", ctypes.c_double),
    ]


class lb_server_stats(ctypes.Structure):
    _fields_ = [
        ("active", ctypes.c_int), ("retiring", ctypes.c_int), ("ready", ctypes.c_int),
        ("device_bytes_used", ctypes.c_int64), ("launches", ctypes.c_int64),
        ("node_updates", ctypes.c_int64), ("clock", ctypes.c_double),
    ]


def _sig(name, res, args):
    fn = getattr(_lib, name)
    fn.restype = res
    fn.argtypes = args
    return fn


_H = ctypes.c_void_p
lb_server_options_init = _sig("lb_server_options_init", None, [ctypes.POINTER(lb_server_options)])
lb_server_create = _sig("lb_server_create", ctypes.c_int,
                        [ctypes.POINTER(lb_server_options), ctypes.POINTER(_H)])
lb_server_submit = _sig("lb_server_submit", ctypes.c_int, [_H, ctypes.POINTER(lb_request)])
lb_server_step = _sig("lb_server_step", ctypes.c_int, [_H, ctypes.c_int64])
lb_server_poll = _sig("lb_server_poll", ctypes.c_int, [_H, ctypes.POINTER(lb_result)])
lb_server_fetch = _sig("lb_server_fetch", ctypes.c_int, [_H, ctypes.c_int64, _VP])
lb_server_stats_get = _sig("lb_server_stats_get", ctypes.c_int,
                           [_H, ctypes.POINTER(lb_server_stats)])
lb_server_sync = _sig("lb_server_sync", ctypes.c_int, [_H])
lb_server_destroy = _sig("lb_server_destroy", ctypes.c_int, [_H])
lb_server_last_error = _sig("lb_server_last_error", ctypes.c_char_p, [_H])

EXPORTED = ["lb_server_options_init", "lb_server_create", "lb_server_submit", "lb_server_step",
            "lb_server_poll", "lb_server_fetch", "lb_server_stats_get", "lb_server_sync",
            "lb_server_destroy", "lb_server_last_error"]


class Server:
    """A continuous-batching server on one GPU.  Not thread-safe."""

    def __init__(self, memory_budget: int = 16 << 30, pinned_bytes: int = 1 << 30,
                 max_active: int = 256, equilibrium: str = "guided", storage: str = "f32s",
                 theta: float = 1.0 / 3.0, rho0: float = 1.0, device: int = -1):
        o = lb_server_options()
        lb_server_options_init(ctypes.byref(o))
        o.memory_budget, o.pinned_bytes, o.max_active = memory_budget, pinned_bytes, max_active
        o.equilibrium = oreg.EQUILIBRIA[equilibrium]
        o.storage = oreg.STORAGES[storage]
        o.theta, o.rho0, o.device = theta, rho0, device
        h = _H()
        st = lb_server_create(ctypes.byref(o), ctypes.byref(h))
        if st != oreg.LB_OK:
            raise oreg.LBError(st, "lb_server_create failed")
        self._h = h

    def _check(self, st):
        if st != oreg.LB_OK:
            raise oreg.LBError(st, (lb_server_last_error(self._h) or b"").decode())

    def submit(self, tag: int, rho, ux, uy, tau: float, steps: int) -> bool:
        """Admit now (True) or report no room (False)."""
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (rho, ux, uy)]
        ny, nx = arrs[0].shape
        r = lb_request(tag, nx, ny, float(tau), int(steps),
                       *[a.ctypes.data_as(_VP) for a in arrs])
        st = lb_server_submit(self._h, ctypes.byref(r))
        if st == oreg.LB_EAGAIN:
            return False
        self._check(st)
        return True

    def step(self, n: int = 1) -> None:
        """Issue up to n batched launches (each advances every resident lattice
        by up to 6 time steps)."""
        self._check(lb_server_step(self._h, int(n)))

    def poll(self):
        """The next finished result's metadata, or None."""
        r = lb_result()
        st = lb_server_poll(self._h, ctypes.byref(r))
        if st == oreg.LB_EAGAIN:
            return None
        self._check(st)
        return r

    def fetch(self, res: lb_result) -> np.ndarray:
        out = np.empty((3, res.ny, res.nx))
        self._check(lb_server_fetch(self._h, res.tag, out.ctypes.data_as(_VP)))
        return out

    def stats(self) -> lb_server_stats:
        s = lb_server_stats()
        self._check(lb_server_stats_get(self._h, ctypes.byref(s)))
        return s

    def sync(self) -> None:
        self._check(lb_server_sync(self._h))

    def close(self) -> None:
        if getattr(self, "_h", None):
            lb_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class StreamReport:
    results: dict = field(default_factory=dict)    # tag -> moments [3, ny, nx]
    latency_s: dict = field(default_factory=dict)  # tag -> arrival -> result in host memory
    node_updates: int = 0
    wall_s: float = 0.0
    launches: int = 0

    def percentile(self, q: float) -> float:
        return float(np.percentile(np.array(list(self.latency_s.values())), q))

    @property
    def mlups(self) -> float:
        return self.node_updates / self.wall_s / 1e6


def shear_wave_fields(n: int, u0: float):
    """Fields of the rotated shear wave of workloads.shear_wave."""
    from .workloads import shear_wave
    return shear_wave(n, u0)


class _FieldPrefetch:
    """Builds request fields on a helper thread, in arrival order, a bounded
    number of requests ahead (numpy releases the GIL for the array work)."""

    def __init__(self, requests, ahead: int = 32):
        import queue
        import threading
        self._q = queue.Queue(maxsize=ahead)
        self._stop = False

        def work():
            for r in requests:
                if self._stop:
                    return
                self._q.put((r.rid, shear_wave_fields(r.n, r.u0)))

        self._t = threading.Thread(target=work, daemon=True)
        self._t.start()
        self._ready = {}

    def get(self, rid):
        while rid not in self._ready:
            k, v = self._q.get()
            self._ready[k] = v
        return self._ready.pop(rid)

    def close(self):
        self._stop = True
        while self._t.is_alive():
            try:
                self._q.get_nowait()
            except Exception:
                self._t.join(0.01)


def run_stream(server: Server, requests, realtime: bool = True, steps_per_call: int = 4,
               keep_results: bool = False, timeout_s: float = 600.0,
               on_result=None) -> StreamReport:
    """Drive ``requests`` (workloads.ServingRequest) through ``server``.

    Requests become visible at their arrival time (``realtime``) or all at
    once; those that do not fit wait in arrival order.  Latency = arrival (or
    start, without realtime) -> the result's moments in host memory.
    ``keep_results`` keeps every result's moments; ``on_result(tag, moments)``
    instead keeps only what it returns (for long streams)."""
    pending = sorted(requests, key=lambda r: r.arrival_s)
    fields = _FieldPrefetch(pending)
    queue = []
    held = {}  # fields of queued requests that did not fit yet
    report = StreamReport()
    arrival_wall = {}
    i = 0
    done = 0
    s0 = server.stats()
    t0 = time.perf_counter()
    try:
        while done < len(pending):
            now = time.perf_counter() - t0
            if now > timeout_s:
                raise TimeoutError(f"serving stream unfinished after {timeout_s} s "
                                   f"({done}/{len(pending)} done)")
            while i < len(pending) and (not realtime or pending[i].arrival_s <= now):
                queue.append(pending[i])
                arrival_wall[pending[i].rid] = t0 + (pending[i].arrival_s if realtime else 0.0)
                i += 1
            while queue:
                r = queue[0]
                rho, ux, uy = held.pop(r.rid) if r.rid in held else fields.get(r.rid)
                if not server.submit(r.rid, rho, ux, uy, r.tau, r.steps):
                    held[r.rid] = (rho, ux, uy)
                    break
                queue.pop(0)
            server.step(steps_per_call)
            while True:
                res = server.poll()
                if res is None:
                    break
                m = server.fetch(res)
                report.latency_s[res.tag] = time.perf_counter() - arrival_wall[res.tag]
                if on_result is not None:
                    report.results[res.tag] = on_result(res.tag, m)
                elif keep_results:
                    report.results[res.tag] = m
                done += 1
            if realtime and i < len(pending) and not queue and server.stats().active == 0:
                # idle until the next arrival
                time.sleep(max(0.0, min(pending[i].arrival_s - (time.perf_counter() - t0), 0.01)))
        server.sync()
    finally:
        fields.close()
    s1 = server.stats()
    report.wall_s = time.perf_counter() - t0
    report.node_updates = s1.node_updates - s0.node_updates
    report.launches = s1.launches - s0.launches
    return report

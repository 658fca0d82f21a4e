"""Python handle on the libcbct serving runtime (cbct_server_*), and a harness that replays a
request stream with given arrival times and reports latency percentiles and throughput."""
from __future__ import annotations

import ctypes as C
import threading
import time

import numpy as np

from ._lib import GeometryDesc, check, context, lib


def _desc(g):
    angles = getattr(g, "angles", None)
    arr = (C.c_double * len(angles))(*angles) if angles is not None else None
    d = GeometryDesc(int(g.nx), int(g.ny), int(g.nz), float(g.hx), float(g.hy), float(g.hz), int(g.nu), int(g.nv),
                     float(g.pu), float(g.pv), float(g.sad), float(g.sdd), int(g.n_views),
                     C.cast(arr, C.POINTER(C.c_double)) if arr is not None else None,
                     float(getattr(g, "sample_ratio", 1.0)))
    return d, arr


class Server:
    """Continuous-admission reconstruction server on the current device (or simulated)."""

    def __init__(self, budget_bytes: float = 200e9, max_slots: int = 8, simulated: bool = False):
        self.simulated = simulated
        h = C.c_void_p()
        if simulated:
            check(lib().cbct_server_create_simulated(C.c_size_t(int(budget_bytes)), int(max_slots), C.byref(h)))
        else:
            import torch
            ctx = context(torch.cuda.current_device())
            check(lib().cbct_server_create(ctx, C.c_size_t(int(budget_bytes)), int(max_slots), C.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, geom, y=None, out=None, lam=0.05, iters=(30,), seconds=0.0, **kw) -> int:
        """Queue a reconstruction of `y` (torch GPU tensor, or numpy array for host input) into
        `out` (torch GPU tensor).  In simulated mode `seconds` is the request's service time."""
        from .ops import Plan
        params, keep = Plan.solve_params(lam, iters, **kw)
        d, arr = _desc(geom)
        t = C.c_uint64()
        if self.simulated:
            check(lib().cbct_server_submit_simulated(self._h, C.byref(d), C.byref(params), float(seconds),
                                                     C.byref(t)))
        else:
            if isinstance(y, np.ndarray):
                y = np.ascontiguousarray(y, dtype=np.float32)
                ptr, on_host = y.ctypes.data, 1
            else:
                ptr, on_host = y.data_ptr(), 0
            check(lib().cbct_server_submit(self._h, C.byref(d), C.byref(params), ptr, on_host, out.data_ptr(),
                                           C.byref(t)))
        self._keep[t.value] = (y, out, arr, keep)
        return t.value

    def poll(self, ticket: int):
        done, st, lat = C.c_int(), C.c_int(), C.c_double()
        check(lib().cbct_server_poll(self._h, ticket, C.byref(done), C.byref(st), C.byref(lat)))
        return bool(done.value), st.value, lat.value

    def times(self, ticket: int):
        t = (C.c_double * 3)()
        check(lib().cbct_server_request_times(self._h, ticket, t))
        return tuple(t)

    def wait_all(self):
        check(lib().cbct_server_wait_all(self._h))

    def stats(self):
        a, b, c, d, e, f = C.c_size_t(), C.c_size_t(), C.c_int(), C.c_int(), C.c_int(), C.c_uint64()
        check(lib().cbct_server_stats(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(d), C.byref(e),
                                      C.byref(f)))
        return dict(in_use=a.value, peak_in_use=b.value, running=c.value, peak_running=d.value, queued=e.value,
                    completed=f.value)

    def batch_stats(self):
        """(batched launches, request items they carried) of the batch engine."""
        a, b = C.c_uint64(), C.c_uint64()
        check(lib().cbct_server_batch_stats(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def close(self):
        if getattr(self, "_h", None):
            lib().cbct_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def replay(server: Server, arrivals, make_request):
    """Submit request r at wall time arrivals[r] (seconds after start); make_request(r) returns
    the submit() keyword arguments.  Waits for all; returns per-request latencies (s) and the
    span from the first submit to the last completion."""
    tickets = [None] * len(arrivals)
    t0 = time.perf_counter()
    for r, ta in enumerate(arrivals):
        dt = ta - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        tickets[r] = server.submit(**make_request(r))
    server.wait_all()
    lat = np.array([server.poll(t)[2] for t in tickets])
    times = np.array([server.times(t) for t in tickets])
    span = float(times[:, 2].max() - times[:, 0].min())
    return lat, span, tickets


def summarize(lat, span):
    return dict(p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                mean_s=float(lat.mean()), requests=int(len(lat)), span_s=span, req_per_s=len(lat) / span)

"""Python front end of the serving engine (include/exohip_serve.h).

The engine (C++, in libexohip.so) queues requests, admits them by memory
and free stream slots, and overlaps their kernels on the GPU.  This module
only marshals arguments, owns the output tensors until a request is waited
for, and drives seeded arrival processes.
"""
from __future__ import annotations

import ctypes
import threading
import time
from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import torch

from . import _lib as L
from .api import Atmos, Context, Response, _prec


class ExoServerCounters(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("submitted", "admitted", "completed", "failed", "rejected", "queued", "in_flight",
                 "peak_in_flight", "bypasses")] + \
               [(n, ctypes.c_double) for n in ("mem_budget_bytes", "mem_in_use_bytes", "mem_peak_bytes")]


def _bind(lib):
    if getattr(lib, "_serve_bound", False):
        return
    V, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    sig = {
        "exo_server_create": ([V, I, ctypes.c_size_t, ctypes.POINTER(V)], I),
        "exo_server_destroy": ([V], I),
        "exo_server_set_policy": ([V, I, I], I),
        "exo_server_submit": ([V, ctypes.POINTER(L.ExoAtmos), ctypes.POINTER(L.ExoResponse), I, V, D,
                               ctypes.POINTER(I64)], I),
        "exo_server_wait": ([V, I64, D, ctypes.POINTER(D), ctypes.POINTER(D)], I),
        "exo_server_stats": ([V, ctypes.POINTER(ExoServerCounters)], I),
        "exo_workspace_bytes": ([V, ctypes.POINTER(L.ExoAtmos), ctypes.POINTER(L.ExoResponse), I],
                                ctypes.c_size_t),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    lib._serve_bound = True


@dataclass
class Result:
    flux: torch.Tensor
    latency_s: float
    queue_s: float


class Server:
    """Continuous-batching server bound to a Context (its resident line lists and grid)."""

    def __init__(self, ctx: Context, n_streams: int = 4, mem_budget_bytes: int = 32 << 30):
        self._lib = L.load_library()
        _bind(self._lib)
        self.ctx = ctx
        h = ctypes.c_void_p()
        L.check(self._lib.exo_server_create(ctx.handle, int(n_streams), int(mem_budget_bytes), ctypes.byref(h)))
        self._h = h
        self._out = {}
        self._lock = threading.Lock()

    def close(self):
        if getattr(self, "_h", None):
            L.check(self._lib.exo_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    POLICIES = {"fifo": 0, "shortest": 1}

    def set_policy(self, policy: str = "fifo", max_passes: int = 16):
        """Admission order: "fifo" (arrival order) or "shortest" (fewest
        evaluations first; a request is passed over at most max_passes times)."""
        L.check(self._lib.exo_server_set_policy(self._h, self.POLICIES[policy], int(max_passes)))

    def workspace_bytes(self, atmos: Atmos, response: Optional[Response], precision="fp32") -> int:
        a, keep = atmos.to_c()
        r = response.to_c() if response is not None else None
        return int(self._lib.exo_workspace_bytes(self.ctx.handle, ctypes.byref(a),
                                                 ctypes.byref(r) if r is not None else None, _prec(precision)))

    def submit(self, atmos: Atmos, response: Optional[Response] = None, precision="fp32",
               arrival_s: float = 0.0) -> int:
        """Queue one spectrum; arrival_s (time.monotonic() seconds, 0: now) is
        the instant latency and queue time are measured from."""
        p = _prec(precision)
        dt = torch.float32 if p == L.EXO_FP32_KAHAN else torch.float64
        n = int(response.out_len) if response is not None else (int(atmos.grid_len) or self.ctx.n_nu)
        out = torch.empty(n, dtype=dt, device=f"cuda:{self.ctx.device}")
        a, keep = atmos.to_c()
        r = response.to_c() if response is not None else None
        t = ctypes.c_int64()
        L.check(self._lib.exo_server_submit(self._h, ctypes.byref(a), ctypes.byref(r) if r is not None else None,
                                            p, ctypes.c_void_p(out.data_ptr()), float(arrival_s),
                                            ctypes.byref(t)))
        with self._lock:
            self._out[t.value] = out
        return t.value

    def wait(self, ticket: int, timeout_s: float = -1.0) -> Result:
        lat, q = ctypes.c_double(), ctypes.c_double()
        rc = self._lib.exo_server_wait(self._h, int(ticket), float(timeout_s), ctypes.byref(lat), ctypes.byref(q))
        with self._lock:
            out = self._out.pop(ticket, None) if rc != L.EXO_EINVAL else self._out.get(ticket)
        L.check(rc)
        return Result(out, lat.value, q.value)

    def stats(self) -> dict:
        c = ExoServerCounters()
        L.check(self._lib.exo_server_stats(self._h, ctypes.byref(c)))
        return {k: getattr(c, k) for k, _ in c._fields_}


def run_stream(server: Server, requests: List[tuple], arrival_s: Optional[np.ndarray] = None,
               precision="fp32", progress: int = 0) -> dict:
    """Submit (atmos, response) pairs at the given arrival times (seconds from
    start; None = all at once) and wait for all.  Each request's latency is
    measured from its scheduled arrival, so a submitter that falls behind
    the schedule adds to it.  progress > 0 prints a line to stderr every
    `progress` submissions.  Returns latencies, results and throughput."""
    import sys
    n = len(requests)
    tickets = [None] * n
    t0 = time.monotonic()

    def submitter():
        for i, (a, r) in enumerate(requests):
            due = t0 + (float(arrival_s[i]) if arrival_s is not None else 0.0)
            delay = due - time.monotonic()
            if delay > 0:
                time.sleep(delay)
            tickets[i] = server.submit(a, r, precision, arrival_s=due)
            if progress and (i + 1) % progress == 0:
                st = server.stats()
                print(f"serving: submitted {i + 1}/{n} at {time.monotonic() - t0:.1f} s, "
                      f"{st['completed']} done, {st['queued']} queued", file=sys.stderr, flush=True)

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    results = [server.wait(t) for t in tickets]
    torch.cuda.synchronize()
    wall = time.monotonic() - t0
    lat = np.array([r.latency_s for r in results])
    return {"results": results, "latency_s": lat, "wall_s": wall,
            "spectra_per_s": n / wall,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3)}

"""Binding of the serving runtime of ``libmg355.so`` (``mg_server_*`` in ``include/mg355.h``).

The scheduler, admission by HBM footprint, the pool of resident hierarchies and the worker
threads with their HIP streams are native; this module only builds the request array from
torch tensors and reads the results back.

    srv = Server(workers=4)
    out = srv.run([Request(rho=r, dx=1/256, bc="periodic", arrival_ms=t) for r, t in ...])
    summary(out)   # p50 / p99 latency, throughput
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

from . import _abi, boundary, params
from ._abi import MG_OK, MG_SERVE_FIFO, MG_SERVE_SKIP, MgError, STATUS_NAMES

__all__ = ["Server", "Request", "summary"]


@dataclass
class Request:
    """One solve.  ``rho``/``phi``: contiguous float64 (n, n, n) device tensors (``phi`` None:
    the result goes to the hierarchy's own slot and is discarded).  In simulate mode ``rho`` may
    be None and ``n`` gives the size."""
    rho: object = None
    dx: float = 0.0
    bc: object = "periodic"
    n: int = 0
    tol: float = 1e-10
    max_cycles: int = 50
    fixed_cycles: int = 0
    precision: str = "fp64"
    mode: str = "fmg"
    layout: str = "dense"
    block_n: int = 16
    scheme: str = "cs"
    lmax: int = 4
    fixed_b: Optional[Sequence] = None
    phi: object = None
    arrival_ms: float = 0.0
    sim_ms: float = 0.0
    want_hist: bool = False
    # results
    status: int = 0
    hist: List[float] = field(default_factory=list)
    n_hist: int = 0
    resid: float = 0.0
    admit_ms: float = 0.0
    start_ms: float = 0.0
    end_ms: float = 0.0
    worker: int = -1
    reused: bool = False

    @property
    def latency_ms(self) -> float:
        return self.end_ms - self.arrival_ms


def _dev_ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("device tensors must be contiguous CUDA/HIP tensors")
    return t.data_ptr()


class Server:
    """Owns an ``mg_server``: ``workers`` host threads, one HIP stream each, and the pool of
    resident hierarchies (kept across ``run`` calls)."""

    def __init__(self, device: int = 0, workers: int = 4, hbm_budget: int = 0, policy: str = "fifo",
                 simulate: bool = False):
        self._lib = _abi.lib()
        cfg = _abi.MgServerConfig()
        cfg.device = int(device)
        cfg.workers = int(workers)
        cfg.hbm_budget = int(hbm_budget)
        cfg.policy = {"fifo": MG_SERVE_FIFO, "skip": MG_SERVE_SKIP}[policy]
        cfg.simulate = 1 if simulate else 0
        h = ctypes.c_void_p()
        st = self._lib.mg_server_create(ctypes.byref(h), ctypes.byref(cfg))
        if st != MG_OK:
            raise MgError(f"mg_server_create failed: {STATUS_NAMES.get(st, st)}")
        self.handle = h
        self.simulate = simulate

    def close(self):
        if getattr(self, "handle", None):
            self._lib.mg_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, n: int, precision: str = "fp64", count: int = 1, layout: str = "dense", block_n: int = 16,
                scheme: str = "cs"):
        p = params(n, 1.0 / n, precision=precision, layout=layout, block_n=block_n, scheme=scheme)
        st = self._lib.mg_server_reserve(self.handle, ctypes.byref(p), int(count))
        if st != MG_OK:
            raise MgError(f"mg_server_reserve: {STATUS_NAMES.get(st, st)}: "
                          f"{self._lib.mg_server_last_error(self.handle).decode()}")

    def run(self, requests: Sequence[Request]) -> Sequence[Request]:
        arr = (_abi.MgRequest * len(requests))()
        keep = []
        for i, r in enumerate(requests):
            n = r.n or (r.rho.shape[0] if r.rho is not None else 0)
            dx = r.dx or (1.0 / n if n else 0.0)
            q = arr[i]
            q.params = params(n, dx, tol=r.tol, max_cycles=r.max_cycles, fixed_cycles=r.fixed_cycles,
                              precision=r.precision, mode=r.mode, layout=r.layout, block_n=r.block_n,
                              scheme=r.scheme)
            q.bc = boundary(r.bc, r.fixed_b, r.lmax)
            q.rho = _dev_ptr(r.rho) if not self.simulate else None
            q.phi = _dev_ptr(r.phi) if not self.simulate else None
            q.arrival_ms = float(r.arrival_ms)
            q.sim_ms = float(r.sim_ms)
            if r.want_hist:
                h = (ctypes.c_double * (max(r.max_cycles, r.fixed_cycles) + 1))()
                keep.append(h)
                q.hist = h
                q.hist_cap = len(h)
        st = self._lib.mg_server_run(self.handle, arr, len(requests))
        if st != MG_OK:
            raise MgError(f"mg_server_run: {STATUS_NAMES.get(st, st)}")
        for i, r in enumerate(requests):
            q = arr[i]
            r.status, r.n_hist, r.resid = q.status, q.n_hist, q.resid
            r.admit_ms, r.start_ms, r.end_ms = q.admit_ms, q.start_ms, q.end_ms
            r.worker, r.reused = q.worker, bool(q.reused)
            r.hist = [q.hist[k] for k in range(min(q.n_hist, q.hist_cap))] if r.want_hist else []
        return requests

    def stats(self) -> dict:
        s = _abi.MgServerStats()
        self._lib.mg_server_get_stats(self.handle, ctypes.byref(s))
        return {k: getattr(s, k) for k, _ in s._fields_}


def _pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def summary(reqs: Sequence[Request]) -> dict:
    """Latency percentiles (arrival to completion), throughput and status counts of a run."""
    done = [r for r in reqs if r.status >= 0]
    lat = [r.latency_ms for r in done]
    span = (max(r.end_ms for r in reqs) - min(r.arrival_ms for r in reqs)) if reqs else 0.0
    dof = sum((r.n or (r.rho.shape[0] if r.rho is not None else 0)) ** 3 for r in done)
    return {"requests": len(reqs), "completed": len(done), "errors": len(reqs) - len(done),
            "latency_ms": {"p50": _pct(lat, 0.5), "p99": _pct(lat, 0.99), "mean": sum(lat) / len(lat) if lat else None},
            "makespan_ms": span, "solves_per_s": len(done) / (span * 1e-3) if span > 0 else None,
            "gdof_per_s": dof / (span * 1e-3) / 1e9 if span > 0 else None}

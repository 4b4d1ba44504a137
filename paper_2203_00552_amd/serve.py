"""Continuous-batching server for ddLPB energy + forces requests on one GPU.

Requests (a cluster with its model parameters) arrive over time.  Up to ``slots``
requests are in flight at once; each runs on its own HIP stream with its own
device workspace, so the kernels of different requests overlap on the device,
and the host-side waits inside one solve block only that request's thread.  A
request is admitted when a slot is free and the workspaces in flight plus its own
fit in the HBM budget; requests are admitted in arrival order.  All numerics run
in the HIP library; this module schedules contexts and records latencies.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from concurrent.futures import Future

import numpy as np

from ._lib import Context, DDLPBError


@dataclasses.dataclass
class Request:
    centers: np.ndarray
    radii: np.ndarray
    charges: np.ndarray
    lmax: int = 8
    n_lebedev: int = 302
    tol: float = 1e-6
    precision: int = 0
    fmm_order: int | None = None  # None: chosen from the atom count
    eps_in: float = 1.0
    eps_out: float = 78.54
    kappa: float = 0.104
    rid: int = 0


@dataclasses.dataclass
class Result:
    rid: int
    atoms: int
    energy: float
    forces: np.ndarray
    t_submit: float
    t_admit: float
    t_done: float
    workspace_bytes: int
    iters: tuple
    residuals: tuple = (0.0, 0.0)  # relative residuals reached by the primal and adjoint solves
    converged: bool = True

    @property
    def latency(self):
        return self.t_done - self.t_submit


class Server:
    """``slots`` concurrent requests, ``hbm_budget`` bytes of workspaces in flight
    (default: 80 % of the free device memory at start).  Requests with at least
    ``fmm_threshold`` atoms use the FMM of order max(fmm_order, lmax + 1).  A solve
    that stops at the iteration limit still returns its result, flagged as not
    converged, with the residual it reached."""

    def __init__(self, slots=4, hbm_budget=None, fmm_threshold=2000, fmm_order=12, options=None):
        import torch
        self.torch = torch
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(0.8 * free)
        self.budget = int(hbm_budget)
        self.fmm_threshold = fmm_threshold
        self.fmm_order = fmm_order
        self.options = dict(options or {})
        self.in_flight = 0
        self.bytes_in_flight = 0
        self.max_in_flight = 0
        self._queue = collections.deque()
        self._cv = threading.Condition()
        self._closed = False
        self._threads = [threading.Thread(target=self._worker, daemon=True) for _ in range(slots)]
        for t in self._threads:
            t.start()

    # ------------------------------------------------------------------ api
    def submit(self, req: Request) -> Future:
        fut = Future()
        with self._cv:
            if self._closed:
                raise RuntimeError("server closed")
            self._queue.append((req, fut, time.perf_counter()))
            self._cv.notify_all()
        return fut

    def close(self):
        with self._cv:
            self._closed = True
            self._cv.notify_all()
        for t in self._threads:
            t.join()

    # ------------------------------------------------------------ internals
    def _order(self, req):
        if req.fmm_order is not None:
            return req.fmm_order
        if len(req.radii) < self.fmm_threshold:
            return 0
        return max(self.fmm_order, req.lmax + 1)

    def _worker(self):
        torch = self.torch
        stream = torch.cuda.Stream()
        while True:
            with self._cv:
                while not self._queue and not self._closed:
                    self._cv.wait()
                if not self._queue:
                    return
                req, fut, t_sub = self._queue.popleft()
            try:
                ctx = Context(req.centers, req.radii, req.charges, eps_in=req.eps_in, eps_out=req.eps_out,
                              kappa=req.kappa, lmax=req.lmax, n_lebedev=req.n_lebedev,
                              fmm_order=self._order(req), options=dict(self.options, precision=req.precision))
            except Exception as e:  # invalid request
                fut.set_exception(e)
                continue
            need = ctx.workspace_bytes()
            with self._cv:
                if need > self.budget:
                    ctx.close()
                    fut.set_exception(DDLPBError(-3, f"request {req.rid}: workspace {need} B exceeds the budget"))
                    continue
                while self.bytes_in_flight + need > self.budget:
                    self._cv.wait()
                self.bytes_in_flight += need
                self.in_flight += 1
                self.max_in_flight = max(self.max_in_flight, self.in_flight)
            t_adm = time.perf_counter()
            try:
                with torch.cuda.stream(stream):
                    ctx.bind_torch()
                    E = ctx.solve(req.tol, allow_noconv=True)
                    ctx.adjoint(req.tol, allow_noconv=True)
                    F = ctx.forces()
                st = ctx.stats()
                resid = (st["resid_primal"], st["resid_adjoint"])
                res = Result(req.rid, len(req.radii), E, F, t_sub, t_adm, time.perf_counter(), need,
                             (st["iters_primal"], st["iters_adjoint"]), resid, max(resid) <= req.tol)
                fut.set_result(res)
            except Exception as e:
                fut.set_exception(e)
            finally:
                ctx.close()
                with self._cv:
                    self.bytes_in_flight -= need
                    self.in_flight -= 1
                    self._cv.notify_all()


def run_arrivals(server: Server, requests, times):
    """Submit request k at time times[k] (s, from the start) and wait for all of
    them; returns (per request: its Result, or the exception that rejected it;
    makespan in s, from the start to the last completion)."""
    t0 = time.perf_counter()
    futs = []
    for req, t in zip(requests, times):
        delay = t0 + t - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        futs.append(server.submit(req))
    results = []
    for f in futs:
        try:
            results.append(f.result())
        except Exception as e:  # rejected (invalid request, over the HBM budget)
            results.append(e)
    done = [r for r in results if isinstance(r, Result)]
    return results, (max(r.t_done for r in done) - t0) if done else 0.0


def run_poisson(server: Server, requests, rate, seed=0):
    """run_arrivals with exponential inter-arrival times of mean 1/rate."""
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, size=len(requests))
    return run_arrivals(server, requests, np.cumsum(gaps))


def latency_summary(results, makespan, offered_atoms=None, arrival_span=None):
    """p50/p99 latency (submission to completion), the same of the time on the device
    (admission to completion) and the median queueing time, and the throughput of the
    served requests (entries of `results` that are exceptions count as rejected);
    offered load when the requested atoms and the arrival span are given."""
    ok = [r for r in results if isinstance(r, Result)]
    rejected = [(k, str(r)) for k, r in enumerate(results) if not isinstance(r, Result)]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    # time on the device (admission to completion) and time queued before admission
    svc = np.array([r.t_done - r.t_admit for r in ok]) if ok else np.zeros(1)
    wait = np.array([r.t_admit - r.t_submit for r in ok]) if ok else np.zeros(1)
    atoms = sum(r.atoms for r in ok)
    conv_atoms = sum(r.atoms for r in ok if r.converged)
    out = {"requests": len(results), "served": len(ok), "rejected": len(rejected),
           "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
           "service_p50_ms": float(np.percentile(svc, 50) * 1e3),
           "service_p99_ms": float(np.percentile(svc, 99) * 1e3),
           "queue_p50_ms": float(np.percentile(wait, 50) * 1e3),
           "atoms_per_s": atoms / makespan if makespan > 0 else 0.0,
           "converged_atoms_per_s": conv_atoms / makespan if makespan > 0 else 0.0,
           "makespan_s": makespan, "atoms": atoms,
           "not_converged": [r.rid for r in ok if not r.converged]}
    if rejected:
        out["rejections"] = sorted({msg for _, msg in rejected})[:8]
    if offered_atoms is not None and arrival_span:
        out["offered_atoms_per_s"] = offered_atoms / arrival_span
        out["arrival_span_s"] = arrival_span
    return out

"""Host logic of the continuous-batching server with a stand-in context (no GPU):
admission by workspace footprint, slot limit, arrival order and error paths."""
import contextlib
import threading
import time
import types

import numpy as np
import pytest

from paper_2203_00552_amd import serve


class FakeContext:
    live = 0
    peak = 0
    lock = threading.Lock()

    def __init__(self, centers, radii, charges, **kw):
        if len(radii) == 0:
            raise ValueError("empty")
        self.n = len(radii)
        self.kw = kw

    def workspace_bytes(self):
        return 100 * self.n

    def bind_torch(self):
        with FakeContext.lock:
            FakeContext.live += self.n
            FakeContext.peak = max(FakeContext.peak, FakeContext.live)

    def solve(self, tol, allow_noconv=False):
        time.sleep(0.01)
        return -float(self.n)

    def adjoint(self, tol, allow_noconv=False):
        pass

    def forces(self):
        return np.zeros((self.n, 3))

    def stats(self):
        return {"iters_primal": 1, "iters_adjoint": 1, "resid_primal": 0.0, "resid_adjoint": 0.0}

    def close(self):
        with FakeContext.lock:
            FakeContext.live -= self.n if hasattr(self, "n") else 0
        self.n = 0


def _server(monkeypatch, **kw):
    import torch
    monkeypatch.setattr(serve, "Context", FakeContext)
    monkeypatch.setattr(torch, "cuda", types.SimpleNamespace(
        Stream=lambda: None, stream=lambda s: contextlib.nullcontext(), mem_get_info=lambda: (10**9, 10**9)))
    return serve.Server(**kw)


def _req(n, rid):
    return serve.Request(np.zeros((n, 3)), np.ones(n), np.zeros(n), rid=rid)


def test_budget_limits_atoms_in_flight(monkeypatch):
    FakeContext.live = FakeContext.peak = 0
    s = _server(monkeypatch, slots=4, hbm_budget=100 * 250)
    futs = [s.submit(_req(100, k)) for k in range(8)]
    res = [f.result() for f in futs]
    s.close()
    assert [r.rid for r in res] == list(range(8))
    assert FakeContext.peak <= 250 and s.max_in_flight == 2
    assert all(r.energy == -100.0 for r in res)


def test_slots_limit_and_errors(monkeypatch):
    FakeContext.live = FakeContext.peak = 0
    s = _server(monkeypatch, slots=2, hbm_budget=10**9)
    ok = [s.submit(_req(10, k)) for k in range(5)]
    too_big = s.submit(_req(10**8, 99))
    bad = s.submit(_req(0, 98))
    assert all(f.result().energy == -10.0 for f in ok)
    with pytest.raises(Exception):
        too_big.result()
    with pytest.raises(ValueError):
        bad.result()
    s.close()
    assert s.max_in_flight <= 2 and s.bytes_in_flight == 0


def test_latency_summary():
    rs = [serve.Result(k, 10, 0.0, None, 0.0, 0.0, 0.01 * (k + 1), 0, (1, 1)) for k in range(100)]
    summ = serve.latency_summary(rs, 1.0)
    assert abs(summ["p50_ms"] - 505.0) < 1e-6 and summ["atoms_per_s"] == 1000.0


def test_latency_summary_splits_queue_and_service():
    # submitted at 0, admitted at 0.1 k, done 0.05 after admission
    rs = [serve.Result(k, 10, 0.0, None, 0.0, 0.1 * k, 0.1 * k + 0.05, 0, (1, 1)) for k in range(11)]
    summ = serve.latency_summary(rs, 2.0)
    assert abs(summ["service_p50_ms"] - 50.0) < 1e-9 and abs(summ["service_p99_ms"] - 50.0) < 1e-9
    assert abs(summ["queue_p50_ms"] - 500.0) < 1e-9 and abs(summ["p50_ms"] - 550.0) < 1e-9

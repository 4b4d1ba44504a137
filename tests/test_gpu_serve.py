"""Continuous batching (GPU): results are the same alone and in a mix of concurrent
requests of different sizes and discretisations, and requests overlap."""
import numpy as np
import pytest

from paper_2203_00552_amd import inputs
from paper_2203_00552_amd.serve import Request, Server, latency_summary, run_poisson

pytestmark = pytest.mark.gpu


def _requests(precision=0):
    spec = [(60, 6, 110), (900, 8, 302), (2500, 8, 302), (300, 6, 302), (1500, 6, 110), (120, 8, 146)]
    out = []
    for k, (n, lmax, nleb) in enumerate(spec):
        x, r, q = inputs.lattice_cluster(n, seed=100 + k)
        out.append(Request(x, r, q, lmax=lmax, n_lebedev=nleb, tol=1e-8, precision=precision, rid=k))
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_alone_equals_mix(precision):
    """FP64 and the mixed path (FP32 preconditioner sweeps): bitwise-deterministic
    kernels, so every result is the same alone and among concurrent requests."""
    reqs = _requests(precision)
    alone = []
    s1 = Server(slots=1)
    for rq in reqs:
        alone.append(s1.submit(rq).result())
    s1.close()
    s4 = Server(slots=4)
    futs = [s4.submit(rq) for rq in reqs]
    mix = [f.result() for f in futs]
    s4.close()
    assert s4.max_in_flight > 1
    for a, b in zip(alone, mix):
        assert a.rid == b.rid
        assert abs(a.energy - b.energy) <= 1e-12 * abs(a.energy)
        assert np.abs(a.forces - b.forces).max() <= 1e-12 * np.abs(a.forces).max()


def test_poisson_latency_summary():
    reqs = _requests()[:4]
    s = Server(slots=3)
    res, span = run_poisson(s, reqs, rate=200.0, seed=1)
    s.close()
    summ = latency_summary(res, span)
    assert summ["requests"] == 4 and summ["p99_ms"] >= summ["p50_ms"] > 0


def test_underresolved_grid_is_rejected():
    """lmax 8 on the 110-point grid (quadrature degree 17 < 2 lmax + 2) is rejected at
    setup (EINVAL) instead of stagnating in the solver; the other requests are served."""
    from paper_2203_00552_amd.serve import run_arrivals
    x, r, q = inputs.lattice_cluster(200, seed=5)
    reqs = [Request(x, r, q, lmax=8, n_lebedev=110, rid=0), Request(x, r, q, lmax=8, n_lebedev=302, rid=1)]
    s = Server(slots=2)
    res, span = run_arrivals(s, reqs, [0.0, 0.0])
    s.close()
    assert isinstance(res[0], Exception) and getattr(res[0], "code", None) == -1
    summ = latency_summary(res, span)
    assert summ["served"] == 1 and summ["rejected"] == 1 and not summ["not_converged"]

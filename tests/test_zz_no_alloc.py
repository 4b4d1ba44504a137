"""The allocation-free potential evaluation (ddlpb_eval_potentials_noalloc) against
the allocating entry point, through the C ABI: two calls in a row, the second with
fewer points, each compared value by value (same kernels: equal bits)."""
import numpy as np
import pytest

from paper_2203_00552_amd import Context, DDLPBError, inputs

pytestmark = pytest.mark.gpu


def _points(x, r, n, seed):
    rng = np.random.default_rng(seed)
    i = rng.integers(0, len(r), size=n)
    d = rng.normal(size=(n, 3))
    d *= (rng.uniform(0.0, 0.98, size=n) * r[i] / np.linalg.norm(d, axis=1))[:, None]
    return x[i] + d, i.astype(np.int32)


def test_noalloc_matches_allocating_entry_point():
    x, r, q = inputs.small_cluster(0)
    ctx = Context(x, r, q, lmax=6, n_lebedev=110)
    ctx.solve(1e-10)
    for n, seed, balls in ((3000, 1, True), (257, 2, False)):
        pts, sph = _points(x, r, n, seed)
        b = sph if balls else None
        ref = ctx.potentials(pts, b)
        got = ctx.potentials(pts, b, noalloc=True)
        for a, e in zip(got, ref):
            assert a.shape == e.shape
            assert np.array_equal(a, e), np.abs(a - e).max()
        assert np.isfinite(ref[0]).all() and np.abs(ref[0]).max() > 0


def test_noalloc_limit_and_errors():
    x, r, q = inputs.small_cluster(1)
    ctx = Context(x, r, q, lmax=4, n_lebedev=110)
    with pytest.raises(DDLPBError):  # before a solve: ESTATE
        ctx.potentials(x[:2], noalloc=True)
    ctx.solve(1e-8)
    big = np.zeros((65537, 3)) + x[0]
    with pytest.raises(DDLPBError) as e:
        ctx.potentials(big, noalloc=True)
    assert e.value.code == -1
    pr, pe, gr, ge = ctx.potentials(np.zeros((0, 3)), noalloc=True)
    assert pr.shape == (0,)

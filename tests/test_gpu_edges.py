"""Edge cases of the GPU path (through the C ABI): smallest and largest degrees and
grids, the smallest and largest FMM orders, one and two atoms with the FMM, and
charges all zero.  Direct-path results are checked against the oracle; FMM results
against the direct GPU path."""
import numpy as np
import pytest

import oracle
from paper_2203_00552_amd import Context, inputs

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _efq(ctx, tol):
    E = ctx.solve(tol)
    ctx.adjoint(tol)
    return E, ctx.forces(), ctx.charge_gradient()


@pytest.mark.parametrize("lmax,nleb", [(0, 6), (1, 14), (10, 974)])
def test_degree_and_grid_extremes_vs_oracle(lmax, nleb):
    x, r, q = inputs.lattice_cluster(20, seed=31)
    ctx = Context(x, r, q, lmax=lmax, n_lebedev=nleb)
    E, F, _ = _efq(ctx, 1e-11)
    ref = oracle.Problem(x, r, q, lmax=lmax, n_lebedev=nleb).solve("gmres", tol=1e-11)
    assert abs(E / ref["energy"] - 1) < 1e-8
    assert _rel(F, ref["forces"]) < 1e-8


@pytest.mark.parametrize("lmax,p", [(4, 5), (6, 16), (10, 16)])
def test_fmm_order_extremes_vs_direct(lmax, p):
    x, r, q = inputs.lattice_cluster(150, seed=32)
    d = _efq(Context(x, r, q, lmax=lmax, n_lebedev=302), 1e-10)
    f = _efq(Context(x, r, q, lmax=lmax, n_lebedev=302, fmm_order=p), 1e-10)
    tol = 1e-4 if p == lmax + 1 else 1e-6
    assert abs(f[0] / d[0] - 1) < tol
    assert _rel(f[1], d[1]) < 100 * tol
    assert _rel(f[2], d[2]) < 10 * tol


@pytest.mark.parametrize("n", [1, 2])
def test_fmm_one_and_two_atoms(n):
    x = np.array([[0.0, 0.0, 0.0], [3.1, 0.4, -0.2]])[:n]
    r = np.array([1.5, 1.7])[:n]
    q = np.array([0.7, -0.3])[:n]
    d = _efq(Context(x, r, q, lmax=6, n_lebedev=110), 1e-11)
    f = _efq(Context(x, r, q, lmax=6, n_lebedev=110, fmm_order=10), 1e-11)
    assert abs(f[0] / d[0] - 1) < 1e-9
    assert _rel(f[1], d[1]) < 1e-7 and _rel(f[2], d[2]) < 1e-8


def test_zero_charges():
    x, r, _ = inputs.lattice_cluster(30, seed=33)
    q = np.zeros(len(r))
    for p in (0, 10):
        E, F, g = _efq(Context(x, r, q, lmax=6, n_lebedev=110, fmm_order=p), 1e-8)
        assert E == 0.0 and np.all(F == 0.0) and np.all(g == 0.0)


def test_krylov_preconditioner_deeper_than_restart():
    """restart 10 with 32 inner GMRES steps on L_AB: the inner Gram-Schmidt uses more
    vectors than the outer basis; the solve must stay in its workspace and match the
    oracle."""
    x, r, q = inputs.small_cluster(4)
    ctx = Context(x, r, q, lmax=6, n_lebedev=110, options=dict(gmres_restart=10, precond_krylov=32))
    E, F, _ = _efq(ctx, 1e-11)
    ref = oracle.Problem(x, r, q, lmax=6, n_lebedev=110).solve("dense")
    assert abs(E / ref["energy"] - 1) < 1e-8
    assert _rel(F, ref["forces"]) < 1e-8


def test_option_after_bind_is_enomem():
    """A bound workspace fixes the layout: an option that needs more memory afterwards
    (precision 2 adds two vectors) makes the next solve fail with ENOMEM instead of
    writing past the caller's block."""
    from paper_2203_00552_amd import DDLPBError
    x, r, q = inputs.small_cluster(0)
    ctx = Context(x, r, q, lmax=4, n_lebedev=110, torch_workspace=True)
    before = ctx.workspace_bytes()
    ctx.set_option("precision", 2)
    assert ctx.workspace_bytes() > before
    with pytest.raises(DDLPBError) as e:
        ctx.solve(1e-8)
    assert e.value.code == -3

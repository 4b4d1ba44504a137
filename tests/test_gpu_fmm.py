"""Fast multipole path against the direct path and the oracle (GPU, through the C ABI).

The FMM only approximates the direct sums, so it is not expected to reproduce the
oracle to 1e-8; the bars here are the measured truncation errors at the tested
orders (relative to the largest entry), the exactness of the adjoint (the
transposed FMM is the exact transpose of the forward FMM), and monotone decrease
of the error with the order p."""
import numpy as np
import pytest

import oracle
from paper_2203_00552_amd import Context, inputs

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.fixture(scope="module")
def cluster():
    return inputs.lattice_cluster(300, seed=4)


def test_fmm_operator_matches_direct(cluster):
    x, r, q = cluster
    d = Context(x, r, q, lmax=6, n_lebedev=302, fmm_order=0)
    rng = np.random.default_rng(0)
    X = rng.normal(size=(2, len(r), 49)) * np.exp(-0.4 * np.repeat(np.arange(7), 2 * np.arange(7) + 1))
    Yd = d.apply(X)
    YdT = d.apply(X, transpose=True)
    errs = []
    for p in (8, 12):
        f = Context(x, r, q, lmax=6, n_lebedev=302, fmm_order=p)
        errs.append((_rel(f.apply(X), Yd), _rel(f.apply(X, transpose=True), YdT)))
    assert errs[-1][0] < 1e-6 and errs[-1][1] < 1e-6, errs
    assert errs[-1][0] < errs[0][0] and errs[-1][1] < errs[0][1], errs


def test_fmm_adjoint_is_exact_transpose(cluster):
    x, r, q = cluster
    f = Context(x, r, q, lmax=6, n_lebedev=302, fmm_order=10)
    rng = np.random.default_rng(1)
    X = rng.normal(size=(2, len(r), 49))
    Z = rng.normal(size=(2, len(r), 49))
    a = (f.apply(X) * Z).sum()
    b = (X * f.apply(Z, transpose=True)).sum()
    assert abs(a - b) < 1e-11 * abs(a)


def test_m2l_block_layouts_agree(cluster):
    """The multipole-to-local kernel gives the same result for every block layout
    (wavefronts per block, coefficient tables in LDS or global memory)."""
    x, r, q = cluster
    rng = np.random.default_rng(2)
    X = rng.normal(size=(2, len(r), 49))
    out = []
    for w in (1, 4, 16):
        f = Context(x, r, q, lmax=6, n_lebedev=302, fmm_order=10, options={"m2l_waves": w})
        out.append((f.apply(X), f.apply(X, transpose=True)))
    for a, b in out[1:]:
        assert _rel(a, out[0][0]) < 1e-13 and _rel(b, out[0][1]) < 1e-13


def test_m2l_generic_kernel_agrees(cluster):
    """The one-node-per-block M2L kernel built on the generic translation (the one
    the M2M and L2L passes use) and the wavefront M2L kernel give the same operator."""
    x, r, q = cluster
    rng = np.random.default_rng(5)
    X = rng.normal(size=(2, len(r), 49))
    out = []
    for w in (0, -1):
        f = Context(x, r, q, lmax=6, n_lebedev=302, fmm_order=10, options={"m2l_waves": w})
        out.append((f.apply(X), f.apply(X, transpose=True)))
        f.close()
    assert _rel(out[1][0], out[0][0]) < 1e-12 and _rel(out[1][1], out[0][1]) < 1e-12


def test_update_centers_rebuilds_tree():
    """A context moved to new centres (ddlpb_update_centers) with the FMM gives the
    energy and forces of a context created at those centres: the tree and its
    interaction lists follow the atoms."""
    x, r, q = inputs.lattice_cluster(1500, seed=10)
    x2 = x + 0.3 * np.random.default_rng(1).normal(size=x.shape)
    a = Context(x, r, q, lmax=6, n_lebedev=302, fmm_order=10)
    a.solve(1e-10)
    a.update_centers(x2)
    Ea = a.solve(1e-10)
    a.adjoint(1e-10)
    Fa = a.forces()
    b = Context(x2, r, q, lmax=6, n_lebedev=302, fmm_order=10)
    Eb = b.solve(1e-10)
    b.adjoint(1e-10)
    Fb = b.forces()
    assert abs(Ea / Eb - 1) < 1e-9
    assert _rel(Fa, Fb) < 1e-7
    a.close()
    b.close()


def test_fmm_error_decreases_with_order(cluster):
    """At a fixed acceptance parameter the far-field error falls with the expansion
    order (the local expansions are evaluated on the sphere grids to full degree p)."""
    x, r, q = cluster
    d = Context(x, r, q, lmax=6, n_lebedev=302, fmm_order=0)
    rng = np.random.default_rng(3)
    X = rng.normal(size=(2, len(r), 49)) * np.exp(-0.4 * np.repeat(np.arange(7), 2 * np.arange(7) + 1))
    Yd = d.apply(X)
    errs = []
    for p in (8, 11, 14):
        f = Context(x, r, q, lmax=6, n_lebedev=302, fmm_order=p, options={"theta": 0.7})
        errs.append(_rel(f.apply(X), Yd))
    assert errs[1] < 0.5 * errs[0] and errs[2] < 0.5 * errs[1], errs


def test_fmm_rhs_matches_direct(cluster):
    x, r, q = cluster
    d = Context(x, r, q, lmax=6, n_lebedev=302, fmm_order=0)
    f = Context(x, r, q, lmax=6, n_lebedev=302, fmm_order=12)
    assert _rel(f.rhs(), d.rhs()) < 1e-6


def test_fmm_energy_forces_vs_oracle():
    """Energy and forces with FMM p = 12 against the oracle (direct sums) on a 120-atom
    cluster: the FMM truncation error stays far below the discretisation error."""
    x, r, q = inputs.lattice_cluster(120, seed=5)
    ref = oracle.Problem(x, r, q, lmax=6, n_lebedev=302).solve("gmres", tol=1e-11)
    out = {}
    for p in (8, 12):
        f = Context(x, r, q, lmax=6, n_lebedev=302, fmm_order=p)
        E = f.solve(1e-11)
        f.adjoint(1e-11)
        F = f.forces()
        out[p] = (abs(E / ref["energy"] - 1), _rel(F, ref["forces"]))
    assert out[12][0] < 1e-7 and out[12][1] < 1e-5, out
    assert out[12][0] <= out[8][0] * 1.01 and out[12][1] <= out[8][1] * 1.01, out


def test_fmm_forces_match_direct_gpu():
    """FMM forces against the GPU direct path at 400 atoms, lmax 8 (p = 12)."""
    x, r, q = inputs.lattice_cluster(400, seed=6)
    d = Context(x, r, q, lmax=8, n_lebedev=302, fmm_order=0)
    Ed = d.solve(1e-10)
    d.adjoint(1e-10)
    Fd = d.forces()
    f = Context(x, r, q, lmax=8, n_lebedev=302, fmm_order=12)
    Ef = f.solve(1e-10)
    f.adjoint(1e-10)
    Ff = f.forces()
    assert abs(Ef / Ed - 1) < 1e-6
    assert _rel(Ff, Fd) < 1e-4


def test_fmm_charge_gradient():
    """dE/dq with the FMM (near list + transposed Laplace FMM) against the direct GPU
    path (itself checked against the oracle in test_gpu_parity), and Euler's identity
    sum q dE/dq = 2E at 2,000 atoms."""
    x, r, q = inputs.lattice_cluster(400, seed=5)
    out = []
    for p in (0, 12):
        f = Context(x, r, q, lmax=6, n_lebedev=302, fmm_order=p)
        f.solve(1e-11)
        f.adjoint(1e-11)
        out.append(f.charge_gradient())
    assert _rel(out[1], out[0]) < 1e-6
    x, r, q = inputs.lattice_cluster(2000, seed=6)
    f = Context(x, r, q, lmax=8, n_lebedev=302, fmm_order=12)
    E = f.solve(1e-10)
    f.adjoint(1e-10)
    g = f.charge_gradient()
    assert abs((q * g).sum() / (2 * E) - 1) < 1e-7


@pytest.mark.parametrize("n,lmax", [(300, 8), (1500, 6)])
def test_m2l_lane_kernel_agrees(n, lmax):
    """Order 12: the one-translation-per-lane multipole-to-local kernels (screened
    Coulomb in the operator and its transpose, Coulomb in the right-hand side and the
    forces) give the operator, its transpose, the energy and the forces of the
    wavefront kernel to rounding."""
    x, r, q = inputs.lattice_cluster(n, seed=7)
    L = (lmax + 1) ** 2
    rng = np.random.default_rng(3)
    X = rng.normal(size=(2, n, L))
    res = []
    for lane in (1, 0):
        f = Context(x, r, q, lmax=lmax, n_lebedev=302, fmm_order=12, options={"m2l_lane": lane})
        Y, YT = f.apply(X), f.apply(X, transpose=True)
        E = f.solve(1e-10)
        f.adjoint(1e-10)
        res.append((Y, YT, E, f.forces()))
    (Y1, YT1, E1, F1), (Y0, YT0, E0, F0) = res
    assert _rel(Y1, Y0) < 1e-12 and _rel(YT1, YT0) < 1e-12
    assert abs(E1 / E0 - 1) < 1e-10
    assert _rel(F1, F0) < 1e-8


@pytest.mark.parametrize("leaf", [2, 4])
def test_leaf_groups_match_direct(leaf):
    """Leaf groups of several spheres (near field sphere by sphere inside rejected pairs
    of groups) keep the FMM operator, its transpose and energy + forces at the accuracy
    of single-sphere leaves against direct sums."""
    x, r, q = inputs.lattice_cluster(700, seed=12)
    L = 49
    X = np.random.default_rng(8).normal(size=(2, 700, L))
    d = Context(x, r, q, lmax=6, n_lebedev=302, fmm_order=0)
    Yd, YTd = d.apply(X), d.apply(X, transpose=True)
    Ed = d.solve(1e-10)
    d.adjoint(1e-10)
    Fd = d.forces()
    f1 = Context(x, r, q, lmax=6, n_lebedev=302, fmm_order=12)
    fk = Context(x, r, q, lmax=6, n_lebedev=302, fmm_order=12, options={"leaf_size": leaf})
    assert fk.stats()["n_m2l"] < f1.stats()["n_m2l"] and fk.stats()["n_near_pairs"] > f1.stats()["n_near_pairs"]
    e1 = max(_rel(f1.apply(X), Yd), _rel(f1.apply(X, transpose=True), YTd))
    ek = max(_rel(fk.apply(X), Yd), _rel(fk.apply(X, transpose=True), YTd))
    assert ek < max(2 * e1, 1e-9), (ek, e1)
    E = fk.solve(1e-10)
    fk.adjoint(1e-10)
    assert abs(E / Ed - 1) < 1e-7
    assert _rel(fk.forces(), Fd) < 1e-5


@pytest.mark.parametrize("n,thresh", [(400, 1), (3000, 1), (3000, 200)])
def test_level_lane_kernels_agree(n, thresh):
    """Order 12, screened Coulomb: the one-node-per-lane multipole-to-multipole and
    local-to-local kernels (every level, or only the levels of at least `thresh` nodes)
    give the operator, its transpose, the energy and the forces of the wavefront
    kernels to rounding."""
    x, r, q = inputs.lattice_cluster(n, seed=21)
    L = 49
    X = np.random.default_rng(4).normal(size=(2, n, L))
    res = []
    for lvl in (thresh, 0):
        f = Context(x, r, q, lmax=6, n_lebedev=302, fmm_order=12, options={"level_lane": lvl, "kernel_timing": 1})
        Y, YT = f.apply(X), f.apply(X, transpose=True)
        E = f.solve(1e-10)
        f.adjoint(1e-10)
        res.append((Y, YT, E, f.forces()))
        assert ("level_lane" in f.kernel_times()) == (lvl > 0)
        f.close()
    (Y1, YT1, E1, F1), (Y0, YT0, E0, F0) = res
    assert _rel(Y1, Y0) < 1e-12 and _rel(YT1, YT0) < 1e-12, (_rel(Y1, Y0), _rel(YT1, YT0))
    assert abs(E1 / E0 - 1) < 1e-10
    assert _rel(F1, F0) < 1e-8

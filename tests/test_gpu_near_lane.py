"""Near-field A/B kernels with one neighbour cap per lane (GPU): the operator, its
transpose, the energy and the forces agree with the cap-list kernels they replace, on
the fly and with the incore cache of harmonics, in FP64 and in FP32, also with
solvent-accessible radii (many more caps and neighbours per sphere)."""
import numpy as np
import pytest

from paper_2203_00552_amd import inputs
from paper_2203_00552_amd._lib import Context

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _ctx(x, r, q, lmax, nleb, fmm, **opts):
    o = {"kernel_timing": 1}
    o.update(opts)
    return Context(x, r, q, lmax=lmax, n_lebedev=nleb, fmm_order=fmm, options=o)


@pytest.mark.parametrize("n,lmax,nleb,fmm,sas", [(60, 2, 110, 0, False), (60, 6, 146, 0, False),
                                                   (200, 8, 302, 0, False), (700, 8, 302, 10, False),
                                                   (150, 6, 302, 0, True)])
def test_lane_operator_agrees(n, lmax, nleb, fmm, sas):
    """L X and L^T X of the lane kernels (on the fly and incore) equal the cap-list
    kernels' to rounding; FP32 lane kernels within FP32 accuracy."""
    x, r, q = inputs.lattice_cluster(n, seed=11)
    if sas:
        r = r + 1.4
    L = (lmax + 1) ** 2
    X = np.random.default_rng(5).normal(size=(2, n, L))
    out = {}
    for key, opts in {"cap": {"near_lane": 0}, "lane": {}, "incore": {"near_incore": 1}}.items():
        f = _ctx(x, r, q, lmax, nleb, fmm, **opts)
        Y, YT = f.apply(X), f.apply(X, transpose=True)
        f.set_option("apply_fp32", 1)
        Y32, YT32 = f.apply(X), f.apply(X, transpose=True)
        names = set(f.kernel_times())
        f.close()
        out[key] = (Y, YT, Y32, YT32, names)
    Yc, YTc, Yc32, YTc32, nc = out["cap"]
    assert "near_ltz" not in nc and "apply_LTZ" in nc
    for key in ("lane", "incore"):
        Y, YT, Y32, YT32, names = out[key]
        assert {"near_lx", "near_ltz", "near_lx_f32", "near_ltz_f32"} <= names, names
        assert _rel(Y, Yc) < 1e-12 and _rel(YT, YTc) < 1e-12, (key, _rel(Y, Yc), _rel(YT, YTc))
        assert _rel(Y32, Yc) < 2e-5 and _rel(YT32, YTc) < 2e-5, (key, _rel(Y32, Yc), _rel(YT32, YTc))
        assert _rel(Y32, Yc32) < 2e-5 and _rel(YT32, YTc32) < 2e-5


def test_lane_solve_and_forces_agree():
    """Energy, adjoint and forces through the lane kernels equal the cap-list path's."""
    x, r, q = inputs.lattice_cluster(400, seed=3)
    res = []
    for opts in ({"near_lane": 0}, {}, {"near_incore": 1}):
        f = _ctx(x, r, q, 8, 302, 12, **opts)
        E = f.solve(1e-10)
        f.adjoint(1e-10)
        res.append((E, f.forces()))
        f.close()
    (E0, F0) = res[0]
    for E, F in res[1:]:
        assert abs(E / E0 - 1) < 1e-10
        assert _rel(F, F0) < 1e-8


def test_lane_after_center_update_and_high_degree_fallback():
    """A centre update rebuilds the lane structures (and the incore cache); lmax 9 has no
    lane kernels and runs the cap-list kernels whatever the option says."""
    x, r, q = inputs.lattice_cluster(120, seed=4)
    x2 = inputs.perturbed(x, seed=9, sigma=0.2)
    L = 81
    X = np.random.default_rng(2).normal(size=(2, 120, L))
    ref = _ctx(x2, r, q, 8, 302, 0, near_lane=0)
    Yr, YTr = ref.apply(X), ref.apply(X, transpose=True)
    ref.close()
    for opts in ({}, {"near_incore": 1}):
        f = _ctx(x, r, q, 8, 302, 0, **opts)
        f.apply(X)
        f.update_centers(x2)
        assert _rel(f.apply(X), Yr) < 1e-12 and _rel(f.apply(X, transpose=True), YTr) < 1e-12
        f.close()
    X9 = np.random.default_rng(2).normal(size=(2, 120, 100))
    a = _ctx(x, r, q, 9, 302, 0)
    b = _ctx(x, r, q, 9, 302, 0, near_lane=0)
    Ya, Yb = a.apply(X9, transpose=True), b.apply(X9, transpose=True)
    assert "near_ltz" not in set(a.kernel_times())
    assert np.array_equal(Ya, Yb)
    a.close()
    b.close()

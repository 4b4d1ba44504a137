"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
symbol declared in include/ddlpb.h, and validates arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2203_00552_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "ddlpb.h")).read()
    return sorted(set(re.findall(r"\b(ddlpb_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_symbols()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTS)


def _setup(**kw):
    args = dict(M=2, x=np.array([[0, 0, 0], [1.0, 0, 0]]), r=np.array([1.5, 1.5]), q=np.array([0.5, -0.5]),
                e1=1.0, e2=78.54, kap=0.104, lmax=4, nleb=110, p=0)
    args.update(kw)
    lib = _lib.load()
    h = ctypes.c_void_p()
    rc = lib.ddlpb_setup(args["M"], _lib.ptr(np.ascontiguousarray(args["x"], dtype=np.float64)),
                         _lib.ptr(np.ascontiguousarray(args["r"], dtype=np.float64)),
                         _lib.ptr(np.ascontiguousarray(args["q"], dtype=np.float64)),
                         args["e1"], args["e2"], args["kap"], args["lmax"], args["nleb"], args["p"], ctypes.byref(h))
    if rc == 0:
        lib.ddlpb_free(h)
    return rc


@pytest.mark.parametrize("kw,code", [
    (dict(), 0),
    (dict(r=np.array([1.5, -1.0])), -1),
    (dict(x=np.array([[0, 0, 0], [np.nan, 0, 0]])), -1),
    (dict(e2=0.0), -1),
    (dict(kap=0.0), -1),
    (dict(lmax=11), -1),
    (dict(nleb=111), -1),
    (dict(lmax=9, nleb=110), -1),   # degree 17 < 2 lmax
    (dict(lmax=8, nleb=110), -1),   # degree 17 < 2 lmax + 2
    (dict(lmax=7, nleb=110), 0),    # degree 17 = 2 lmax + 2
    (dict(lmax=8, nleb=146), 0),
    (dict(x=np.array([[0, 0, 0], [0, 0, 0]])), -2),
    (dict(M=0), -1),
])
def test_setup_validation(kw, code):
    assert _setup(**kw) == code


def test_call_order_and_options():
    lib = _lib.load()
    h = ctypes.c_void_p()
    x = np.array([[0.0, 0, 0], [1.0, 0, 0]])
    r = np.array([1.5, 1.5])
    q = np.array([0.5, -0.5])
    assert lib.ddlpb_setup(2, _lib.ptr(x), _lib.ptr(r), _lib.ptr(q), 1.0, 78.54, 0.104, 4, 110, 0, ctypes.byref(h)) == 0
    F = np.zeros((2, 3))
    assert lib.ddlpb_adjoint(h, 1e-8) == -6
    assert lib.ddlpb_forces(h, _lib.ptr(F)) == -6
    assert lib.ddlpb_set_option(h, b"eta", 0.2) == 0
    assert lib.ddlpb_set_option(h, b"eta", 1.5) == -1
    assert lib.ddlpb_set_option(h, b"nonsense", 1.0) == -1
    assert lib.ddlpb_workspace_bytes(h) > 0
    assert lib.ddlpb_strerror(-5) == b"solver did not converge"
    lib.ddlpb_free(h)
    lib.ddlpb_free(None)


def test_workspace_grows_with_krylov_preconditioner_depth():
    """The dot-product scratch and the inner basis are sized for the deepest Krylov
    space (outer restart, inner preconditioner steps or DIIS history), not the
    restart alone."""
    lib = _lib.load()
    x = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 1.2, 0]])
    r = np.array([1.5, 1.5, 1.4])
    q = np.array([0.5, -0.5, 0.0])
    sizes = {}
    for k in (16, 32, 64):
        h = ctypes.c_void_p()
        assert lib.ddlpb_setup(3, _lib.ptr(x), _lib.ptr(r), _lib.ptr(q), 1.0, 78.54, 0.104, 4, 110, 0,
                               ctypes.byref(h)) == 0
        assert lib.ddlpb_set_option(h, b"gmres_restart", 10) == 0
        assert lib.ddlpb_set_option(h, b"precond_krylov", k) == 0
        sizes[k] = lib.ddlpb_workspace_bytes(h)
        lib.ddlpb_free(h)
    D = 2 * 3 * 25  # 2 M L doubles per vector
    for a, b in ((16, 32), (32, 64)):
        # (b - a) more inner basis vectors and (b - a) more rows of 1024 partial dot products
        assert sizes[b] - sizes[a] >= (b - a) * (D * 8 + 1024 * 8) - 2 * 256


def test_precision_and_kernel_options_are_validated():
    """The mixed-precision and kernel-choice options accept exactly their documented
    values (host-side checks, no device needed)."""
    lib = _lib.load()
    h = ctypes.c_void_p()
    x = np.array([[0.0, 0, 0], [1.0, 0, 0]])
    r = np.array([1.5, 1.5])
    q = np.array([0.5, -0.5])
    assert lib.ddlpb_setup(2, _lib.ptr(x), _lib.ptr(r), _lib.ptr(q), 1.0, 78.54, 0.104, 4, 110, 0, ctypes.byref(h)) == 0
    for key in (b"mixed_m2l", b"mixed_forces", b"mixed_near_sl", b"mixed_levels", b"cap_lists", b"inner_reorth"):
        assert lib.ddlpb_set_option(h, key, 0) == 0, key
        assert lib.ddlpb_set_option(h, key, 1) == 0, key
        assert lib.ddlpb_set_option(h, key, 2) == -1, key
        assert lib.ddlpb_set_option(h, key, 0.5) == -1, key
    for v in (0, 1, 2, 3):
        assert lib.ddlpb_set_option(h, b"apply_fp32", v) == 0
    assert lib.ddlpb_set_option(h, b"apply_fp32", 4) == -1
    assert lib.ddlpb_set_option(h, b"apply_fp32", -1) == -1
    lib.ddlpb_free(h)

"""ctypes binding of libddlpb.so (argument marshalling only; all numerics run in
the library's HIP kernels).  Importing this module does not touch the GPU; the
library is loaded on first use and its absence is an error, never a fallback."""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddlpb.so")

ERRORS = {0: "ok", -1: "EINVAL", -2: "EGEOM", -3: "ENOMEM", -4: "EDEVICE", -5: "ENOCONV", -6: "ESTATE"}

# every symbol declared in include/ddlpb.h
EXPORTS = ["ddlpb_setup", "ddlpb_solve", "ddlpb_adjoint", "ddlpb_forces", "ddlpb_free", "ddlpb_set_option",
           "ddlpb_update_centers", "ddlpb_workspace_bytes", "ddlpb_bind_workspace", "ddlpb_set_stream",
           "ddlpb_get_stats", "ddlpb_strerror", "ddlpb_get_grid", "ddlpb_get_solution", "ddlpb_get_rhs",
           "ddlpb_apply", "ddlpb_kernel_times", "ddlpb_kernel_times_reset", "ddlpb_charge_gradient",
           "ddlpb_eval_potentials", "ddlpb_eval_potentials_noalloc",
           "ddlpb_dielectric_gradient", "ddlpb_radius_gradient"]


class DDLPBError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {ERRORS.get(code, code)}")


class Stats(ctypes.Structure):
    _fields_ = [("iters_primal", ctypes.c_int32), ("iters_adjoint", ctypes.c_int32),
                ("resid_primal", ctypes.c_double), ("resid_adjoint", ctypes.c_double),
                ("ms_setup", ctypes.c_double), ("ms_rhs", ctypes.c_double), ("ms_primal", ctypes.c_double),
                ("ms_adjoint", ctypes.c_double), ("ms_forces", ctypes.c_double),
                ("n_cap_pairs", ctypes.c_int64), ("n_active_points", ctypes.c_int64),
                ("n_near_pairs", ctypes.c_int64), ("n_m2l", ctypes.c_int64), ("fmm_order", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("refinements", ctypes.c_int32),
                ("fmm_order_below_lmax", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2203_00552_amd.build.build()")
        # torch ships its own HIP runtime under the same soname as the system one: load it
        # first, so that the library binds to it and the process holds one runtime (torch
        # cannot initialise the device after another runtime has)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        c_void_p, c_int, c_double, c_size_t = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
        lib.ddlpb_setup.argtypes = [c_int, _dp, _dp, _dp, c_double, c_double, c_double, c_int, c_int, c_int,
                                    ctypes.POINTER(c_void_p)]
        lib.ddlpb_solve.argtypes = [c_void_p, c_double, _dp]
        lib.ddlpb_adjoint.argtypes = [c_void_p, c_double]
        lib.ddlpb_forces.argtypes = [c_void_p, _dp]
        lib.ddlpb_charge_gradient.argtypes = [c_void_p, _dp]
        lib.ddlpb_dielectric_gradient.argtypes = [c_void_p, _dp]
        lib.ddlpb_radius_gradient.argtypes = [c_void_p, _dp]
        lib.ddlpb_eval_potentials.argtypes = [c_void_p, c_int, _dp, ctypes.POINTER(ctypes.c_int32), _dp]
        lib.ddlpb_eval_potentials_noalloc.argtypes = [c_void_p, c_int, _dp, ctypes.POINTER(ctypes.c_int32), _dp]
        lib.ddlpb_free.argtypes = [c_void_p]
        lib.ddlpb_free.restype = None
        lib.ddlpb_set_option.argtypes = [c_void_p, ctypes.c_char_p, c_double]
        lib.ddlpb_update_centers.argtypes = [c_void_p, _dp]
        lib.ddlpb_workspace_bytes.argtypes = [c_void_p]
        lib.ddlpb_workspace_bytes.restype = c_size_t
        lib.ddlpb_bind_workspace.argtypes = [c_void_p, c_void_p, c_size_t]
        lib.ddlpb_set_stream.argtypes = [c_void_p, c_void_p]
        lib.ddlpb_get_stats.argtypes = [c_void_p, ctypes.POINTER(Stats)]
        lib.ddlpb_strerror.argtypes = [c_int]
        lib.ddlpb_strerror.restype = ctypes.c_char_p
        lib.ddlpb_get_grid.argtypes = [c_void_p, _dp, _dp]
        lib.ddlpb_get_solution.argtypes = [c_void_p, _dp, _dp]
        lib.ddlpb_get_rhs.argtypes = [c_void_p, _dp]
        lib.ddlpb_apply.argtypes = [c_void_p, c_int, _dp, _dp]
        lib.ddlpb_kernel_times.argtypes = [c_void_p, c_int, ctypes.c_char_p, _dp, ctypes.POINTER(ctypes.c_int64), _dp]
        lib.ddlpb_kernel_times_reset.argtypes = [c_void_p]
        _lib = lib
    return _lib


def ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def check(rc, where):
    if rc != 0:
        raise DDLPBError(rc, where)


class Context:
    """One ddLPB problem on the current GPU (wraps a ddlpb_ctx*).

    If ``torch_workspace`` is true, the device memory is a torch uint8 tensor
    bound to the context and work runs on torch's current stream."""

    def __init__(self, centers, radii, charges, eps_in=1.0, eps_out=78.54, kappa=0.104, lmax=6, n_lebedev=110,
                 fmm_order=0, eta=None, precision=None, options=None, torch_workspace=False):
        lib = load()
        self.x = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
        self.r = np.ascontiguousarray(radii, dtype=np.float64).ravel()
        self.q = np.ascontiguousarray(charges, dtype=np.float64).ravel()
        self.M = self.x.shape[0]
        self.lmax, self.N = int(lmax), int(n_lebedev)
        self.L = (self.lmax + 1) ** 2
        h = ctypes.c_void_p()
        check(lib.ddlpb_setup(self.M, ptr(self.x), ptr(self.r), ptr(self.q), float(eps_in), float(eps_out),
                              float(kappa), self.lmax, self.N, int(fmm_order), ctypes.byref(h)), "ddlpb_setup")
        self._h = h
        self._ws = None
        opts = dict(options or {})
        if eta is not None:
            opts["eta"] = eta
        if precision is not None:
            opts["precision"] = precision
        for k, v in opts.items():
            check(lib.ddlpb_set_option(self._h, k.encode(), float(v)), f"set_option({k})")
        if torch_workspace:
            self.bind_torch()

    def bind_torch(self):
        import torch
        nbytes = int(load().ddlpb_workspace_bytes(self._h))
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        addr = self._ws.data_ptr()
        addr = (addr + 255) & ~255
        check(load().ddlpb_bind_workspace(self._h, ctypes.c_void_p(addr), nbytes), "bind_workspace")
        stream = torch.cuda.current_stream().cuda_stream
        check(load().ddlpb_set_stream(self._h, ctypes.c_void_p(stream)), "set_stream")

    def use_current_stream(self):
        """Enqueue the context's work on torch's current stream (the context keeps its
        own device workspace, which it may enlarge when the geometry changes)."""
        import torch
        check(load().ddlpb_set_stream(self._h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
              "set_stream")

    def set_option(self, key, value):
        check(load().ddlpb_set_option(self._h, key.encode(), float(value)), f"set_option({key})")

    def workspace_bytes(self):
        return int(load().ddlpb_workspace_bytes(self._h))

    def solve(self, tol=1e-8, allow_noconv=False):
        e = ctypes.c_double()
        rc = load().ddlpb_solve(self._h, float(tol), ctypes.byref(e))
        if rc != 0 and not (allow_noconv and rc == -5):
            check(rc, "ddlpb_solve")
        return e.value

    def adjoint(self, tol=1e-8, allow_noconv=False):
        rc = load().ddlpb_adjoint(self._h, float(tol))
        if rc != 0 and not (allow_noconv and rc == -5):
            check(rc, "ddlpb_adjoint")

    def forces(self):
        F = np.zeros((self.M, 3))
        check(load().ddlpb_forces(self._h, ptr(F)), "ddlpb_forces")
        return F

    def charge_gradient(self):
        """dE/dq_k [M] from the adjoint solution (needs a prior adjoint)."""
        g = np.zeros(self.M)
        check(load().ddlpb_charge_gradient(self._h, ptr(g)), "ddlpb_charge_gradient")
        return g

    def potentials(self, points, spheres=None, noalloc=False):
        """psi_r, psi_e [n] and their gradients [n, 3] at the points [n, 3] from the
        expansions of the given balls (default: the ball with the smallest
        |x - x_i| / r_i); needs a prior solve.  noalloc: the entry point that stages
        in the library's fixed device array (at most 65536 points, no allocation)."""
        p = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
        n = p.shape[0]
        b = None
        if spheres is not None:
            b = np.ascontiguousarray(spheres, dtype=np.int32).ravel()
            if b.size != n:
                raise ValueError("one ball index per point")
        out = np.zeros((n, 8))
        fn = load().ddlpb_eval_potentials_noalloc if noalloc else load().ddlpb_eval_potentials
        check(fn(self._h, n, ptr(p), None if b is None else b.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                 ptr(out)), "ddlpb_eval_potentials" + ("_noalloc" if noalloc else ""))
        return out[:, 0].copy(), out[:, 1].copy(), out[:, 2:5].copy(), out[:, 5:8].copy()

    def dielectric_gradient(self):
        """(dE/d eps_in, dE/d eps_out) from the adjoint solution; needs a prior adjoint."""
        out = np.zeros(2)
        check(load().ddlpb_dielectric_gradient(self._h, ptr(out)), "ddlpb_dielectric_gradient")
        return out

    def radius_gradient(self):
        """dE/dr_j [M] from the adjoint solution (needs a prior adjoint)."""
        g = np.zeros(self.M)
        check(load().ddlpb_radius_gradient(self._h, ptr(g)), "ddlpb_radius_gradient")
        return g

    def update_centers(self, centers):
        x = np.ascontiguousarray(centers, dtype=np.float64).reshape(self.M, 3)
        check(load().ddlpb_update_centers(self._h, ptr(x)), "ddlpb_update_centers")
        self.x = x

    def stats(self):
        s = Stats()
        check(load().ddlpb_get_stats(self._h, ctypes.byref(s)), "ddlpb_get_stats")
        return s.as_dict()

    def kernel_times(self):
        """{kernel name: (ms, launches, algorithmic flops)} (needs the option kernel_timing=1)."""
        out = {}
        k = 0
        name = ctypes.create_string_buffer(64)
        ms, work = ctypes.c_double(), ctypes.c_double()
        nl = ctypes.c_int64()
        while load().ddlpb_kernel_times(self._h, k, name, ctypes.byref(ms), ctypes.byref(nl), ctypes.byref(work)) == 0:
            out[name.value.decode()] = (ms.value, nl.value, work.value)
            k += 1
        return out

    def kernel_times_reset(self):
        check(load().ddlpb_kernel_times_reset(self._h), "ddlpb_kernel_times_reset")

    def grid(self):
        f = np.zeros((self.M, self.N))
        U = np.zeros((self.M, self.N))
        check(load().ddlpb_get_grid(self._h, ptr(f), ptr(U)), "ddlpb_get_grid")
        return f, U

    def solution(self, adjoint=True):
        X = np.zeros((2, self.M, self.L))
        Xa = np.zeros((2, self.M, self.L)) if adjoint else None
        check(load().ddlpb_get_solution(self._h, ptr(X), ptr(Xa)), "ddlpb_get_solution")
        return X, Xa

    def rhs(self):
        g = np.zeros((2, self.M, self.L))
        check(load().ddlpb_get_rhs(self._h, ptr(g)), "ddlpb_get_rhs")
        return g

    def apply(self, X, transpose=False):
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(2, self.M, self.L)
        Y = np.zeros_like(X)
        check(load().ddlpb_apply(self._h, 1 if transpose else 0, ptr(X), ptr(Y)), "ddlpb_apply")
        return Y

    def close(self):
        if getattr(self, "_h", None):
            load().ddlpb_free(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

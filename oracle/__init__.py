"""ddLPB oracle -- TEST INFRASTRUCTURE ONLY.

ctypes front-end of ``libddlpb_oracle.so`` (built from ``ddlpb_oracle.cpp`` by
``oracle.build()``): a plain FP64 CPU implementation of the discrete ddLPB
energy, adjoint solve and analytical forces with direct O(M^2) summation.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP product
path; the Lebedev rule it uses comes straight from SciPy's ``lebedev_rule``
(a library primitive), independent of the table compiled into the product.

Functions with no independent pin are marked "parity unpinned" in their
docstring; every other function is pinned by a test in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ddlpb_oracle.cpp")
_LIB = os.path.join(_HERE, "libddlpb_oracle.so")

# Lebedev rules by point count -> quadrature degree (SciPy's lebedev_rule orders)
LEBEDEV_DEGREE = {6: 3, 14: 5, 26: 7, 38: 9, 50: 11, 74: 13, 86: 15, 110: 17, 146: 19,
                  170: 21, 194: 23, 230: 25, 266: 27, 302: 29, 350: 31, 434: 35,
                  590: 41, 770: 47, 974: 53}


def build(verbose: bool = False) -> str:
    """Compile the oracle shared library with g++ (FP64, OpenMP)."""
    tmp = f"{_LIB}.{os.getpid()}.tmp"
    cmd = ["g++", "-O2", "-fopenmp", "-std=c++17", "-shared", "-fPIC", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(tmp, _LIB)  # a process that has the old library loaded keeps its copy
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB)
    return _lib


def lebedev(n_points: int):
    """Lebedev points s_n [N,3] and weights w_n [N] with sum w = 4 pi (SciPy)."""
    from scipy.integrate import lebedev_rule
    x, w = lebedev_rule(LEBEDEV_DEGREE[n_points])
    s = np.ascontiguousarray(x.T, dtype=np.float64)
    assert s.shape[0] == n_points
    return s, np.ascontiguousarray(w, dtype=np.float64)


_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def _ptr(a):
    return a.ctypes.data_as(_dp)


class Problem:
    """Inputs of one ddLPB evaluation (FP64 copies owned by this object)."""

    def __init__(self, centers, radii, charges, eps_in=1.0, eps_out=78.54, kappa=0.104,
                 lmax=6, n_lebedev=110, eta=0.05, s=None, w=None):
        self.x = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
        self.r = np.ascontiguousarray(radii, dtype=np.float64).ravel()
        self.q = np.ascontiguousarray(charges, dtype=np.float64).ravel()
        self.M = self.x.shape[0]
        self.eps1, self.eps2, self.kappa, self.eta = float(eps_in), float(eps_out), float(kappa), float(eta)
        self.lmax = int(lmax)
        self.L = (self.lmax + 1) ** 2
        if s is None:
            s, w = lebedev(n_lebedev)
        self.s = np.ascontiguousarray(s, dtype=np.float64)
        self.w = np.ascontiguousarray(w, dtype=np.float64)
        self.N = self.s.shape[0]

    def _args(self):
        return (ctypes.c_int(self.M), _ptr(self.x), _ptr(self.r), _ptr(self.q),
                ctypes.c_double(self.eps1), ctypes.c_double(self.eps2), ctypes.c_double(self.kappa),
                ctypes.c_double(self.eta), ctypes.c_int(self.lmax), ctypes.c_int(self.N),
                _ptr(self.s), _ptr(self.w))

    # ---------------------------------------------------------------- pieces
    def sphere_constants(self):
        """C_l^j (Sec. 2.2, C1/C2 definition) and i_l'(r_j)/i_l(r_j) (d/dr), each [M, lmax+1]."""
        out = np.zeros((2, self.M, self.lmax + 1))
        _load().oracle_sphere_constants(*self._args(), _ptr(out))
        return out[0], out[1]

    def grid_fields(self):
        """f^i and chi^eta_i at every grid point x_i^n (Sec. 3.1), each [M, N]; neighbour counts [M]."""
        f = np.zeros((self.M, self.N))
        U = np.zeros((self.M, self.N))
        nn = np.zeros(self.M, dtype=np.int32)
        _load().oracle_grid_fields(*self._args(), _ptr(f), _ptr(U), nn.ctypes.data_as(_ip))
        return f, U, nn

    def rhs(self):
        """g = (G0 + F0, F0) (Sec. 2.2), [2, M, L]."""
        g = np.zeros((2, self.M, self.L))
        _load().oracle_rhs(*self._args(), _ptr(g))
        return g

    def apply(self, X, transpose=False, part="L"):
        """L X or L^T X (matrix-free, Sec. 2.2 and the adjoint system of Sec. 3);
        part "AB" applies only [A 0; 0 B], part "C" only [C1 C2; C1 C2] (Sec. 4 splitting)."""
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(2, self.M, self.L)
        Y = np.zeros_like(X)
        _load().oracle_apply(*self._args(), ctypes.c_int(1 if transpose else 0),
                             ctypes.c_int({"L": 0, "AB": 1, "C": 2}[part]), _ptr(X), _ptr(Y))
        return Y

    def dense(self):
        """Literal assembly of L [(2ML)^2] and g [2ML] from the matrix definitions."""
        D = 2 * self.M * self.L
        Lm = np.zeros((D, D))
        g = np.zeros(D)
        _load().oracle_dense(*self._args(), _ptr(Lm), _ptr(g))
        return Lm, g

    # ---------------------------------------------------------------- solve
    def solve(self, method="auto", tol=1e-12, restart=200, maxit=2000, forces=True):
        """Energy, X, X_adj and forces F = -grad E (e^2/A units).

        method "dense" = LU of the literal matrix; "gmres" = matrix-free GMRES;
        "fgmres" = matrix-free flexible GMRES preconditioned by inner GMRES solves of
        L_AB (the paper's preconditioner, Sec. 4), for the larger cases.
        """
        if method == "auto":
            method = "dense" if 2 * self.M * self.L <= 4000 else "gmres"
        D = 2 * self.M * self.L
        X = np.zeros(D)
        Xa = np.zeros(D)
        F = np.zeros((self.M, 3))
        E = ctypes.c_double(0.0)
        info = np.zeros(2, dtype=np.int32)
        code = {"dense": 0, "gmres": 1, "fgmres": 2}[method]
        rc = _load().oracle_solve(*self._args(), ctypes.c_int(code),
                                  ctypes.c_double(tol), ctypes.c_int(restart), ctypes.c_int(maxit),
                                  ctypes.byref(E), _ptr(X), _ptr(Xa), _ptr(F) if forces else None,
                                  info.ctypes.data_as(_ip))
        if rc != 0:
            raise RuntimeError(f"oracle solve failed (rc={rc})")
        return dict(energy=E.value, X=X.reshape(2, self.M, self.L), Xadj=Xa.reshape(2, self.M, self.L),
                    forces=F if forces else None, iters=tuple(int(v) for v in info))

    def single_layer_field(self, m):
        """Phi[m] at every grid point with chi^eta > 0 (zero elsewhere), [M, N], for
        per-sphere coefficients m [M, L] (Sec. 2.2, the single-layer potential with
        basis k_l(kappa |x - x_j|) / k_l(kappa r_j) Y_lm of every sphere j)."""
        m = np.ascontiguousarray(m, dtype=np.float64).reshape(self.M, self.L)
        out = np.zeros((self.M, self.N))
        _load().oracle_single_layer_field(*self._args(), _ptr(m), _ptr(out))
        return out

    def forces_from(self, X, Xadj):
        """Forces from given X and X_adj (Sec. 3 force equation)."""
        X = np.ascontiguousarray(X, dtype=np.float64)
        Xa = np.ascontiguousarray(Xadj, dtype=np.float64)
        F = np.zeros((self.M, 3))
        _load().oracle_forces_from(*self._args(), _ptr(X), _ptr(Xa), _ptr(F))
        return F

    def potentials(self, X, points, spheres=None, h=1e-4):
        """Reaction and extended potentials at points from the expansions of a ball
        (Sec. 2, the representation of psi_r and psi_e once X is known):
            psi_r(x) = sum_lm X_r,ilm (|x - x_i| / r_i)^l Y_lm(x - x_i),
            psi_e(x) = sum_lm X_e,ilm i_l(kappa |x - x_i|) / i_l(kappa r_i) Y_lm(x - x_i),
        written out term by term; the gradients are central differences of the same
        sums with step h r_i.  spheres None: the ball with the smallest |x - x_i| / r_i.
        Returns psi_r [n], psi_e [n], grad psi_r [n, 3], grad psi_e [n, 3]."""
        X = np.asarray(X, dtype=np.float64).reshape(2, self.M, self.L)
        pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
        if spheres is None:
            d2 = ((pts[:, None, :] - self.x[None, :, :]) ** 2).sum(-1) / self.r[None, :] ** 2
            spheres = d2.argmin(axis=1)
        lmax = self.lmax
        deg = np.repeat(np.arange(lmax + 1), 2 * np.arange(lmax + 1) + 1)

        def values(x, i):
            v = x - self.x[i]
            d = float(np.sqrt(v @ v))
            ir = bessel(lmax, self.kappa * self.r[i])[0]
            if d == 0.0:  # only l = 0 survives: Y_00 = 1 / sqrt(4 pi), i_0(0) = 1
                y00 = 1.0 / np.sqrt(4.0 * np.pi)
                return X[0, i, 0] * y00, X[1, i, 0] * y00 / ir[0]
            Y = sph_harm(lmax, v)[0]
            rad_r = (d / self.r[i]) ** deg
            rad_e = (bessel(lmax, self.kappa * d)[0] / ir)[deg]
            return float((X[0, i] * rad_r * Y).sum()), float((X[1, i] * rad_e * Y).sum())

        n = pts.shape[0]
        pr, pe = np.zeros(n), np.zeros(n)
        gr, ge = np.zeros((n, 3)), np.zeros((n, 3))
        for k in range(n):
            i = int(spheres[k])
            pr[k], pe[k] = values(pts[k], i)
            step = h * self.r[i]
            for c in range(3):
                e = np.zeros(3)
                e[c] = step
                a = values(pts[k] + e, i)
                b = values(pts[k] - e, i)
                gr[k, c] = (a[0] - b[0]) / (2 * step)
                ge[k, c] = (a[1] - b[1]) / (2 * step)
        return pr, pe, gr, ge

    def charge_gradient(self, method="auto", tol=1e-12):
        """dE/dq_k for every atom.  E is a quadratic form in the charges (g and Q are
        linear in q, Sec. 2.2 and 3), so the central difference with unit step,
        (E(q + e_k) - E(q - e_k)) / 2, is its derivative exactly (up to rounding)."""
        out = np.zeros(self.M)
        q0 = self.q.copy()
        try:
            for k in range(self.M):
                e = []
                for sgn in (1.0, -1.0):
                    self.q = q0.copy()
                    self.q[k] += sgn
                    e.append(self.solve(method, tol=tol, forces=False)["energy"])
                out[k] = 0.5 * (e[0] - e[1])
        finally:
            self.q = q0
        return out

    def dielectric_gradient(self, method="auto", tol=1e-12, h=1e-3):
        """(dE/d eps_in, dE/d eps_out) by Richardson-extrapolated central differences of
        the energy of the solved discrete problem (relative step h, error O(h^4)).  The
        energy is a smooth function of the permittivities: they enter g through psi_0 and
        the normal-derivative term and L through the ratio eps_in/eps_out (Sec. 2.2)."""
        out = np.zeros(2)
        e0 = (self.eps1, self.eps2)
        try:
            for k in range(2):
                E = {}
                for s in (-2, -1, 1, 2):
                    eps = list(e0)
                    eps[k] = e0[k] * (1.0 + s * h)
                    self.eps1, self.eps2 = eps
                    E[s] = self.solve(method, tol=tol, forces=False)["energy"]
                step = e0[k] * h
                out[k] = (8.0 * (E[1] - E[-1]) - (E[2] - E[-2])) / (12.0 * step)
        finally:
            self.eps1, self.eps2 = e0
        return out

    def energy_complex_step(self, atom, coord, h=1e-30):
        """dE/dx_{atom,coord} by the complex step Im E(x + i h e)/h (dense path);
        coord 3 gives dE/dr_atom (the radius with every radial constant of Sec. 2.2 that
        depends on it: r^-l, i_l(kappa r), k_l(kappa r), i_l'/i_l, C_l)."""
        d = ctypes.c_double(0.0)
        rc = _load().oracle_energy_cs(*self._args(), ctypes.c_int(atom), ctypes.c_int(coord),
                                      ctypes.c_double(h), ctypes.byref(d))
        if rc != 0:
            raise RuntimeError("complex-step solve failed")
        return d.value


    def radius_gradient(self, atoms=None, h=1e-30):
        """dE/dr_j for the listed atoms (all by default) by complex steps of the dense
        solve (Sec. 3: the energy as a function of any parameter of the model)."""
        atoms = range(self.M) if atoms is None else atoms
        return np.array([self.energy_complex_step(a, 3, h) for a in atoms])


# ------------------------------------------------------------ table routines
def sph_harm(lmax, v):
    """Real orthonormal Y_lm(v/|v|), [n, (lmax+1)^2], index l*l+l+m."""
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((v.shape[0], (lmax + 1) ** 2))
    _load().oracle_sph_harm(ctypes.c_int(lmax), ctypes.c_int(v.shape[0]), _ptr(v), _ptr(out))
    return out


def bessel(lmax, z):
    """(i_l, k_l, i_l', k_l') at z for l = 0..lmax, each [lmax+1]."""
    out = np.zeros((4, lmax + 1))
    _load().oracle_bessel(ctypes.c_int(lmax), ctypes.c_double(z), _ptr(out))
    return out


def switch(eta, t):
    """(chi_eta(t), chi_eta'(t)) (Sec. 3.1 regularised characteristic function)."""
    t = np.ascontiguousarray(t, dtype=np.float64).ravel()
    out = np.zeros((2, t.size))
    _load().oracle_switch(ctypes.c_double(eta), ctypes.c_int(t.size), _ptr(t), _ptr(out))
    return out[0], out[1]

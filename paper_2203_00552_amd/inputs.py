"""Seeded synthetic workloads (no ddLPB arithmetic lives here).

These generators stand in for the paper's PDB structures, which are not
available: they draw atom centres, radii and charges with the shapes, sizes and
distributions of the benchmark configurations.  Both the tests' oracle runs and
the HIP path receive the same arrays from here.

* ``small_cluster``: 12 (or n) centres uniform in a cube with a minimum pair
  distance (rejection sampling), radii U[1.4, 2.0] x 1.1, charges U[-0.5, 0.5]
  shifted to sum zero.
* ``lattice_cluster``: cubic lattice (2.2 A) with uniform +-0.4 A jitter, the
  n points nearest the origin kept (a ball), radii from {1.2, 1.5, 1.7, 1.8} A
  with probabilities {0.5, 0.2, 0.2, 0.1}, charges N(0, 0.3) minus their mean.
"""
from __future__ import annotations

import numpy as np


def small_cluster(seed: int = 0, n: int = 12, box: float = 6.0, min_sep: float = 1.0):
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        p = rng.uniform(0.0, box, size=3)
        if all(np.linalg.norm(p - o) >= min_sep for o in pts):
            pts.append(p)
    x = np.array(pts)
    r = rng.uniform(1.4, 2.0, size=n) * 1.1
    q = rng.uniform(-0.5, 0.5, size=n)
    q -= q.mean()
    return x, r, q


def lattice_cluster(n: int, seed: int = 0, spacing: float = 2.2, jitter: float = 0.4):
    rng = np.random.default_rng(seed)
    side = int(np.ceil((n * 6.0 / np.pi) ** (1.0 / 3.0))) + 3
    g = (np.arange(side) - (side - 1) / 2.0) * spacing
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    pts = pts + rng.uniform(-jitter, jitter, size=pts.shape)
    order = np.argsort(np.einsum("ij,ij->i", pts, pts), kind="stable")
    x = np.ascontiguousarray(pts[order[:n]])
    r = rng.choice(np.array([1.2, 1.5, 1.7, 1.8]), size=n, p=[0.5, 0.2, 0.2, 0.1])
    q = rng.normal(0.0, 0.3, size=n)
    q -= q.mean()
    return x, r, q


def perturbed(x, seed: int, sigma: float = 0.05):
    """Gaussian displacement of every coordinate (conformation batches)."""
    rng = np.random.default_rng(seed)
    return x + rng.normal(0.0, sigma, size=x.shape)


def serving_requests(n_requests: int = 512, rate: float = 200.0, seed: int = 0,
                     n_min: int = 50, n_max: int = 20000):
    """Poisson arrival times and per-request (atom count, lmax, N_leb, seed)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps)
    sizes = np.exp(rng.uniform(np.log(n_min), np.log(n_max), size=n_requests)).astype(int)
    lmax = rng.choice([6, 8], size=n_requests)
    nleb = rng.choice([110, 302], size=n_requests)
    seeds = rng.integers(0, 2**31 - 1, size=n_requests)
    return [dict(t=float(t[k]), n=int(sizes[k]), lmax=int(lmax[k]), n_lebedev=int(nleb[k]),
                 seed=int(seeds[k])) for k in range(n_requests)]

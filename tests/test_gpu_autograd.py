"""ddLPB energy as a torch.autograd.Function (GPU, through the C ABI): the backward
(adjoint solve + force assembly) against the oracle forces and against central
finite differences of the energy, and a batch of perturbed conformations against
independent contexts."""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_00552_amd import Context, inputs
from paper_2203_00552_amd.autograd import DDLPBEnergy

pytestmark = pytest.mark.gpu


def test_backward_is_minus_oracle_forces():
    x, r, q = inputs.small_cluster(0)
    model = DDLPBEnergy(r, q, tol=1e-11, lmax=6, n_lebedev=110)
    X = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    E = model(X)
    E.backward()
    ref = oracle.Problem(x, r, q, lmax=6, n_lebedev=110).solve("dense")
    assert abs(E.item() / ref["energy"] - 1) < 1e-8
    F = ref["forces"]
    assert np.abs(X.grad.numpy() + F).max() < 1e-8 * np.abs(F).max()
    model.close()


def test_backward_matches_central_differences_config4():
    """Central differences (h = 1e-4 A) of the FP64 direct-sum energy of the 2,000-atom
    cluster (lattice generator, seed 0; lmax 8, 302 points) on 20 atoms chosen with
    seed 1 x 3 coordinates, against the backward pass.  A coordinate whose +-h
    perturbation moves a grid point across f = 1 (where U has a kink, so the energy is
    only piecewise C^1) is skipped and counted; the solves are warm-started."""
    x, r, q = inputs.lattice_cluster(2000, seed=0)
    model = DDLPBEnergy(r, q, tol=1e-12, lmax=8, n_lebedev=302)
    X = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    model(X).backward()
    g = X.grad.numpy()
    atoms = np.random.default_rng(1).choice(len(r), 20, replace=False)
    h = 1e-4
    err, skipped = 0.0, 0
    with torch.no_grad():
        for a in atoms:
            for c in range(3):
                E, side = [], []
                for sgn in (1.0, -1.0):
                    xs = x.copy()
                    xs[a, c] += sgn * h
                    E.append(model(torch.tensor(xs)).item())
                    side.append(model._slots[0].ctx.grid()[0] > 1.0)
                if np.any(side[0] != side[1]):
                    skipped += 1
                    continue
                err = max(err, abs((E[0] - E[1]) / (2 * h) - g[a, c]))
    print(f"config 4 finite differences: max error {err / np.abs(g).max():.2e} of max|grad|, "
          f"{skipped} of 60 coordinates skipped at f = 1")
    assert skipped <= 10
    assert err < 2e-5 * np.abs(g).max(), err
    model.close()


def test_batch_of_perturbed_conformations():
    """16 conformations of a 2,000-atom cluster (Gaussian displacements 0.05 A), FMM
    p = 12: energies and gradients equal those of independent contexts."""
    x, r, q = inputs.lattice_cluster(2000, seed=10)
    rng = np.random.default_rng(12)
    B = 16
    xs = x[None] + 0.05 * rng.normal(size=(B,) + x.shape)
    kw = dict(lmax=8, n_lebedev=302, fmm_order=12)
    model = DDLPBEnergy(r, q, tol=1e-8, **kw)
    X = torch.tensor(xs, requires_grad=True)
    E = model(X)
    E.sum().backward()
    for b in (0, 7, 15):
        c = Context(xs[b], r, q, **kw)
        Eb = c.solve(1e-8)
        c.adjoint(1e-8)
        Fb = c.forces()
        assert abs(E[b].item() / Eb - 1) < 1e-12
        assert np.abs(X.grad[b].numpy() + Fb).max() < 1e-10 * np.abs(Fb).max()
        c.close()
    model.close()

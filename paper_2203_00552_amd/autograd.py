"""ddLPB energy as a torch.autograd.Function.

Forward: solve L X = g for the given atom centres and return the solvation energy
E (Sec. 3 energy equation).  Backward: the adjoint solve L^T X_adj = Q followed by
the analytical force assembly (Sec. 3, force equation); the gradient with respect
to the centres is -F times the incoming gradient.  Both passes run in the HIP
library; this module only moves centres and forces between torch and the context.

One context per conformation slot keeps the geometry-dependent state (grids,
lists, the tree) and the solutions resident on the device, so a batch of
conformations differentiates without re-solving; a slot whose state was replaced
by a later forward is re-solved before its backward.
"""
from __future__ import annotations

import numpy as np
import torch

from ._lib import Context


class _Slot:
    def __init__(self, make):
        self.make = make
        self.ctx = None
        self.generation = 0
        self.x = None

    def solve(self, x, tol):
        if self.ctx is None:
            self.ctx = self.make(x)
        else:
            self.ctx.update_centers(x)
        self.generation += 1
        self.x = x
        return self.ctx.solve(tol)


class _EnergyFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, centers, slot, tol):
        x = centers.detach().to("cpu", torch.float64).contiguous().numpy()
        E = slot.solve(x, tol)
        ctx.slot, ctx.tol, ctx.generation = slot, tol, slot.generation
        ctx.x = x
        ctx.meta = (centers.dtype, centers.device)
        return torch.tensor(E, dtype=centers.dtype, device=centers.device)

    @staticmethod
    def backward(ctx, gE):
        slot = ctx.slot
        if slot.generation != ctx.generation or not np.array_equal(slot.x, ctx.x):
            slot.solve(ctx.x, ctx.tol)  # the slot was reused by a later forward
        slot.ctx.adjoint(ctx.tol)
        F = torch.from_numpy(slot.ctx.forces())
        dtype, device = ctx.meta
        grad = (-F).to(device=device, dtype=dtype) * gE
        return grad, None, None


class DDLPBEnergy(torch.nn.Module):
    """E(centres) for fixed radii, charges and model parameters.

    ``forward`` takes centres [M, 3] (returns a scalar) or a batch [B, M, 3]
    (returns [B]); gradients flow to the centres.  Keyword arguments are those of
    ``Context`` (eps_in, eps_out, kappa, lmax, n_lebedev, fmm_order, precision,
    options)."""

    def __init__(self, radii, charges, tol=1e-8, **context_kw):
        super().__init__()
        self.radii = np.ascontiguousarray(radii, dtype=np.float64).ravel()
        self.charges = np.ascontiguousarray(charges, dtype=np.float64).ravel()
        self.tol = float(tol)
        self.context_kw = dict(context_kw)
        self._slots = []

    def _slot(self, b):
        while len(self._slots) <= b:
            self._slots.append(_Slot(lambda x: Context(x, self.radii, self.charges, **self.context_kw)))
        return self._slots[b]

    def forward(self, centers):
        if centers.dim() == 2:
            return _EnergyFn.apply(centers, self._slot(0), self.tol)
        if centers.dim() != 3:
            raise ValueError("centres must be [M, 3] or [B, M, 3]")
        return torch.stack([_EnergyFn.apply(centers[b], self._slot(b), self.tol) for b in range(centers.shape[0])])

    def close(self):
        for s in self._slots:
            if s.ctx is not None:
                s.ctx.close()
        self._slots = []

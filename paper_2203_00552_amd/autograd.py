"""ddLPB energy as a torch.autograd.Function.

Forward: solve L X = g for the given atom centres and return the solvation energy
E (Sec. 3 energy equation).  Backward: the adjoint solve L^T X_adj = Q followed by
the analytical force assembly (Sec. 3, force equation); the gradient with respect
to the centres is -F times the incoming gradient.  Both passes run in the HIP
library; this module only moves centres and forces between torch and the context.

One context per conformation slot keeps the geometry-dependent state (grids,
lists, the tree) and the solutions resident on the device, so a batch of
conformations differentiates without re-solving; a slot whose state was replaced
by a later forward is re-solved before its backward.  The slots of a batch work
concurrently: each has its own HIP stream and device workspace, and one host
thread per slot waits on its own solves, so the kernels of different
conformations overlap on the device.
"""
from __future__ import annotations

import contextlib
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from ._lib import Context


class _Slot:
    def __init__(self, make):
        self.make = make
        self.ctx = None
        self.stream = None
        self.generation = 0
        self.x = None

    def _on_stream(self):
        if self.stream is None and torch.cuda.is_available():
            self.stream = torch.cuda.Stream()
        return torch.cuda.stream(self.stream) if self.stream is not None else contextlib.nullcontext()

    def solve(self, x, tol):
        with self._on_stream():  # the context's workspace and work live on this stream
            if self.ctx is None:
                self.ctx = self.make(x)
            else:
                self.ctx.update_centers(x)
            self.generation += 1
            self.x = x
            return self.ctx.solve(tol)

    def gradient(self, x, tol, generation):
        if self.generation != generation or not np.array_equal(self.x, x):
            self.solve(x, tol)  # the slot was reused by a later forward
        with self._on_stream():
            self.ctx.adjoint(tol)
            return self.ctx.forces()


def _each(fn, n):
    """fn(b) for b < n, one host thread per slot (each waits on its own stream)."""
    if n == 1:
        return [fn(0)]
    with ThreadPoolExecutor(max_workers=min(n, 16)) as ex:
        return list(ex.map(fn, range(n)))


class _EnergyFn(torch.autograd.Function):
    """E for a batch of conformations [B, M, 3] -> [B], one slot per conformation."""

    @staticmethod
    def forward(ctx, centers, slots, tol):
        xs = centers.detach().to("cpu", torch.float64).contiguous().numpy()
        E = _each(lambda b: slots[b].solve(xs[b], tol), len(slots))
        ctx.slots, ctx.tol, ctx.xs = slots, tol, xs
        ctx.generations = [s.generation for s in slots]
        ctx.meta = (centers.dtype, centers.device)
        return torch.tensor(E, dtype=centers.dtype, device=centers.device)

    @staticmethod
    def backward(ctx, gE):
        F = _each(lambda b: ctx.slots[b].gradient(ctx.xs[b], ctx.tol, ctx.generations[b]), len(ctx.slots))
        dtype, device = ctx.meta
        grad = -torch.from_numpy(np.stack(F)).to(device=device, dtype=dtype) * gE.reshape(-1, 1, 1)
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
            self._slots.append(_Slot(lambda x: self._make(x)))
        return self._slots[b]

    def _make(self, x):
        # the work runs on the slot's stream (current when the slot creates its context);
        # the context owns its workspace, which update_centers may enlarge
        c = Context(x, self.radii, self.charges, **self.context_kw)
        c.use_current_stream()
        return c

    def forward(self, centers):
        if centers.dim() == 2:
            return _EnergyFn.apply(centers[None], [self._slot(0)], self.tol)[0]
        if centers.dim() != 3:
            raise ValueError("centres must be [M, 3] or [B, M, 3]")
        return _EnergyFn.apply(centers, [self._slot(b) for b in range(centers.shape[0])], self.tol)

    def close(self):
        for s in self._slots:
            if s.ctx is not None:
                s.ctx.close()
        self._slots = []

"""Host logic of the autograd wrapper, with a stand-in context (no GPU): gradients
are -F times the incoming gradient, batches map to slots, and a slot reused by a
later forward is re-solved before its backward."""
import numpy as np
import torch

from paper_2203_00552_amd import autograd as ag


class FakeContext:
    """E = sum |x - a|^2, F = -2 (x - a); counts solves."""

    def __init__(self, x, a):
        self.a = a
        self.x = np.array(x)
        self.solves = 0
        self.adjoint_x = None

    def update_centers(self, x):
        self.x = np.array(x)

    def solve(self, tol):
        self.solves += 1
        return float(((self.x - self.a) ** 2).sum())

    def adjoint(self, tol):
        self.adjoint_x = self.x.copy()

    def forces(self):
        return -2.0 * (self.adjoint_x - self.a)

    def close(self):
        pass


def _model(a):
    m = ag.DDLPBEnergy(np.ones(3), np.zeros(3))
    made = []

    def slot(b):
        while len(m._slots) <= b:
            s = ag._Slot(lambda x: made.append(FakeContext(x, a)) or made[-1])
            m._slots.append(s)
        return m._slots[b]

    m._slot = slot
    return m, made


def test_gradient_and_batch():
    a = np.arange(9.0).reshape(3, 3) * 0.1
    m, made = _model(a)
    xs = torch.tensor(np.random.default_rng(0).normal(size=(4, 3, 3)), requires_grad=True)
    E = m(xs)
    (E * torch.arange(1.0, 5.0, dtype=torch.float64)).sum().backward()
    for b in range(4):
        np.testing.assert_allclose(xs.grad[b].numpy(), (b + 1) * 2.0 * (xs[b].detach().numpy() - a))
    assert len(made) == 4


def test_stale_slot_is_resolved():
    a = np.zeros((3, 3))
    m, made = _model(a)
    x1 = torch.tensor(np.ones((3, 3)), requires_grad=True)
    x2 = torch.tensor(2 * np.ones((3, 3)), requires_grad=True)
    E1 = m(x1)
    E2 = m(x2)  # same slot: overwrites the state of the first forward
    E1.backward()
    np.testing.assert_allclose(x1.grad.numpy(), 2.0 * np.ones((3, 3)))
    assert made[0].solves == 3
    E2.backward()
    np.testing.assert_allclose(x2.grad.numpy(), 4.0 * np.ones((3, 3)))

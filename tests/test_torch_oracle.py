"""The PyTorch (autograd) oracle of one step, pinned to the C oracle and to
finite differences of itself.  CPU only."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle.torch_step import TorchStep
from tests.helpers import normwise, random_state


def grid(dim):
    return oracle.Grid(dim=dim, nx=5, ny=4, nz=3 if dim == 3 else 1, dx=1.1, dy=0.9, dz=1.2, dt=0.45)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("nonrel", [False, True])
def test_torch_step_matches_the_c_oracle(dim, nonrel):
    g = grid(dim)
    g.nonrel = nonrel
    rng = np.random.default_rng(7 + dim)
    x, u, w, sp, E, B = random_state(g, 150, rng, umax=1.5, bmax=2.0, emax=0.5)
    ref = oracle.step(g, x, u, w, sp, E, B)
    ts = TorchStep(g)
    t = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64))
    x1, u1, E1, B1, Eth = ts.step(t(x), t(u), t(w), sp, t(E), t(B))
    assert normwise(Eth.numpy(), ref["E_theta"]) < 1e-12
    assert normwise(E1.numpy(), ref["E"]) < 1e-12
    assert normwise(B1.numpy(), ref["B"]) < 1e-12
    assert normwise(u1.numpy(), ref["u"]) < 1e-12
    d = x1.numpy() - ref["x"]
    L = np.array(g.L)[:, None]
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-12


def test_torch_gradient_matches_finite_differences():
    """d F / d eps for F = field energy after 2 steps, B0 = B + eps b."""
    g = grid(2)
    rng = np.random.default_rng(3)
    x, u, w, sp, E, B = random_state(g, 120, rng, umax=1.0, bmax=1.0, emax=0.2)
    bdir = rng.standard_normal((3, g.N))
    ts = TorchStep(g)
    t = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64))

    def F(eps):
        xx, uu, EE, BB = t(x), t(u), t(E), t(B) + eps * t(bdir)
        for _ in range(2):
            xx, uu, EE, BB, _ = ts.step(xx, uu, t(w), sp, EE, BB)
        return ts.field_energy(EE, BB)

    eps = torch.tensor(0.0, dtype=torch.float64, requires_grad=True)
    val = F(eps)
    (grad,) = torch.autograd.grad(val, eps)
    h = 1e-6
    with torch.no_grad():
        fd = (F(torch.tensor(h, dtype=torch.float64)) - F(torch.tensor(-h, dtype=torch.float64))) / (2 * h)
    assert abs(grad.item() - fd.item()) <= 1e-6 * abs(fd.item())


def test_torch_gradient_wrt_particles_matches_finite_differences():
    g = grid(2)
    rng = np.random.default_rng(4)
    x, u, w, sp, E, B = random_state(g, 60, rng, umax=1.0, bmax=1.0, emax=0.2)
    ts = TorchStep(g)
    t = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64))
    du = rng.standard_normal((3, x.shape[1]))
    dx = rng.standard_normal((2, x.shape[1]))

    def F(s):
        xx, uu = t(x) + s * t(dx), t(u) + s * t(du)
        EE, BB = t(E), t(B)
        xx, uu, EE, BB, _ = ts.step(xx, uu, t(w), sp, EE, BB)
        return ts.field_energy(EE, BB) + (uu * uu).sum()

    s = torch.tensor(0.0, dtype=torch.float64, requires_grad=True)
    (grad,) = torch.autograd.grad(F(s), s)
    h = 1e-7
    with torch.no_grad():
        fd = (F(torch.tensor(h, dtype=torch.float64)) - F(torch.tensor(-h, dtype=torch.float64))) / (2 * h)
    assert abs(grad.item() - fd.item()) <= 1e-5 * abs(fd.item())

"""BHEnergy (torch.autograd.Function) against the oracle: gradients of E and of a loss that mixes H and E,
for position, moment and external field."""
import numpy as np
import pytest
import torch

from paper_1212_2934_amd import workloads
from paper_1212_2934_amd.autograd import bh_energy
from paper_1212_2934_amd.binding import BarnesHut

from gpu_util import grad_check

pytestmark = pytest.mark.gpu


def _t(a, grad=True):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda().requires_grad_(grad)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32_mixed", 1e-5)])
def test_energy_gradient_through_autograd(oracle_mod, precision, tol):
    w = workloads.uniform_cube(3000, 30.0, seed=17, hext=(0.2, 0.0, 0.8))
    bh = BarnesHut(w.n, 1, 16, 0.5, precision)
    pos, mom, hext = _t(w.pos), _t(w.mom), _t(w.hext)
    H, E = bh_energy(pos, mom, hext, bh)
    E.sum().backward()
    _, Eref, dr, dm = oracle_mod.Tree(w.pos, w.mom, 16).energy_grad(0.5, w.hext)
    assert abs(E.item() - Eref) <= tol * np.abs(w.mom * H.detach().cpu().numpy()).sum()
    grad_check(pos.grad.cpu().numpy(), dr, precision, "autograd dE/dr")
    grad_check(mom.grad.cpu().numpy(), dm, precision, "autograd dE/dm")
    np.testing.assert_allclose(hext.grad.cpu().numpy(), -w.mom.sum(axis=1), rtol=1e-12)


def test_mixed_loss_vjp(oracle_mod):
    w = workloads.config3(seed=23, n=4000)
    bh = BarnesHut(w.n, 1, 16, 0.6, "fp64")
    pos, mom, hext = _t(w.pos), _t(w.mom), _t(np.zeros(3))
    wts = torch.from_numpy(np.random.default_rng(3).standard_normal((3, w.n))).cuda()
    H, E = bh_energy(pos, mom, hext, bh)
    loss = (wts * H).sum() + 2.0 * E.sum()
    loss.backward()
    t = oracle_mod.Tree(w.pos, w.mom, 16)
    Href, _, _ = t.field(0.6)
    dr, dm = t.vjp(0.6, wts.cpu().numpy() - 0.5 * 2.0 * w.mom)
    dm = dm + 2.0 * (-0.5 * Href)
    grad_check(pos.grad.cpu().numpy(), dr, "fp64", "autograd mixed loss dL/dr")
    grad_check(mom.grad.cpu().numpy(), dm, "fp64", "autograd mixed loss dL/dm")

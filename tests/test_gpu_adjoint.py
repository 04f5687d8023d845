"""Adjoint through the C ABI against the oracle's frozen-structure adjoint (whose pins are FD, theta = 0
== the all-pairs analytic gradient built from the paper's f_dip, and the invariants).

E = -1/2 sum m.H - sum m.H_ext; dE/dr, dE/dm and a general vector-Jacobian product with upstream dL/dH.
FP64 path: relative L2 within 1e-12 and every particle within 1e-10 (FP64 atomics only reorder sums);
FP32-mixed: relative L2 and the 99.9th percentile of the per-particle error within 1e-5.
"""
import numpy as np
import pytest
import torch

from paper_1212_2934_amd import workloads
from paper_1212_2934_amd.binding import BarnesHut

from gpu_util import grad_check

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-12, "fp32_mixed": 1e-5}


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _gpu_grad(pos, mom, hext, theta, precision, gH=None, gE=1.0, leaf=16, want_dhext=False, tuning_id=-1):
    bh = BarnesHut(pos.shape[-1], 1 if pos.ndim == 2 else pos.shape[0], leaf, theta, precision,
                   tuning_id=tuning_id)
    p = torch.from_numpy(pos).cuda()
    m = torch.from_numpy(mom).cuda()
    he = torch.from_numpy(np.asarray(hext, float)).cuda()
    g = None if gH is None else torch.from_numpy(gH).cuda()
    ge = None if gE is None else torch.full((bh.batch,), gE, dtype=torch.float64, device="cuda")
    bh.build(p)
    out = bh.field_backward(m, he, gH=g, gE=ge, want_dhext=want_dhext)
    assert bh.check_status() == 0
    return [None if o is None else o.cpu().numpy() for o in out]


# 64, 32 and 16 targets per wave; each walk split over the root's children, with 64, 32 and 16 targets per
# wave; one persistent cost-ordered launch with 2, 4 and 1 waves per workgroup; one wave per item in the
# cost order with 1, 2 and 4 waves per workgroup
@pytest.mark.parametrize("tuning_id", [0, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14])
@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_energy_gradient_config1(oracle_mod, precision, tuning_id):
    w = workloads.uniform_cube(4096, 32.0, seed=1001, hext=(0.0, 0.0, 1.0))
    H, E, dr, dm = oracle_mod.Tree(w.pos, w.mom, 16).energy_grad(0.5, w.hext)
    gdr, gdm, gdh = _gpu_grad(w.pos, w.mom, w.hext, 0.5, precision, want_dhext=True, tuning_id=tuning_id)
    grad_check(gdr, dr, precision, f"dE/dr uniform 4096 tuning {tuning_id}")
    grad_check(gdm, dm, precision, f"dE/dm uniform 4096 tuning {tuning_id}")
    np.testing.assert_allclose(gdh[0], -w.mom.sum(axis=1), rtol=1e-12)


@pytest.mark.parametrize("tuning_id", [0, 2, 5, 7, 10])
@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("theta", [0.3, 0.7])
def test_general_vjp_chains(oracle_mod, precision, theta, tuning_id):
    w = workloads.config3(seed=11, n=5000 + 3)
    rng = np.random.default_rng(12)
    gH = rng.standard_normal((3, w.n))
    gE = 0.3
    hext = np.array([0.2, -0.1, 0.05])
    t = oracle_mod.Tree(w.pos, w.mom, 16)
    H, _, _ = t.field(theta)
    dr, dm = t.vjp(theta, gH - 0.5 * gE * w.mom)
    dm = dm + gE * (-0.5 * H - hext[:, None])
    gdr, gdm = _gpu_grad(w.pos, w.mom, hext, theta, precision, gH=gH, gE=gE, tuning_id=tuning_id)
    grad_check(gdr, dr, precision, f"dL/dr chains theta {theta} tuning {tuning_id}")
    grad_check(gdm, dm, precision, f"dL/dm chains theta {theta} tuning {tuning_id}")


def test_theta_zero_equals_allpairs_force(oracle_mod):
    w = workloads.uniform_cube(1500, 20.0, seed=21)
    g = oracle_mod.allpairs_grad_r(w.pos, w.mom)
    gdr, gdm = _gpu_grad(w.pos, w.mom, np.zeros(3), 0.0, "fp64")
    assert rel(gdr, g) <= 1e-12
    assert rel(gdm, -oracle_mod.allpairs_field(w.pos, w.mom)) <= 1e-12


@pytest.mark.parametrize("tuning_id", [0, 3, 5, 6, 8, 9])
def test_batched_adjoint(oracle_mod, tuning_id):
    B, n = 3, 2000 + 77  # ragged: the last workgroup of each system is partly empty
    ws = [workloads.uniform_cube(n, 26.0, seed=30 + b) for b in range(B)]
    pos = np.stack([x.pos for x in ws])
    mom = np.stack([x.mom for x in ws])
    hext = np.array([0.0, 0.0, 0.7])
    gdr, gdm = _gpu_grad(pos, mom, hext, 0.5, "fp32_mixed", tuning_id=tuning_id)
    for b, x in enumerate(ws):
        _, _, dr, dm = oracle_mod.Tree(x.pos, x.mom, 16).energy_grad(0.5, hext)
        grad_check(gdr[b], dr, "fp32_mixed", f"dE/dr batch {b} tuning {tuning_id}")
        grad_check(gdm[b], dm, "fp32_mixed", f"dE/dm batch {b} tuning {tuning_id}")


@pytest.mark.parametrize("n", [1, 2, 3, 16, 17, 65, 300])
@pytest.mark.parametrize("tuning_id", [0, 6])
def test_small_systems(oracle_mod, n, tuning_id):
    """Down to a single particle and a root that is a leaf (n <= 16), where a split walk has one part."""
    w = workloads.uniform_cube(n, 4.0 + n ** (1.0 / 3.0) * 2.0, seed=60 + n, hext=(0.3, 0.0, 0.5))
    H, E, dr, dm = oracle_mod.Tree(w.pos, w.mom, 16).energy_grad(0.5, w.hext)
    gdr, gdm = _gpu_grad(w.pos, w.mom, w.hext, 0.5, "fp64", tuning_id=tuning_id)
    if n == 1:
        assert np.abs(gdr).max() == 0.0
        np.testing.assert_allclose(gdm, dm, rtol=1e-14)
        return
    grad_check(gdr, dr, "fp64", f"dE/dr n {n}")
    grad_check(gdm, dm, "fp64", f"dE/dm n {n}")


@pytest.mark.parametrize("tuning_id", [9, 11, 12, 14])
@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_persistent_launch_repeats(oracle_mod, precision, tuning_id):
    """The cost-ordered launches (persistent: 9, 11; one wave per item: 12, 14) order their items by the
    previous launch's costs: the first call runs them in index order, later calls heavy items first and
    light ones last.  Every call agrees with the oracle (ragged batch of 3)."""
    B, n = 3, 3000 + 5
    ws = [workloads.uniform_cube(n, 30.0, seed=70 + b) for b in range(B)]
    pos = np.stack([x.pos for x in ws])
    mom = np.stack([x.mom for x in ws])
    hext = np.array([0.2, 0.0, 0.4])
    bh = BarnesHut(n, B, 16, 0.5, precision, tuning_id=tuning_id)
    p = torch.from_numpy(pos).cuda()
    m = torch.from_numpy(mom).cuda()
    he = torch.from_numpy(hext).cuda()
    ge = torch.ones(B, dtype=torch.float64, device="cuda")
    bh.build(p)
    refs = [oracle_mod.Tree(x.pos, x.mom, 16).energy_grad(0.5, hext) for x in ws]
    for call in range(3):
        dr, dm = bh.field_backward(m, he, gE=ge)
        assert bh.check_status() == 0
        dr, dm = dr.cpu().numpy(), dm.cpu().numpy()
        for b in range(B):
            grad_check(dr[b], refs[b][2], precision, f"dE/dr call {call} system {b}")
            grad_check(dm[b], refs[b][3], precision, f"dE/dm call {call} system {b}")


def test_invariants_at_full_size_c4():
    """Differentiation workload at full size (N = 2^18): translation invariance and the energy symmetry
    of the transposed traversal hold at any size."""
    w = workloads.config4()
    gdr, gdm = _gpu_grad(w.pos, w.mom, np.zeros(3), 0.5, "fp64")
    assert np.abs(gdr.sum(axis=1)).max() <= 1e-10 * np.abs(gdr).sum()

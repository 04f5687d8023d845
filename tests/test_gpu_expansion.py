"""Order-2 cells (the paper's pseudo-particle plus each accepted cell's first moment; an accuracy variant
beyond the paper) through the C ABI against the oracle's order-2 traversal, whose pins are the opposed-pair
closed forms and the parallel-axis identity.  FP64 within 1e-12 (relative L2: the GPU forms a parent's
first moment from its children's, the oracle from the members), FP32-mixed within 1e-5.  The acceptance
decisions are the paper's, so interaction counts equal the order-1 counts."""
import numpy as np
import pytest
import torch

from paper_1212_2934_amd import workloads
from paper_1212_2934_amd.binding import BarnesHut, BHError, md_params
from gpu_util import run_field

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-12, "fp32_mixed": 1e-5}


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("kind,theta", [("uniform", 0.5), ("uniform", 0.8), ("chains", 0.5), ("chains", 0.3)])
def test_field_matches_oracle(oracle_mod, precision, kind, theta):
    w = workloads.uniform_cube(4096, 32.0, seed=1001) if kind == "uniform" else workloads.config3(seed=77, n=5000)
    out = run_field(w.pos, w.mom, theta=theta, precision=precision, expansion=2)
    assert out["flags"] == 0
    H2, nf, nr = oracle_mod.Tree(w.pos, w.mom, 16).field(theta, order=2)
    assert rel(out["H"], H2) <= TOL[precision]
    assert (out["n_far"] == nf).all() and (out["n_near"] == nr).all()
    # the energy follows the order-2 field
    E = -0.5 * np.sum(w.mom * H2)
    assert abs(out["E"][0] - E) <= TOL[precision] * abs(E)


def test_batched_ragged(oracle_mod):
    B, n = 3, 2000 + 77
    ws = [workloads.uniform_cube(n, 26.0, seed=40 + b) for b in range(B)]
    pos = np.stack([x.pos for x in ws])
    mom = np.stack([x.mom for x in ws])
    out = run_field(pos, mom, theta=0.6, precision="fp32_mixed", counters=False, expansion=2)
    for b, x in enumerate(ws):
        H2, _, _ = oracle_mod.Tree(x.pos, x.mom, 16).field(0.6, order=2)
        assert rel(out["H"][b], H2) <= 1e-5


def test_opposed_pair_closed_form():
    """+m z at (0,0,+delta), -m z at (0,0,-delta), target on the axis at R: 12 delta m / R^4 along z."""
    R, delta = 40.0, 0.3
    pos = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [delta, -delta, R]])
    mom = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 0.0], [1.0, -1.0, 0.0]])
    out = run_field(pos, mom, theta=0.9, leaf=2, precision="fp64", expansion=2)
    assert out["n_far"][2] == 1
    np.testing.assert_allclose(out["H"][:, 2], [0.0, 0.0, 12.0 * delta / R ** 4], rtol=1e-13, atol=1e-20)
    out1 = run_field(pos, mom, theta=0.9, leaf=2, precision="fp64", expansion=1)
    assert np.abs(out1["H"][:, 2]).max() == 0.0


@pytest.mark.parametrize("n", [1, 2, 5, 17, 300])
def test_small_systems(oracle_mod, n):
    w = workloads.uniform_cube(n, 4.0 + 2.0 * n ** (1.0 / 3.0), seed=90 + n)
    out = run_field(w.pos, w.mom, theta=0.7, precision="fp64", expansion=2)
    H2, _, _ = oracle_mod.Tree(w.pos, w.mom, 16).field(0.7, order=2)
    if n == 1:
        assert np.abs(out["H"]).max() == 0.0
    else:
        assert rel(out["H"], H2) <= 1e-12


def test_more_accurate_than_order_one(oracle_mod):
    w = workloads.uniform_cube(6000, 40.0, seed=13)
    Ha = oracle_mod.allpairs_field(w.pos, w.mom)
    e1 = rel(run_field(w.pos, w.mom, theta=0.5, precision="fp32_mixed", counters=False)["H"], Ha)
    e2 = rel(run_field(w.pos, w.mom, theta=0.5, precision="fp32_mixed", counters=False, expansion=2)["H"], Ha)
    assert e2 < 0.6 * e1, (e1, e2)


def test_backward_and_md_step_rejected():
    """The adjoint and the MD forces follow the paper's cells only: order-2 handles refuse them before
    anything is enqueued."""
    w = workloads.uniform_cube(500, 12.0, seed=3)
    bh = BarnesHut(w.n, 1, 16, 0.5, "fp64", expansion=2)
    p = torch.from_numpy(w.pos).cuda()
    m = torch.from_numpy(w.mom).cuda()
    bh.build(p)
    with pytest.raises(BHError) as ei:
        bh.field_backward(m, gE=torch.ones(1, dtype=torch.float64, device="cuda"))
    assert ei.value.status == -1
    st = {"pos": p.clone(), "vel": torch.zeros_like(p), "mom": m.clone(), "omega": torch.zeros_like(p),
          "step": torch.zeros(1, dtype=torch.int64, device="cuda")}
    C3 = __import__("ctypes").c_double * 3
    mdp = md_params(1e-3, 1.0, 0.1, 0.1, 1.0, 0.1, 1.0, 1.0, C3(0, 0, 0), C3(12, 12, 12), None, 1)
    with pytest.raises(BHError):
        bh.md_step(st, mdp)
    assert torch.equal(st["pos"], p)

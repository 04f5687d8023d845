"""The oracle's subset functions (the checkers of sampled targets at full size) against its full functions:
every row of a subset evaluation is bitwise equal to the same particle's row of the full evaluation, for
targets in any order, repeated, and at the ends of the index range.  The full functions are pinned by the
closed forms, the brute-force definition of the traversal and the invariants of the other oracle tests."""
import numpy as np
import pytest

from paper_1212_2934_amd import workloads


@pytest.fixture(scope="module")
def system():
    w = workloads.uniform_cube(3000, 24.0, seed=41, hext=(0.0, 0.0, 0.0))
    rng = np.random.default_rng(5)
    t = np.concatenate([[0, w.n - 1, 17, 17], rng.choice(w.n, 200, replace=False)])
    return w, t


def test_allpairs_field_subset_rows(oracle_mod, system):
    w, t = system
    H = oracle_mod.allpairs_field(w.pos, w.mom)
    Hs = oracle_mod.allpairs_field_subset(w.pos, w.mom, t)
    assert np.array_equal(Hs, H[:, t])


def test_allpairs_grad_subset_rows(oracle_mod, system):
    w, t = system
    g = oracle_mod.allpairs_grad_r(w.pos, w.mom)
    gs = oracle_mod.allpairs_grad_r_subset(w.pos, w.mom, t)
    assert np.array_equal(gs, g[:, t])


@pytest.mark.parametrize("theta", [0.0, 0.5, 0.9])
def test_bh_field_subset_rows(oracle_mod, system, theta):
    w, t = system
    tree = oracle_mod.Tree(w.pos, w.mom, 16)
    H, nf, nr = tree.field(theta)
    Hs, nfs, nrs = tree.field_subset(theta, t)
    assert np.array_equal(Hs, H[:, t])
    assert np.array_equal(nfs, nf[t]) and np.array_equal(nrs, nr[t])

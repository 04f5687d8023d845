"""Pins of the oracle's pair kernels against hand-worked closed forms and independent formulas.

Eq. (H_dip) and the reduced force f_dip are from Sec. 2 of the paper; the golden values are worked by hand
(tests/golden/closed_forms.json).  The pairwise energy formula used below, sum_{i<j} [m_i.m_j -
3 (m_i.u)(m_j.u)] / r^3, is the textbook dipole-dipole energy; it shares no code or arrangement with the
oracle's field-then-energy route.
"""
import json
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def _cases():
    with open(GOLD) as f:
        return json.load(f)


@pytest.mark.parametrize("case", _cases()["cases"], ids=lambda c: c["name"])
def test_allpairs_closed_forms(oracle_mod, case):
    pos = np.array(case["pos"], float)
    mom = np.array(case["mom"], float)
    H = oracle_mod.allpairs_field(pos, mom)
    np.testing.assert_allclose(H, np.array(case["H"]), rtol=1e-14, atol=1e-15)
    E = oracle_mod.energy(mom, H)
    assert abs(E - case["E"]) <= 1e-14 * max(1.0, abs(case["E"]))


@pytest.mark.parametrize("case", _cases()["cases"], ids=lambda c: c["name"])
def test_bh_closed_forms_theta_half(oracle_mod, case):
    # with fewer particles than a leaf the tree is one leaf: Barnes-Hut is the direct sum
    pos = np.array(case["pos"], float)
    mom = np.array(case["mom"], float)
    H, nf, nr = oracle_mod.Tree(pos, mom, 16).field(0.5)
    np.testing.assert_allclose(H, np.array(case["H"]), rtol=1e-14, atol=1e-15)
    assert nf.sum() == 0 and (nr == pos.shape[1] - 1).all()


def test_two_dipole_gradient(oracle_mod):
    g = _cases()["gradient"]
    r = g["r"]
    pos = np.array([[0.0, 0.0], [0.0, 0.0], [0.0, r]])
    mom = np.array([[0.0, 0.0], [0.0, 0.0], [1.0, 1.0]])
    d = oracle_mod.allpairs_grad_r(pos, mom)
    assert abs(d[2, 1] - g["dEdz_upper"]) < 1e-14
    assert abs(d[2, 0] + g["dEdz_upper"]) < 1e-14
    assert np.abs(d[:2]).max() < 1e-15
    # the adjoint of the one-leaf tree gives the same
    _, _, dr, _ = oracle_mod.Tree(pos, mom, 16).energy_grad(0.5)
    np.testing.assert_allclose(dr, d, rtol=1e-14, atol=1e-15)


def _pairwise_energy(pos, mom):
    n = pos.shape[1]
    e = 0.0
    for i in range(n):
        for j in range(i + 1, n):
            x = pos[:, i] - pos[:, j]
            r = np.sqrt(x @ x)
            u = x / r
            e += (mom[:, i] @ mom[:, j] - 3.0 * (mom[:, i] @ u) * (mom[:, j] @ u)) / r ** 3
    return e


def _random_system(seed, n=24, side=6.0):
    from paper_1212_2934_amd.workloads import rsa_uniform, unit_vectors
    rng = np.random.default_rng(seed)
    pos = rsa_uniform(rng, n, (0, 0, 0), (side, side, side))
    mom = unit_vectors(rng, n) * rng.uniform(0.5, 1.5, size=n)  # non-unit moments too
    return pos, mom


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_allpairs_energy_matches_pairwise_formula(oracle_mod, seed):
    pos, mom = _random_system(seed)
    H = oracle_mod.allpairs_field(pos, mom)
    e1 = oracle_mod.energy(mom, H)
    e2 = _pairwise_energy(pos, mom)
    assert abs(e1 - e2) <= 1e-12 * np.abs(H * mom).sum()


@pytest.mark.parametrize("seed", [4, 5])
def test_allpairs_gradient_matches_fd_of_pairwise_energy(oracle_mod, seed):
    pos, mom = _random_system(seed, n=12, side=4.0)
    g = oracle_mod.allpairs_grad_r(pos, mom)
    h = 1e-6
    fd = np.zeros_like(pos)
    for a in range(3):
        for i in range(pos.shape[1]):
            p = pos.copy()
            p[a, i] += h
            ep = _pairwise_energy(p, mom)
            p[a, i] -= 2 * h
            em = _pairwise_energy(p, mom)
            fd[a, i] = (ep - em) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-6 * np.abs(g).max()
    # Newton's third law: the forces sum to zero
    assert np.abs(g.sum(axis=1)).max() <= 1e-13 * np.abs(g).sum()


def test_allpairs_rotation_covariance(oracle_mod):
    pos, mom = _random_system(7)
    rng = np.random.default_rng(0)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    H = oracle_mod.allpairs_field(pos, mom)
    Hr = oracle_mod.allpairs_field(q @ pos, q @ mom)
    np.testing.assert_allclose(Hr, q @ H, rtol=0, atol=1e-13 * np.abs(H).max())

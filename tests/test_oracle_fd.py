"""Central finite differences (h = 1e-6, FP64) of the frozen-structure Barnes-Hut energy against the
oracle's adjoint, on the 512-particle subset of the differentiation workload (the particles nearest the
centre of the N = 2^18, phi = 0.05 cube, taken as a standalone system with H_ext = (0, 0, 1), theta 0.5).

E = -1/2 sum m_i.H_i - sum m_i.H_ext with H the Barnes-Hut field (Sec. 3.2 traversal, Eq. magCenter
pseudo-particles, Eq. H_dip pair field); the tree, memberships and acceptance decisions are frozen, so the
energy is a smooth function of (r, m) whose exact gradient the adjoint must return.
"""
import numpy as np
import pytest

from paper_1212_2934_amd import workloads


@pytest.fixture(scope="module")
def subset512():
    w = workloads.config4()
    idx = workloads.nearest_to_centre(w.pos, 512)
    return w.pos[:, idx].copy(), w.mom[:, idx].copy(), w.hext.copy()


def test_frozen_energy_equals_traversal_energy(oracle_mod, subset512):
    pos, mom, hext = subset512
    t = oracle_mod.Tree(pos, mom, 16)
    H, E, _, _ = t.energy_grad(0.5, hext)
    st = oracle_mod.frozen_structure(t, 0.5)
    Ef = oracle_mod.energy_frozen(pos, mom, hext, st)
    assert abs(E - Ef) <= 1e-12 * np.abs(mom * H).sum()


def test_adjoint_matches_central_fd(oracle_mod, subset512):
    pos, mom, hext = subset512
    t = oracle_mod.Tree(pos, mom, 16)
    _, _, dr, dm = t.energy_grad(0.5, hext)
    st = oracle_mod.frozen_structure(t, 0.5)
    assert st["far_ptr"][-1] > 0  # the subset has far-field interactions
    fr, fm = oracle_mod.fd_grad_frozen(pos, mom, hext, st, 1e-6)
    err_r = np.linalg.norm(dr - fr) / np.linalg.norm(dr)
    err_m = np.linalg.norm(dm - fm) / np.linalg.norm(dm)
    assert err_r < 1e-7 and err_m < 1e-7, (err_r, err_m)
    assert np.abs(dr - fr).max() < 1e-6 * np.abs(dr).max()

"""Pins of the oracle's order-2 cells (the first-moment term added to the paper's pseudo-particle; an
accuracy variant beyond the paper): closed forms for an opposed dipole pair seen from its axis and from its
equatorial plane, the parallel-axis identity and the vanishing cases of the first moment, theta = 0, and
the gain in accuracy against the all-pairs sum."""
import numpy as np

from paper_1212_2934_amd import workloads


def _pair_and_target(target, delta, m):
    """Dipoles +m z at (0,0,+delta) and -m z at (0,0,-delta), then one target particle (moment x)."""
    pos = np.array([[0.0, 0.0, target[0]], [0.0, 0.0, target[1]], [delta, -delta, target[2]]])
    mom = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 0.0], [m, -m, 0.0]])
    return pos, mom


def test_opposed_pair_on_axis(oracle_mod):
    """On the axis, at distance R from the pair's centre, the first-moment field is 12 delta m / R^4 along
    z (D = 2 delta m z z^T; the expansion of 2m [(R - delta)^-3 - (R + delta)^-3]); the pseudo-particle
    alone (M = 0) gives nothing."""
    R, delta, m = 40.0, 0.3, 1.0
    pos, mom = _pair_and_target((0.0, 0.0, R), delta, m)
    t = oracle_mod.Tree(pos, mom, 2)
    H2, nf, _ = t.field(0.9, order=2)
    H1, _, _ = t.field(0.9, order=1)
    assert nf[2] == 1  # the pair's leaf is accepted by the target
    np.testing.assert_allclose(H2[:, 2], [0.0, 0.0, 12.0 * delta * m / R ** 4], rtol=1e-13, atol=1e-20)
    assert np.abs(H1[:, 2]).max() == 0.0
    # the exact sum is 12 delta m / R^4 (1 + (10/3) eps^2 + O(eps^4)), eps = delta / R
    exact = oracle_mod.allpairs_field(pos, mom)[:, 2]
    eps = delta / R
    np.testing.assert_allclose(exact[2] - H2[2, 2], 10.0 / 3.0 * eps ** 2 * H2[2, 2], rtol=0.01)
    # the pair members see each other directly and the single target through its own (D = 0) cell
    np.testing.assert_allclose(H2[:, :2], oracle_mod.allpairs_field(pos, mom)[:, :2], rtol=1e-13)


def test_opposed_pair_in_equatorial_plane(oracle_mod):
    """In the pair's equatorial plane the first-moment field is -6 delta m / R^4 along the offset."""
    R, delta, m = 30.0, 0.2, 1.0
    pos, mom = _pair_and_target((R, 0.0, 0.0), delta, m)
    t = oracle_mod.Tree(pos, mom, 2)
    H2, nf, _ = t.field(0.9, order=2)
    assert nf[2] == 1
    np.testing.assert_allclose(H2[:, 2], [-6.0 * delta * m / R ** 4, 0.0, 0.0], rtol=1e-13, atol=1e-20)
    # the exact sum is -6 R delta m / (R^2 + delta^2)^(5/2) = -6 delta m / R^4 (1 - (5/2) eps^2 + O(eps^4))
    exact = oracle_mod.allpairs_field(pos, mom)[:, 2]
    eps = delta / R
    np.testing.assert_allclose(exact[0] - H2[0, 2], -2.5 * eps ** 2 * H2[0, 2], rtol=0.01)


def test_first_moment_identities(oracle_mod):
    w = workloads.uniform_cube(3000, 28.0, seed=17)
    t = oracle_mod.Tree(w.pos, w.mom, 8)
    e = t.export()
    D = t.first_moments()
    nn = e["count"].size
    # single-member cells have no first moment
    assert np.abs(D[e["count"] == 1]).max() == 0.0
    # parallel axis: a parent's first moment is its children's, shifted to the parent's centre
    for p in range(nn):
        k = int(e["nchild"][p])
        if k == 0:
            continue
        ch = e["child"][p, :k]
        shifted = D[ch].sum(axis=0) + np.einsum("ck,cb->kb", e["c"][ch] - e["c"][p], e["M"][ch])
        np.testing.assert_allclose(D[p], shifted, rtol=0, atol=1e-10 * (1.0 + np.abs(D[p]).max()))
    # cells whose members share one moment have D = (sum of offsets) m^T = 0
    same = np.tile(np.array([[0.6], [0.0], [0.8]]), (1, w.n))
    Ds = oracle_mod.Tree(w.pos, same, 8).first_moments()
    bound = 1e-14 * e["count"] * 28.0  # rounding of count terms of size <= side
    assert (np.abs(Ds).reshape(nn, 9).max(axis=1) <= bound).all()
    # translation leaves D unchanged
    Dt = oracle_mod.Tree(w.pos + np.array([[3.25], [-7.5], [11.0]]), w.mom, 8).first_moments()
    np.testing.assert_allclose(Dt, D, rtol=0, atol=1e-9)


def test_theta_zero_is_the_direct_sum(oracle_mod):
    w = workloads.uniform_cube(800, 16.0, seed=5)
    t = oracle_mod.Tree(w.pos, w.mom, 16)
    H2, nf, _ = t.field(0.0, order=2)
    H1, _, _ = t.field(0.0, order=1)
    assert nf.max() == 0
    assert np.array_equal(H1, H2)
    Ha = oracle_mod.allpairs_field(w.pos, w.mom)
    assert np.linalg.norm(H2 - Ha) <= 1e-13 * np.linalg.norm(Ha)


def test_order_two_is_more_accurate(oracle_mod):
    """Against the all-pairs sum the first-moment term cuts the error at every theta, by more at smaller
    theta (one more power of theta): a dropped term or a wrong sign would raise it instead."""
    w = workloads.uniform_cube(2000, 24.0, seed=3)
    t = oracle_mod.Tree(w.pos, w.mom, 16)
    Ha = oracle_mod.allpairs_field(w.pos, w.mom)
    ratio = {}
    for th in (0.25, 0.5, 0.7):
        e1 = np.linalg.norm(t.field(th, 1)[0] - Ha) / np.linalg.norm(Ha)
        e2 = np.linalg.norm(t.field(th, 2)[0] - Ha) / np.linalg.norm(Ha)
        assert e2 < 0.7 * e1, (th, e1, e2)
        ratio[th] = e1 / e2
    assert ratio[0.25] > 1.5 * ratio[0.5] and ratio[0.5] > ratio[0.7]
    slope = np.log(ratio[0.25] / ratio[0.5]) / np.log(2.0)  # gained power of theta
    assert 0.5 < slope < 1.6, slope


def test_order_two_adjoint_matches_finite_differences(oracle_mod):
    """The order-2 adjoint (the first-moment term's gradient to targets and cell centres, dL/dD_C to the
    members) against central differences of the frozen-structure order-2 energy; the frozen energy itself
    equals the traversal's."""
    w = workloads.uniform_cube(240, 9.0, seed=23, hext=(0.1, -0.2, 0.3))
    t = oracle_mod.Tree(w.pos, w.mom, 4)
    st = oracle_mod.frozen_structure(t, 0.7)
    assert st["far_ptr"][-1] > 5 * w.n  # many accepted cells, so the first-moment terms matter
    H, E, dr, dm = t.energy_grad(0.7, w.hext, order=2)
    Ef = oracle_mod.energy_frozen(w.pos, w.mom, w.hext, st, order=2)
    assert abs(Ef - E) <= 1e-13 * abs(E)
    fr, fm = oracle_mod.fd_grad_frozen(w.pos, w.mom, w.hext, st, h=1e-6, order=2)
    assert np.linalg.norm(dr - fr) <= 1e-7 * np.linalg.norm(fr)
    assert np.linalg.norm(dm - fm) <= 1e-7 * np.linalg.norm(fm)
    # and the order-2 terms are not negligible here: the order-1 gradient differs by far more
    _, _, dr1, dm1 = t.energy_grad(0.7, w.hext, order=1)
    assert np.linalg.norm(dr1 - fr) > 100 * np.linalg.norm(dr - fr)

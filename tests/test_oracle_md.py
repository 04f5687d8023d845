"""Pins of the MD reference: its Philox stream and Box-Muller normals against distribution laws, the
deterministic friction decay of a free particle (exact geometric law of the Euler scheme), equipartition of
translational and rotational kinetic energy, and the Langevin magnetisation law <m.h> = L(|h|/kT) of
non-interacting dipoles (Eq. Langevin, Sec. 5), which fixes the sign of the torque m x H and the noise
amplitude together."""
import json
import os

import numpy as np
import pytest

from oracle import md

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_philox_known_answer_vectors():
    """The generator against the known-answer vectors its authors publish (Salmon et al., SC'11): a wrong
    multiplier, Weyl constant, round count or word order changes every output word."""
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        ctr = [np.array([int(x, 16)], np.uint64) for x in c["ctr"]]
        k0, k1 = (np.uint64(int(x, 16)) for x in c["key"])
        out = md.philox4x32_10(*ctr, k0, k1)
        assert ["%08x" % int(w[0]) for w in out] == c["out"], c["name"]


def test_philox_words_uniform_and_independent():
    n = 1 << 18
    i = np.arange(n, dtype=np.uint64)
    w = md.philox4x32_10(np.full(n, 7), np.zeros(n), i, np.zeros(n), 123, 456)
    allw = np.concatenate(w)
    u = (allw.astype(np.float64) + 0.5) / 2 ** 32
    assert abs(u.mean() - 0.5) < 2e-3
    # every bit is set half of the time
    for bit in range(32):
        f = ((allw >> np.uint64(bit)) & np.uint64(1)).mean()
        assert abs(f - 0.5) < 3e-3, bit
    # chi-square over 256 equal bins
    h = np.bincount((allw >> np.uint64(24)).astype(np.int64), minlength=256)
    chi2 = ((h - allw.size / 256) ** 2 / (allw.size / 256)).sum()
    assert chi2 < 400  # 255 dof: mean 255, sd ~23
    # neighbouring counters and the four words are uncorrelated
    for a in range(4):
        for b in range(a + 1, 4):
            assert abs(np.corrcoef(w[a].astype(float), w[b].astype(float))[0, 1]) < 0.01
    assert abs(np.corrcoef(w[0][:-1].astype(float), w[0][1:].astype(float))[0, 1]) < 0.01
    # a different key gives a different stream
    w2 = md.philox4x32_10(np.full(n, 7), np.zeros(n), i, np.zeros(n), 124, 456)
    assert (w2[0] != w[0]).mean() > 0.99


def test_normals_moments():
    x = np.concatenate([md.normals(99, b, s, 20000).ravel() for b in range(2) for s in range(3)])
    assert abs(x.mean()) < 0.01
    assert abs(x.var() - 1.0) < 0.01
    assert abs((x ** 4).mean() - 3.0) < 0.05
    assert abs((x ** 3).mean()) < 0.03


def _params(**kw):
    p = dict(dt=1e-3, kT=1.0, gamma_t=0.1, gamma_r=0.1, mass=1.0, inertia=0.1, wca_eps=0.0, wca_sigma=1.0,
             box_lo=(-1e3, -1e3, -1e3), box_hi=(1e3, 1e3, 1e3), hext=None, seed=5)
    p.update(kw)
    return p


def test_free_particle_friction_decay():
    st = dict(pos=np.array([[[0.0], [0.0], [0.0]]]), vel=np.array([[[1.0], [-2.0], [0.5]]]),
              mom=np.array([[[0.0], [0.0], [1.0]]]), omega=np.array([[[0.3], [0.0], [0.0]]]))
    p = _params(kT=0.0, gamma_t=2.0, gamma_r=1.0, dt=0.01)
    v0, r0 = st["vel"].copy(), st["pos"].copy()
    r_exp = r0.copy()
    for k in range(50):
        r_exp = r_exp + p["dt"] * v0 * (1 - p["gamma_t"] * p["dt"]) ** k
        st = md.md_step(st, p, k)
    np.testing.assert_allclose(st["vel"], v0 * (1 - p["gamma_t"] * p["dt"]) ** 50, rtol=1e-12)
    np.testing.assert_allclose(st["pos"], r_exp, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(st["omega"][0, 0, 0], 0.3 * (1 - p["gamma_r"] * p["dt"] / p["inertia"]) ** 50,
                               rtol=1e-12)
    assert abs(np.linalg.norm(st["mom"][0, :, 0]) - 1.0) < 1e-14


def test_equipartition_noninteracting():
    rng = np.random.default_rng(3)
    n = 3000
    st = dict(pos=rng.uniform(-50, 50, (1, 3, n)), vel=np.zeros((1, 3, n)),
              mom=np.tile(np.array([[[0.0], [0.0], [1.0]]]), (1, 1, n)), omega=np.zeros((1, 3, n)))
    p = _params(gamma_t=1.0, gamma_r=1.0, dt=0.01)
    v2, w2 = [], []
    for k in range(1500):
        st = md.md_step(st, p, k, field=False)
        if k >= 500:
            v2.append((st["vel"] ** 2).sum(axis=1).mean())
            w2.append((st["omega"] ** 2).sum(axis=1).mean())
    assert abs(np.mean(v2) / (3 * p["kT"] / p["mass"]) - 1.0) < 0.05
    assert abs(np.mean(w2) / (3 * p["kT"] / p["inertia"]) - 1.0) < 0.15  # EM bias O(gamma_r dt / I)


@pytest.mark.parametrize("alpha", [0.7, 2.0])
def test_langevin_magnetisation_law(alpha):
    rng = np.random.default_rng(int(alpha * 10))
    n = 3000
    m0 = rng.standard_normal((1, 3, n))
    m0 /= np.linalg.norm(m0, axis=1, keepdims=True)
    st = dict(pos=rng.uniform(-50, 50, (1, 3, n)), vel=np.zeros((1, 3, n)), mom=m0, omega=np.zeros((1, 3, n)))
    p = _params(gamma_r=1.0, gamma_t=1.0, inertia=0.1, dt=2e-3, hext=np.array([[0.0, 0.0, alpha]]))
    mz = []
    for k in range(6000):
        st = md.md_step(st, p, k, field=False)
        if k >= 1500:
            mz.append(st["mom"][0, 2].mean())
    assert abs(np.mean(mz) - md.langevin(alpha)) < 0.015, (np.mean(mz), md.langevin(alpha))


def test_paper_short_range_force_law():
    """Eq. LJ as printed: the force vanishes at r = s (the equilibrium distance the paper names), is minus the
    derivative of the potential 2 eps (s/r)^12 - 4 eps (s/r)^6 (well depth 2 eps at s; checked by central
    differences of that potential, written independently of the force), repels below s, attracts above,
    and is cut at 2.5 s by default."""
    s, eps = 1.3, 0.7
    pot = lambda r: 2.0 * eps * (s / r) ** 12 - 4.0 * eps * (s / r) ** 6
    for r in (0.9 * s, s, 1.2 * s, 2.0 * s):
        pos = np.array([[0.0, r], [0.0, 0.0], [0.0, 0.0]])
        F = md.lj_forces(pos, s, eps)
        h = 1e-6 * r
        fd = -(pot(r + h) - pot(r - h)) / (2.0 * h)
        assert abs(F[0, 1] - fd) <= 1e-6 * max(1.0, abs(fd)), (r, F[0, 1], fd)
        assert F[0, 0] == -F[0, 1] and not F[1:].any()
    assert md.lj_forces(np.array([[0.0, s], [0.0, 0.0], [0.0, 0.0]]), s, eps)[0, 1] == 0.0
    far = np.array([[0.0, 2.6 * s], [0.0, 0.0], [0.0, 0.0]])
    assert not md.lj_forces(far, s, eps).any()
    assert md.lj_forces(far, s, eps, cut=3.0 * s)[0, 1] < 0.0  # attractive: particle 1 (at +x) pulled back


def test_paper_short_range_momentum_and_walls():
    rng = np.random.default_rng(12)
    pos = rng.uniform(0.0, 6.0, (3, 200))
    F = md.lj_forces(pos, 1.0, 1.0)
    assert np.abs(F.sum(axis=1)).max() <= 1e-9 * np.abs(F).max()  # pair forces cancel
    # walls of the same type (sigma_w = sigma / 2): zero at distance sigma_w, repulsive inside, attractive
    # outside up to half the pair cut-off
    lo, hi = (0.0, 0.0, 0.0), (10.0, 10.0, 10.0)
    x = np.array([[0.5, 0.4, 0.8, 1.3, 5.0], [5.0] * 5, [5.0] * 5])
    W = md.wall_forces(x, lo, hi, 1.0, 1.0, kind=1)
    assert W[0, 0] == 0.0 and W[0, 1] > 0.0 and W[0, 2] < 0.0 and W[0, 3] == 0.0 and W[0, 4] == 0.0
    assert not W[1:].any()


def _wca_potential(r, s, eps):
    """WCA potential written from its definition (Weeks, Chandler, Andersen 1971): the Lennard-Jones
    potential 4 eps [(s/r)^12 - (s/r)^6] cut at its minimum 2^(1/6) s and shifted up by eps, zero beyond."""
    rc = 2.0 ** (1.0 / 6.0) * s
    return np.where(r < rc, 4.0 * eps * ((s / r) ** 12 - (s / r) ** 6) + eps, 0.0)


def test_wca_pair_force_law():
    """The default short-range law: minus the derivative of the WCA potential (central differences of the
    potential above, written independently of the force), repulsive everywhere inside the cut, exactly zero
    at and beyond 2^(1/6) s, and equal and opposite on the two particles."""
    s, eps = 1.3, 0.7
    rc = 2.0 ** (1.0 / 6.0) * s
    for r in (0.85 * s, 0.95 * s, s, 1.05 * s, 0.999 * rc):
        pos = np.array([[0.0, r], [0.0, 0.0], [0.0, 0.0]])
        F = md.wca_forces(pos, s, eps)
        h = 1e-6 * r
        fd = -(_wca_potential(r + h, s, eps) - _wca_potential(r - h, s, eps)) / (2.0 * h)
        assert abs(F[0, 1] - fd) <= 1e-6 * max(1.0, abs(fd)), (r, F[0, 1], fd)
        assert F[0, 1] > 0.0  # particle 1 (at +x) pushed away
        assert F[0, 0] == -F[0, 1] and not F[1:].any()
    # the force of the law is zero at the cut itself (the minimum of the unshifted potential)
    at_cut = 24.0 * eps * (2.0 * 0.5 ** 2 - 0.5) / rc
    assert abs(at_cut) < 1e-15
    for r in (rc, 1.01 * rc, 2.0 * s):
        pos = np.array([[0.0, r], [0.0, 0.0], [0.0, 0.0]])
        assert not md.wca_forces(pos, s, eps).any(), r
    # a skew pair: the force points along the separation with the magnitude of the radial law
    d = np.array([0.4, -0.5, 0.6])
    pos = np.stack([np.zeros(3), d], axis=1)
    F = md.wca_forces(pos, s, eps)
    r = np.linalg.norm(d)
    h = 1e-6 * r
    fr = -(_wca_potential(r + h, s, eps) - _wca_potential(r - h, s, eps)) / (2.0 * h)
    np.testing.assert_allclose(F[:, 1], fr * d / r, rtol=1e-6)


def test_wca_walls():
    """WCA walls on the centre-to-face distance with s_w = s / 2: minus the derivative of the WCA potential
    of s_w in that distance (pushing the particle into the box), zero from 2^(1/6) s_w on, floored at
    s_w / 10, and each face acting only along its own axis."""
    s, eps = 1.0, 1.0
    sw = 0.5 * s
    lo, hi = (0.0, 0.0, 0.0), (10.0, 10.0, 10.0)
    for dist in (0.3, 0.45, 0.5, 0.55):
        x = np.array([[dist, 10.0 - dist], [5.0, 5.0], [5.0, 5.0]])
        W = md.wall_forces(x, lo, hi, s, eps, kind=0)
        h = 1e-7
        fd = -(_wca_potential(dist + h, sw, eps) - _wca_potential(dist - h, sw, eps)) / (2.0 * h)
        assert abs(W[0, 0] - fd) <= 1e-6 * max(1.0, abs(fd)), (dist, W[0, 0], fd)
        assert W[0, 0] > 0.0 and abs(W[0, 1] + W[0, 0]) <= 1e-12 * W[0, 0]  # 10 - (10 - d) rounds
        assert not W[1:].any()
    rcw = 2.0 ** (1.0 / 6.0) * sw
    x = np.array([[rcw, 1.0, 5.0], [5.0] * 3, [5.0] * 3])
    assert not md.wall_forces(x, lo, hi, s, eps, kind=0).any()
    # below a tenth of s_w the distance is floored: the force stops growing
    x = np.array([[0.01, 0.04], [5.0, 5.0], [5.0, 5.0]])
    W = md.wall_forces(x, lo, hi, s, eps, kind=0)
    assert W[0, 0] == W[0, 1] > 0.0


def _wall_bounce(v0, eps, dt, z0=2.0, steps=100000):
    """Outgoing speed of one particle thrown at a WCA wall under the explicit update (positions advance
    with the velocity of the start of the step), no friction, no noise."""
    pos = np.array([[5.0], [5.0], [z0]])
    vel = np.array([[0.0], [0.0], [-v0]])
    for _ in range(steps):
        F = md.wall_forces(pos, (0.0, 0.0, 0.0), (10.0, 10.0, 10.0), 1.0, eps, 0)
        pos, vel = pos + dt * vel, vel + dt * F
        if pos[2, 0] > z0 and vel[2, 0] > 0:
            return float(vel[2, 0])
    raise AssertionError("no bounce")


def test_explicit_step_gains_energy_at_a_stiff_wall():
    """Stability limit of the explicit Euler-Maruyama step (Sec. 4) at WCA contacts: the position moves with
    the old velocity, so the particle overshoots into the wall by v dt and leaves faster than it came.  At
    eps = kT = 7.14 (the magnetisation benchmark's lambda = 0.28) and dt = 1e-3 the speed grows by 17 % at
    5 and 80 % at 20, which a friction of 0.1 cannot remove; at dt = 2.5e-4 the gain at 20 is 13 %.  (The
    pin is on the reference scheme; the GPU step follows it to 1e-12.)"""
    g = lambda v0, eps, dt: _wall_bounce(v0, eps, dt) / v0
    assert 1.15 < g(5.0, 7.142857, 1e-3) < 1.20
    assert 1.7 < g(20.0, 7.142857, 1e-3) < 1.9
    assert g(20.0, 7.142857, 1e-3) > g(10.0, 7.142857, 1e-3) > g(5.0, 7.142857, 1e-3)  # grows with speed
    assert 1.10 < g(20.0, 7.142857, 2.5e-4) < 1.16
    assert g(2.0, 1.0, 1e-3) < 1.07  # the benchmark's kT = eps = 1: thermal speeds gain a few per cent

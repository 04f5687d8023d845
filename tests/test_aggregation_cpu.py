"""Host logic of the chain-formation driver: the SI -> reduced-unit mapping against the paper's own
definitions (Eq. lambda; T_ch of Sec. 2), and the bond / cluster analysis on hand-built configurations."""
import math

import numpy as np

from paper_1212_2934_amd import aggregation as agg


def test_reduced_units_reproduce_the_papers_coupling_constant():
    T, Ms, R, D = 300.0, 3.1e5, 10e-9, 5000.0
    u = agg.reduced_units(T=T, Ms=Ms, R=R)
    m = Ms * 4.0 / 3.0 * math.pi * R ** 3
    lam = agg.MU0 * m * m / (16.0 * math.pi * R ** 3 * agg.KB * T)  # Eq. lambda, SI
    assert abs(u["lambda"] - lam) < 1e-12 * lam
    assert 10.1 < lam < 10.3
    # time unit: t0 = sqrt(M d^2 / e0) against the paper's T_ch = (R / Ms) sqrt(3 D / (4 mu0))
    M = D * 4.0 / 3.0 * math.pi * R ** 3
    e0 = agg.MU0 * m * m / (4.0 * math.pi * (2 * R) ** 3)
    t0 = math.sqrt(M * (2 * R) ** 2 / e0)
    tch = R / Ms * math.sqrt(3.0 * D / (4.0 * agg.MU0))
    assert abs(t0 / tch - u["t0_over_Tch"]) < 1e-12 * u["t0_over_Tch"]
    assert abs(u["dt"] * u["t0_over_Tch"] - 1e-3) < 1e-15
    # the rotational friction per inertia in T_ch units is Gamma_r / (2/5): (gamma_r / I) t0 / ratio
    assert abs(u["gamma_r"] / u["inertia"] / u["t0_over_Tch"] - 0.1 / 0.4) < 1e-12


def _chain(start, axis, k, spacing=1.05):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    p = np.asarray(start, float)[None] + spacing * np.arange(k)[:, None] * a[None]
    return p, np.tile(a, (k, 1))


def test_clusters_on_hand_built_chains():
    parts = [_chain((5, 5, 5), (1, 0, 0), 5), _chain((20, 5, 5), (0, 1, 0), 5), _chain((5, 20, 20), (1, 1, 1), 3)]
    # a side-by-side parallel pair repels (u = +1/r^3): not bonded
    parts.append((np.array([[40.0, 40, 40], [40.0, 41.1, 40]]), np.array([[0.0, 0, 1], [0.0, 0, 1]])))
    # an antiparallel head-to-tail pair (u = +2/r^3) is not bonded either
    parts.append((np.array([[50.0, 50, 50], [50.0, 50, 51.05]]), np.array([[0.0, 0, 1], [0.0, 0, -1]])))
    # isolated particles
    parts.append((np.array([[60.0 + 3 * i, 10, 10] for i in range(6)]), np.tile([0.0, 0, 1], (6, 1))))
    p = np.concatenate([a for a, _ in parts]).T
    m = np.concatenate([b for _, b in parts]).T
    c = agg.clusters(p, m)
    n = p.shape[1]
    assert n == 5 + 5 + 3 + 2 + 2 + 6
    assert c["clusters"] == 3
    assert abs(c["mean_cluster_size"] - 13 / 3) < 1e-12
    assert c["largest_cluster"] == 5
    assert abs(c["bonded_fraction"] - 13 / n) < 1e-12
    assert abs(c["bonds_per_particle"] - 2 * (4 + 4 + 2) / n) < 1e-12
    assert c["branch_fraction"] == 0.0


def test_clusters_branch_and_threshold():
    # a Y junction: three neighbours at 120 degrees around a centre with m along x, each moment set to the
    # direction of the centre's dipole field there, u = -sqrt(1 + 3 cos^2) / r^3 = -1.14 for |cos| = 1/2
    r = 1.05
    p, m = [np.zeros(3)], [np.array([1.0, 0, 0])]
    for ang in (0.0, 2 * math.pi / 3, 4 * math.pi / 3):
        e = np.array([math.cos(ang), math.sin(ang), 0.0])
        h = 3.0 * e[0] * e - np.array([1.0, 0, 0])
        p.append(r * e)
        m.append(h / np.linalg.norm(h))
    c = agg.clusters(np.array(p).T, np.array(m).T)
    assert c["clusters"] == 1 and c["largest_cluster"] == 4
    assert c["branch_fraction"] == 0.25 and c["bonds_per_particle"] == 1.5
    # beyond 1.3 d no bond, however favourable the orientation
    c2 = agg.clusters(np.array([[0.0, 0, 0], [1.31, 0, 0]]).T, np.array([[1.0, 0, 0], [1.0, 0, 0]]).T)
    assert c2["clusters"] == 0 and c2["bonded_fraction"] == 0.0
    # an energy just below -1 at 1.25 d (head-to-tail u = -2 / 1.25^3 = -1.024) bonds
    c3 = agg.clusters(np.array([[0.0, 0, 0], [1.25, 0, 0]]).T, np.array([[1.0, 0, 0], [1.0, 0, 0]]).T)
    assert c3["clusters"] == 1

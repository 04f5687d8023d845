"""Physics-level check of md_step (the magnetisation benchmark of Sec. 5, scaled down): weakly coupled
dipoles (lambda = 0.28, phi = 0.01) in a field along z reach the Langevin magnetisation <u_z> = L(alpha)
(Eq. Langevin) to within the small dipolar enhancement the paper describes, the mean dipolar field points
along the applied field, and the Barnes-Hut and all-pairs evaluations of it agree on sampled states.
Friction 1.0 keeps the explicit Euler-Maruyama heating of the rotation (about (torque frequency)^2 dt
against 2 gamma_r / I) near 1 % at dt = 1e-3."""
import pytest

from paper_1212_2934_amd.magnetisation import run_point

pytestmark = pytest.mark.gpu


def test_magnetisation_curve_point_and_mean_dipolar_field():
    r = run_point(2.0, n=500, batch=16, steps_eq=2000, steps_avg=2000, every=50, field_every=250, gamma=1.0)
    print(r)
    assert r["status_flags"] == 0
    assert abs(r["uz"] - r["langevin"]) < 0.03 + 3.0 * r["uz_sem"], r
    assert r["hz_ap"] > 0.0, r
    assert abs(r["hz_bh"] - r["hz_ap"]) <= 0.05 * abs(r["hz_ap"]), r
    assert r["field_rel_l2_bh_vs_ap"] < 0.05, r

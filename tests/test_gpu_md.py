"""md_step through the C ABI against the reference integrator (oracle/md.py): same Philox stream, same
forces, same update.  FP64: states agree to 1e-11 after several steps; FP32-mixed: the dipolar force
differs at the 1e-6 relative level, which moves the state by dt * 1e-6 per step.  Also equipartition for
a batch of non-interacting single-particle systems.  Resuming from a saved state continues the same trajectory:
the noise is bit-exact (counter-based, device step counter); the forces agree to FP64 rounding (the adjoint
reduces with FP64 atomics, whose order is not fixed)."""
import functools

import numpy as np
import pytest
import torch

from oracle import md as omd
from paper_1212_2934_amd import workloads
from paper_1212_2934_amd.binding import BarnesHut, BHError, md_params

pytestmark = pytest.mark.gpu


def _mdp(p, hext_dev):
    return md_params(p["dt"], p["kT"], p["gamma_t"], p["gamma_r"], p["mass"], p["inertia"], p["wca_eps"],
                     p["wca_sigma"], (C3 := __import__("ctypes").c_double * 3)(*p["box_lo"]), C3(*p["box_hi"]),
                     None if hext_dev is None else hext_dev.data_ptr(), p["seed"])


def _state(w, rng, B=1):
    pos = w.pos[None] if w.pos.ndim == 2 else w.pos
    mom = w.mom[None] if w.mom.ndim == 2 else w.mom
    vel = rng.standard_normal(pos.shape)
    om = rng.standard_normal(pos.shape) * np.sqrt(10.0)
    return dict(pos=pos.copy(), vel=vel, mom=mom.copy(), omega=om)


def _to_dev(st, step=0):
    d = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in st.items()}
    d["step"] = torch.tensor([step], dtype=torch.int64, device="cuda")
    return d


def _params(side, hext=(0.0, 0.0, 0.5)):
    return dict(dt=1e-3, kT=1.0, gamma_t=0.1, gamma_r=0.1, mass=1.0, inertia=0.1, wca_eps=1.0, wca_sigma=1.0,
                box_lo=(0.0, 0.0, 0.0), box_hi=(side, side, side), hext=np.array([hext]), seed=2002)


@pytest.mark.parametrize("precision,tol,tuning_id", [("fp64", 1e-11, -1), ("fp32_mixed", 1e-8, -1),
                                                     ("fp64", 1e-11, 5), ("fp32_mixed", 1e-8, 5),
                                                     ("fp64", 1e-11, 6), ("fp32_mixed", 1e-8, 7),
                                                     ("fp64", 1e-11, 9), ("fp32_mixed", 1e-8, 10)])
def test_trajectory_matches_reference(precision, tol, tuning_id):
    """tuning 5: adjoint waves of 16 targets; 6 and 7: walks split over the root's children (the
    small-system launch shapes); 9 and 10: one persistent launch ordered by the previous step's costs."""
    w = workloads.uniform_cube(1500, 20.0, seed=4)
    rng = np.random.default_rng(5)
    st = _state(w, rng)
    p = _params(20.0)
    bh = BarnesHut(w.n, 1, 16, 0.5, precision, tuning_id=tuning_id)
    d = _to_dev(st)
    he = torch.from_numpy(p["hext"]).cuda()
    mp = _mdp(p, he)
    ref = st
    for k in range(4):
        bh.md_step(d, mp)
        ref = omd.md_step(ref, p, k, theta=0.5, leaf=16)
    assert bh.check_status() == 0
    assert int(d["step"].item()) == 4
    for key in ("pos", "vel", "mom", "omega"):
        g = d[key].cpu().numpy()
        err = np.abs(g - ref[key]).max() / np.abs(ref[key]).max()
        assert err <= tol, (key, err)


@pytest.mark.parametrize("batch", [1, 3])
def test_chain_contacts_short_range_forces(batch):
    """Chains (spacing 1.05 d) put every bead's neighbours inside the WCA cut-off (2^(1/6) d), and the
    walls touch the outermost beads: two FP64 steps against the reference integrator, whose WCA term is a
    brute-force sum over all pairs.  Three realisations in a batch exercise per-system grids of different
    levels (box sides 16, 30 and 60)."""
    rng = np.random.default_rng(31)
    sides = [16.0, 30.0, 60.0][:batch] if batch > 1 else [30.0]
    n = 900
    pos, mom = [], []
    for side in sides:
        p_, m_ = workloads.rsa_chains(rng, n, (0.0, 0.0, 0.0), (side, side, side))
        pos.append(p_)
        mom.append(m_)
    st = dict(pos=np.stack(pos), vel=rng.standard_normal((batch, 3, n)), mom=np.stack(mom),
              omega=rng.standard_normal((batch, 3, n)))
    side = max(sides)
    p = _params(side)
    p["hext"] = np.tile(p["hext"], (batch, 1))
    p["box_hi"] = (side, side, side)
    bh = BarnesHut(n, batch, 16, 0.5, "fp64")
    d = _to_dev(st)
    he = torch.from_numpy(p["hext"]).cuda()
    mp = _mdp(p, he)
    ref = st
    for k in range(2):
        bh.md_step(d, mp)
        ref = omd.md_step(ref, p, k, theta=0.5, leaf=16)
    assert bh.check_status() == 0
    for key in ("pos", "vel", "mom", "omega"):
        g = d[key].cpu().numpy()
        err = np.abs(g - ref[key]).max() / np.abs(ref[key]).max()
        assert err <= 1e-11, (key, err)


@pytest.mark.parametrize("batch,sr_cut", [(1, 0.0), (3, 0.0), (3, 2.0)])
def test_paper_short_range_law(batch, sr_cut):
    """The paper's short-range force (Eq. LJ, Sec. 2; sr_kind 1): zero at sigma, attractive out to the
    cut-off (2.5 sigma by default), walls of the same law at half the cut.  Chains at spacing 1.05 d sit
    just outside the zero, so every bead feels attraction from its neighbours and repulsion-free walls
    within reach; two FP64 steps against the reference integrator's brute-force pair sum.  The longer
    cut-off coarsens the cell grid of each system (sides 16, 30 and 60)."""
    rng = np.random.default_rng(41)
    sides = [16.0, 30.0, 60.0][:batch] if batch > 1 else [20.0]
    n = 900
    pos, mom = [], []
    for side in sides:
        p_, m_ = workloads.rsa_chains(rng, n, (0.0, 0.0, 0.0), (side, side, side))
        pos.append(p_)
        mom.append(m_)
    st = dict(pos=np.stack(pos), vel=rng.standard_normal((batch, 3, n)), mom=np.stack(mom),
              omega=rng.standard_normal((batch, 3, n)))
    side = max(sides)
    p = _params(side)
    p["hext"] = np.tile(p["hext"], (batch, 1))
    p["sr_kind"], p["sr_cut"] = 1, sr_cut
    bh = BarnesHut(n, batch, 16, 0.5, "fp64")
    d = _to_dev(st)
    he = torch.from_numpy(p["hext"]).cuda()
    mp = _mdp(p, he)
    mp.sr_kind, mp.sr_cut = 1, sr_cut
    ref = st
    for k in range(2):
        bh.md_step(d, mp)
        ref = omd.md_step(ref, p, k, theta=0.5, leaf=16)
    assert bh.check_status() == 0
    for key in ("pos", "vel", "mom", "omega"):
        g = d[key].cpu().numpy()
        err = np.abs(g - ref[key]).max() / np.abs(ref[key]).max()
        assert err <= 1e-11, (key, err)


def test_short_range_law_argument_checks():
    """An unknown law or a negative or non-finite cut-off is rejected before anything is enqueued."""
    w = workloads.uniform_cube(256, 10.0, seed=3)
    st = _to_dev(_state(w, np.random.default_rng(3)))
    p = _params(10.0)
    he = torch.from_numpy(p["hext"]).cuda()
    bh = BarnesHut(w.n, 1, 16, 0.5, "fp64")
    before = {k: v.clone() for k, v in st.items()}
    for kind, cut in [(2, 0.0), (-1, 0.0), (1, -1.0), (1, float("nan")), (1, float("inf"))]:
        mp = _mdp(p, he)
        mp.sr_kind, mp.sr_cut = kind, cut
        with pytest.raises(BHError):
            bh.md_step(st, mp)
    torch.cuda.synchronize()
    for k in before:
        assert torch.equal(before[k], st[k]), k


@functools.lru_cache(maxsize=1)
def _two_systems_and_reference(steps):
    """Two systems of 8192 particles (16384 over the batch) and their reference trajectory."""
    w = workloads.uniform_cube(8192, 32.0, seed=8)
    rng = np.random.default_rng(9)
    one = _state(w, rng)
    two = _state(w, rng)
    st = {k: np.concatenate([one[k], two[k]]) for k in one}
    p = _params(32.0)
    p["hext"] = np.array([[0.0, 0.0, 0.5], [0.2, 0.0, 0.3]])
    ref = st
    for k in range(steps):
        ref = omd.md_step(ref, p, k, theta=0.5, leaf=16)
    return w.n, st, p, ref


@pytest.mark.parametrize("tuning_id", [-1, 9])
def test_steps_on_a_user_stream_are_ordered_with_it(tuning_id):
    """md_step forks part of its work onto the handle's own stream (from 16384 particles over the batch).
    On a user stream that is still busy (a chain of products) when the state is written and the steps are
    enqueued, with no host synchronisation anywhere, every step must see the state written before it and
    the copies enqueued after it must see the step complete: the result equals the reference trajectory."""
    n, st, p, ref = _two_systems_and_reference(3)
    bh = BarnesHut(n, 2, 16, 0.5, "fp64", tuning_id=tuning_id)
    src = _to_dev(st)
    d = {k: torch.zeros_like(v) for k, v in src.items()}
    he = torch.from_numpy(p["hext"]).cuda()
    mp = _mdp(p, he)
    a = torch.randn(2048, 2048, device="cuda")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for _ in range(8):  # keeps the stream busy while the host enqueues the rest
            a = torch.tanh(a @ a)
        for k in d:
            d[k].copy_(src[k])
        for _ in range(3):
            bh.md_step(d, mp)
        out = {k: v.clone() for k, v in d.items()}
    s.synchronize()
    assert int(out["step"].item()) == 3
    for key in ("pos", "vel", "mom", "omega"):
        g = out[key].cpu().numpy()
        err = np.abs(g - ref[key]).max() / np.abs(ref[key]).max()
        assert err <= 1e-11, (key, err)
    assert bh.check_status() == 0


@pytest.mark.parametrize("tuning_id", [-1, 9])
def test_caller_owned_handle_steps_without_a_side_stream(tuning_id):
    """A handle made by bh_init in caller memory has no side stream: md_step runs everything on the
    caller's stream and follows the same reference trajectory; its build and field equal a bh_create
    handle's bit for bit."""
    n, st, p, ref = _two_systems_and_reference(3)
    bh = BarnesHut(n, 2, 16, 0.5, "fp64", tuning_id=tuning_id, caller_memory=True)
    d = _to_dev(st)
    he = torch.from_numpy(p["hext"]).cuda()
    mp = _mdp(p, he)
    for _ in range(3):
        bh.md_step(d, mp)
    torch.cuda.synchronize()
    assert int(d["step"].item()) == 3
    for key in ("pos", "vel", "mom", "omega"):
        g = d[key].cpu().numpy()
        err = np.abs(g - ref[key]).max() / np.abs(ref[key]).max()
        assert err <= 1e-11, (key, err)
    assert bh.check_status() == 0
    pos = torch.from_numpy(np.ascontiguousarray(st["pos"])).cuda()
    mom = torch.from_numpy(np.ascontiguousarray(st["mom"])).cuda()
    out = []
    for caller_memory in (False, True):
        h = BarnesHut(n, 2, 16, 0.5, "fp32_mixed", caller_memory=caller_memory)
        h.build(pos)
        out.append(h.field(mom, he))
        assert h.check_status() == 0
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])


def test_resume_continues_the_same_trajectory():
    w = workloads.uniform_cube(2000, 24.0, seed=6)
    rng = np.random.default_rng(7)
    st = _state(w, rng)
    p = _params(24.0)
    he = torch.from_numpy(p["hext"]).cuda()
    a = _to_dev(st)
    bh = BarnesHut(w.n, 1, 16, 0.5, "fp64")
    for _ in range(6):
        bh.md_step(a, _mdp(p, he))
    b = _to_dev(st)
    bh1 = BarnesHut(w.n, 1, 16, 0.5, "fp64")
    for _ in range(3):
        bh1.md_step(b, _mdp(p, he))
    saved = {k: v.clone() for k, v in b.items()}
    bh2 = BarnesHut(w.n, 1, 16, 0.5, "fp64")  # a fresh handle resumes from the saved state
    for _ in range(3):
        bh2.md_step(saved, _mdp(p, he))
    # the noise stream is exact (device step counter); the forces differ only in FP64 summation order
    # (the adjoint scatters with FP64 atomics), so the states agree to rounding
    assert torch.equal(a["step"], saved["step"])
    for k in ("pos", "vel", "mom", "omega"):
        err = ((a[k] - saved[k]).abs().max() / a[k].abs().max()).item()
        assert err <= 1e-12, (k, err)


def test_batched_equipartition_single_particle_systems():
    B = 4096
    rng = np.random.default_rng(8)
    st = dict(pos=np.full((B, 3, 1), 5.0), vel=np.zeros((B, 3, 1)),
              mom=np.tile(np.array([0.0, 0.0, 1.0])[None, :, None], (B, 1, 1)), omega=np.zeros((B, 3, 1)))
    p = dict(dt=0.01, kT=1.0, gamma_t=1.0, gamma_r=1.0, mass=1.0, inertia=0.1, wca_eps=0.0, wca_sigma=1.0,
             box_lo=(0.0, 0.0, 0.0), box_hi=(10.0, 10.0, 10.0), hext=None, seed=11)
    bh = BarnesHut(1, B, 16, 0.5, "fp64")
    d = _to_dev(st)
    mp = _mdp(p, None)
    v2, w2 = [], []
    for k in range(800):
        bh.md_step(d, mp)
        if k >= 300 and k % 10 == 0:
            v2.append((d["vel"] ** 2).sum(dim=1).mean().item())
            w2.append((d["omega"] ** 2).sum(dim=1).mean().item())
    assert bh.check_status() == 0
    assert abs(np.mean(v2) / 3.0 - 1.0) < 0.05
    assert abs(np.mean(w2) / 30.0 - 1.0) < 0.15
    # one more step from rest: a lone particle away from the walls, with no field, feels only the noise,
    # so v' = sqrt(2 gamma_t kT dt) / M xi_t and w' = sqrt(2 gamma_r kT dt) / I xi_r with the reference
    # generator's normals of its system at the device's step count
    step = int(d["step"].item())
    d["vel"].zero_()
    d["omega"].zero_()
    d["pos"].fill_(5.0)
    bh.md_step(d, mp)
    assert bh.check_status() == 0
    vel, om = d["vel"].cpu().numpy(), d["omega"].cpu().numpy()
    at, ar = np.sqrt(2.0 * 0.01), np.sqrt(2.0 * 0.01) / 0.1
    for b in (0, 17, 1000, B - 1):
        xi = omd.normals(11, b, step, 1)
        np.testing.assert_allclose(vel[b, :, 0], at * xi[:3, 0], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(om[b, :, 0], ar * xi[3:, 0], rtol=1e-12, atol=1e-13)

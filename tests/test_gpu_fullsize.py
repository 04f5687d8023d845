"""Parity at the full workload sizes, in the launch configuration the benchmark times.

- 2^20 chains (phi 0.1), theta in {0.3, 0.5, 0.7}: FP32-mixed (and FP64 at 0.5) field against the oracle on
  2048 sampled targets (the oracle computes targets one by one), interaction counts equal on every sampled
  target; energy against the oracle's full evaluation at theta 0.5; at theta 0.5 also in launch shape 11,
  a persistent cost-ordered shape of the kind the benchmark's autotuner picks for the MD step.
- 2^20 chains: the MD step's fused forward + adjoint walk in launch shape 11, both precisions, two calls
  (the second ordered by the first's costs), against the oracle's full frozen-structure adjoint.
- 2^18 differentiation workload: full FP32-mixed adjoint against the oracle's frozen-structure adjoint, and
  on the 512-particle subset the GPU adjoint against central finite differences of the oracle's frozen
  energy (h = 1e-6).
- 2^17 dilute MD: 100 steps of an FP32-mixed and an FP64 trajectory; on every step the FP32-mixed state's
  field in both precisions against the oracle on sampled targets (the series is written out on request).
- 32 x 2^16 slab: 1000 graph-replayed batched steps in the autotuned launch shape flag nothing and stay
  finite; field and gradients of realisations 0 and 31 against the oracle at steps 0 and 1000.
"""
import ctypes
import os

import numpy as np
import pytest
import torch

from gpu_util import energy_err, errors, grad_check
from paper_1212_2934_amd import workloads
from paper_1212_2934_amd.binding import BarnesHut, md_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def chains():
    return workloads.cached("chains_n1048576_seed1003", lambda: workloads.config3())


def _field(w, theta, precision, counters=True, tuning_id=-1):
    bh = BarnesHut(w.n, 1, 16, theta, precision, tuning_id=tuning_id)
    pos = torch.from_numpy(w.pos).cuda()
    mom = torch.from_numpy(w.mom).cuda()
    bh.build(pos)
    cnt = bh.enable_counters() if counters else None
    H, E = bh.field(mom, torch.from_numpy(np.asarray(w.hext, float)).cuda())
    assert bh.check_status() == 0
    out = dict(H=H.cpu().numpy(), E=E.item())
    if cnt:
        out["nf"], out["nr"] = cnt[0].cpu().numpy()[0], cnt[1].cpu().numpy()[0]
    return out


@pytest.mark.parametrize("theta,precision,tuning_id", [(0.3, "fp32_mixed", -1), (0.5, "fp32_mixed", -1),
                                                       (0.7, "fp32_mixed", -1), (0.5, "fp64", -1),
                                                       (0.5, "fp32_mixed", 11), (0.5, "fp64", 11)])
def test_chains_2p20_sampled_targets(oracle_mod, chains, theta, precision, tuning_id):
    w = chains
    t = oracle_mod.Tree(w.pos, w.mom, 16)
    idx = np.sort(np.random.default_rng(int(theta * 100)).choice(w.n, 2048, replace=False))
    Href, nf, nr = t.field_subset(theta, idx)
    g = _field(w, theta, precision, tuning_id=tuning_id)
    assert (g["nf"][idx] == nf).all() and (g["nr"][idx] == nr).all()
    e = errors(g["H"][:, idx], Href)
    tol = 1e-5 if precision == "fp32_mixed" else 1e-12
    assert e["l2"] <= tol and (e["p999"] <= tol if precision == "fp32_mixed" else e["max"] <= 1e-10), e
    if theta == 0.5:
        H, _, _ = t.field(theta)
        assert energy_err(g["E"], oracle_mod.energy(w.mom, H), w.mom, H) <= tol


@pytest.fixture(scope="module")
def chains_grad(oracle_mod, chains):
    _, _, dr, dm = oracle_mod.Tree(chains.pos, chains.mom, 16).energy_grad(0.5, None)
    return dr, dm


@pytest.mark.parametrize("precision,tol", [("fp32_mixed", 1e-5), ("fp64", 1e-12)])
def test_chains_2p20_md_adjoint_bench_shape(chains, chains_grad, precision, tol):
    w = chains
    dr, dm = chains_grad
    bh = BarnesHut(w.n, 1, 16, 0.5, precision, tuning_id=11)
    bh.build(torch.from_numpy(w.pos).cuda())
    mom = torch.from_numpy(w.mom).cuda()
    for call in range(2):
        gdr, gdm = bh.field_backward(mom, None, gE=torch.ones(1, dtype=torch.float64, device="cuda"))
        assert bh.check_status() == 0
        gdr, gdm = gdr.cpu().numpy(), gdm.cpu().numpy()
        grad_check(gdr, dr, precision, f"dE/dr chains 2^20 call {call}")
        grad_check(gdm, dm, precision, f"dE/dm chains 2^20 call {call}")


def test_differentiation_2p18_full_adjoint(oracle_mod):
    w = workloads.config4()
    _, _, dr, dm = oracle_mod.Tree(w.pos, w.mom, 16).energy_grad(0.5, w.hext)
    bh = BarnesHut(w.n, 1, 16, 0.5, "fp32_mixed")
    bh.build(torch.from_numpy(w.pos).cuda())
    gdr, gdm = bh.field_backward(torch.from_numpy(w.mom).cuda(), torch.from_numpy(w.hext).cuda(),
                                 gE=torch.ones(1, dtype=torch.float64, device="cuda"))
    assert bh.check_status() == 0
    gdr, gdm = gdr.cpu().numpy(), gdm.cpu().numpy()
    grad_check(gdr, dr, "fp32_mixed", "dE/dr uniform 2^18")
    grad_check(gdm, dm, "fp32_mixed", "dE/dm uniform 2^18")


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-7), ("fp32_mixed", 1e-5)])
def test_differentiation_subset_against_finite_differences(oracle_mod, precision, tol):
    w = workloads.config4()
    idx = workloads.nearest_to_centre(w.pos, 512)
    pos, mom = w.pos[:, idx].copy(), w.mom[:, idx].copy()
    st = oracle_mod.frozen_structure(oracle_mod.Tree(pos, mom, 16), 0.5)
    fr, fm = oracle_mod.fd_grad_frozen(pos, mom, w.hext, st, 1e-6)
    bh = BarnesHut(512, 1, 16, 0.5, precision)
    bh.build(torch.from_numpy(pos).cuda())
    gdr, gdm = bh.field_backward(torch.from_numpy(mom).cuda(), torch.from_numpy(w.hext).cuda(),
                                 gE=torch.ones(1, dtype=torch.float64, device="cuda"))
    gdr, gdm = gdr.cpu().numpy(), gdm.cpu().numpy()
    assert np.linalg.norm(gdr - fr) / np.linalg.norm(fr) <= tol
    assert np.linalg.norm(gdm - fm) / np.linalg.norm(fm) <= tol


def _series_out(name, text):
    """Write a measured series when FFBH_SERIES_DIR names a folder (the profiles are made this way)."""
    d = os.environ.get("FFBH_SERIES_DIR")
    if d:
        os.makedirs(d, exist_ok=True)
        with open(os.path.join(d, name), "w") as f:
            f.write(text)


def _md_state(w, rng, batch_shape):
    return {"pos": torch.from_numpy(w.pos.reshape(batch_shape).copy()).cuda(),
            "vel": torch.from_numpy(rng.standard_normal(batch_shape)).cuda(),
            "mom": torch.from_numpy(w.mom.reshape(batch_shape).copy()).cuda(),
            "omega": torch.from_numpy(rng.standard_normal(batch_shape) * np.sqrt(10.0)).cuda(),
            "step": torch.zeros(1, dtype=torch.int64, device="cuda")}


def test_dilute_md_2p17_100_steps_both_precisions(oracle_mod):
    """Dilute MD workload: 100 steps (dt 1e-3, kT 1, H_ext (0, 0, 0.5)) of an FP32-mixed and an FP64
    trajectory from the same state with the same noise.  On every step the FP32-mixed trajectory's state is
    evaluated by the FP32-mixed field, by the FP64 field and by the oracle (1024 sampled targets): FP32-mixed
    within 1e-5 (relative L2 and 99.9th percentile), FP64 within 1e-12 (relative L2) and 1e-10 (every
    target).  The distance between the two trajectories is reported."""
    w = workloads.config2()
    rng = np.random.default_rng(2002)
    side = float(w.box_hi[0])
    s32 = _md_state(w, rng, (1, 3, w.n))
    s64 = {k: v.clone() for k, v in s32.items()}
    hext = torch.from_numpy(np.array([w.hext])).cuda()
    C3 = ctypes.c_double * 3
    mdp = md_params(1e-3, 1.0, 0.1, 0.1, 1.0, 0.1, 1.0, 1.0, C3(0, 0, 0), C3(side, side, side), hext.data_ptr(), 2002)
    md32 = BarnesHut(w.n, 1, 16, 0.5, "fp32_mixed")
    md64 = BarnesHut(w.n, 1, 16, 0.5, "fp64")
    p32 = BarnesHut(w.n, 1, 16, 0.5, "fp32_mixed")
    p64 = BarnesHut(w.n, 1, 16, 0.5, "fp64")
    idx = np.sort(np.random.default_rng(7).choice(w.n, 1024, replace=False))
    rows = []
    for step in range(101):
        pos = s32["pos"][0].contiguous()
        mom = s32["mom"][0].contiguous()
        p32.build(pos)
        H32 = p32.field(mom, energy=False).cpu().numpy()
        p64.build(pos)
        H64 = p64.field(mom, energy=False).cpu().numpy()
        pn, mn = pos.cpu().numpy(), mom.cpu().numpy()
        Href, _, _ = oracle_mod.Tree(pn, mn, 16).field_subset(0.5, idx)
        e32 = errors(H32[:, idx], Href)
        e64 = errors(H64[:, idx], Href)
        dtraj = (s32["pos"] - s64["pos"]).abs().max().item()
        rows.append((step, e32, e64, dtraj))
        assert e32["l2"] <= 1e-5 and e32["p999"] <= 1e-5, (step, e32)
        assert e64["l2"] <= 1e-12 and e64["max"] <= 1e-10, (step, e64)
        if step < 100:
            md32.md_step(s32, mdp)
            md64.md_step(s64, mdp)
    assert md32.check_status() == 0 and md64.check_status() == 0
    assert p32.check_status() == 0 and p64.check_status() == 0
    w32 = max(r[1]["l2"] for r in rows)
    print(f"[dilute MD] 100 steps: worst FP32-mixed field error {w32:.2e}, worst FP64 "
          f"{max(r[2]['l2'] for r in rows):.2e}, trajectories apart by {rows[-1][3]:.2e}")
    lines = ["| step | FP32-mixed rel. L2 | FP32-mixed p99.9 | FP32-mixed max | FP64 rel. L2 | FP64 max | "
             "max abs(r_FP32 - r_FP64) |", "|---|---|---|---|---|---|---|"]
    lines += [f"| {st} | {a['l2']:.2e} | {a['p999']:.2e} | {a['max']:.2e} | {b['l2']:.2e} | {b['max']:.2e} | "
              f"{d:.2e} |" for st, a, b, d in rows]
    _series_out("dilute_md_n131072_100_steps.md", "\n".join(lines) + "\n")


@pytest.fixture(scope="module")
def slab():
    return workloads.cached("slab_b32_n65536_seed1005", lambda: workloads.config5())


def _slab_checks(oracle_mod, w, state, tag, precision="fp32_mixed"):
    """Field (1024 sampled targets) and the full energy gradient of realisations 0 and 31 of a batched state
    against the oracle."""
    pos = state["pos"].contiguous()
    mom = state["mom"].contiguous()
    hext = torch.from_numpy(w.hext).cuda()
    bh = BarnesHut(w.n, w.batch, 16, 0.5, precision)
    bh.build(pos)
    H, _ = bh.field(mom, hext)
    dr, dm = bh.field_backward(mom, hext, gE=torch.ones(w.batch, dtype=torch.float64, device="cuda"))
    assert bh.check_status() == 0
    H, dr, dm = H.cpu().numpy(), dr.cpu().numpy(), dm.cpu().numpy()
    pn, mn = pos.cpu().numpy(), mom.cpu().numpy()
    for b in (0, 31):
        t = oracle_mod.Tree(pn[b], mn[b], 16)
        idx = np.sort(np.random.default_rng(b).choice(w.n, 1024, replace=False))
        Href, _, _ = t.field_subset(0.5, idx)
        e = errors(H[b][:, idx], Href)
        assert e["l2"] <= 1e-5 and e["p999"] <= 1e-5, (tag, b, e)
        _, _, gr, gm = t.energy_grad(0.5, w.hext[b])
        grad_check(dr[b], gr, precision, f"slab {tag} realisation {b} dE/dr")
        grad_check(dm[b], gm, precision, f"slab {tag} realisation {b} dE/dm")


def test_slab_batch_1000_steps(oracle_mod, slab):
    """Batched slab: 32 realisations of 2^16, 1000 graph-replayed FP32-mixed MD steps in the launch shape
    the autotuner picks for these MD steps; the status word is read every 100 steps and must stay clear;
    the state stays finite, inside the slab, with unit moments; field and gradients of realisations 0 and
    31 against the oracle at steps 0 and 1000."""
    from paper_1212_2934_amd.autotune import autotune
    w = slab
    rng = np.random.default_rng(2005)
    hext = torch.from_numpy(w.hext).cuda()
    C3 = ctypes.c_double * 3
    mdp = md_params(1e-3, 1.0, 0.1, 0.1, 1.0, 0.1, 1.0, 1.0, C3(*w.box_lo), C3(*w.box_hi), hext.data_ptr(), 2005)
    state = _md_state(w, rng, w.pos.shape)
    _slab_checks(oracle_mod, w, state, "step 0")
    tune = autotune(state["pos"], state["mom"], hext, precision="fp32_mixed", md=(state, mdp))
    print(f"[slab] autotuned shape {tune['tuning_id']}", flush=True)
    g = BarnesHut(w.n, w.batch, 16, 0.5, "fp32_mixed", tuning_id=tune["tuning_id"])
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = g.capture_md_graph(state, mdp, s)
    for block in range(10):
        for _ in range(100):
            graph.launch(s)
        s.synchronize()
        with torch.cuda.stream(s):
            flags = g.check_status()
        assert flags == 0, (block, flags)
    assert int(state["step"].item()) == 1000
    for k in ("pos", "vel", "mom", "omega"):
        assert torch.isfinite(state[k]).all()
    p = state["pos"]
    assert (p[:, 2] > -0.5).all() and (p[:, 2] < 8.5).all()
    assert ((state["mom"].norm(dim=1) - 1.0).abs() < 1e-12).all()
    _slab_checks(oracle_mod, w, state, "step 1000")

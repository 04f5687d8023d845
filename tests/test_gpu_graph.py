"""Batched MD replayed from a captured HIP graph against eager md_step calls, and the autotuner's
result-invariance rule.  Each graph replay is followed by eager work and a synchronisation, and every
replay is checked against the eager trajectory (to FP64 rounding: the adjoint reduces with atomics)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1212_2934_amd import autotune, workloads
from paper_1212_2934_amd.binding import BarnesHut, md_params

pytestmark = pytest.mark.gpu


def _mdp(box_lo, box_hi, hext_dev, seed=2005):
    C3 = ctypes.c_double * 3
    return md_params(1e-3, 1.0, 0.1, 0.1, 1.0, 0.1, 1.0, 1.0, C3(*box_lo), C3(*box_hi),
                     None if hext_dev is None else hext_dev.data_ptr(), seed)


def _state(pos, mom, seed):
    rng = np.random.default_rng(seed)
    d = dict(pos=pos, vel=rng.standard_normal(pos.shape), mom=mom, omega=rng.standard_normal(pos.shape) * 3.0)
    out = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in d.items()}
    out["step"] = torch.zeros(1, dtype=torch.int64, device="cuda")
    return out


def _close(a, b, tol=1e-12):
    for k in ("pos", "vel", "mom", "omega"):
        err = ((a[k] - b[k]).abs().max() / b[k].abs().max()).item()
        assert err <= tol, (k, err)
    assert torch.equal(a["step"], b["step"])


@pytest.mark.parametrize("precision,tuning_id,caller_memory", [("fp64", -1, False), ("fp32_mixed", -1, False),
                                                               ("fp32_mixed", 10, False), ("fp32_mixed", 10, True)])
def test_batched_slab_graph_replay_matches_eager(precision, tuning_id, caller_memory):
    """tuning 10: the persistent adjoint launch, whose item order comes from the previous replay's costs
    (ordering kernel and work-counter reset inside the graph).  caller_memory: handles made by bh_init,
    whose steps (and so the captured graph) use no side stream."""
    w = workloads.config5(batch=4, n=4096, box=(64.0, 64.0, 8.0))
    hext = torch.from_numpy(w.hext).cuda()
    mdp = _mdp(w.box_lo, w.box_hi, hext)
    s0 = _state(w.pos, w.mom, 5)
    eager = {k: v.clone() for k, v in s0.items()}
    bh = BarnesHut(w.n, w.batch, 16, 0.5, precision, tuning_id=tuning_id, caller_memory=caller_memory)
    snaps = []
    for _ in range(4):
        bh.md_step(eager, mdp)
        snaps.append({k: v.clone() for k, v in eager.items()})
    torch.cuda.synchronize()

    g_state = {k: v.clone() for k, v in s0.items()}
    bh2 = BarnesHut(w.n, w.batch, 16, 0.5, precision, tuning_id=tuning_id, caller_memory=caller_memory)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = bh2.capture_md_graph(g_state, mdp, stream)
    assert int(g_state["step"].item()) == 0  # capture does not execute
    for k in range(4):
        graph.launch(stream)
        stream.synchronize()
        _ = [float(v.double().norm()) for v in g_state.values()]  # eager work between replays
        torch.cuda.synchronize()
        _close(g_state, snaps[k])
    assert bh2.check_status() == 0


def test_autotune_candidates_are_result_invariant(tmp_path):
    w = workloads.config3(seed=5, n=20000)
    pos = torch.from_numpy(w.pos).cuda()
    mom = torch.from_numpy(w.mom).cuda()
    cache = str(tmp_path / "tune.json")
    r = autotune.autotune(pos, mom, None, 0.5, 16, "fp32_mixed", repeats=2, cache_path=cache)
    from paper_1212_2934_amd.binding import lib
    assert set(r["times_ms"]) == set(range(int(lib().bh_num_tunings())))
    r2 = autotune.autotune(pos, mom, None, 0.5, 16, "fp32_mixed", cache_path=cache)
    assert r2["tuning_id"] == r["tuning_id"]


@pytest.mark.parametrize("precision,tuning_id", [("fp64", -1), ("fp32_mixed", 11)])
def test_build_field_backward_captured_by_the_caller(precision, tuning_id):
    """bh_build, bh_field and bh_field_backward captured by the caller (torch's graph capture) and replayed
    on new inputs.  At 20000 particles the build forks the handle's own stream and joins it again, which
    become edges of the graph; tuning 11 adds the persistent adjoint launch with its ordering kernel.
    Every replay equals eager calls on a second handle: the field and energy bit for bit, the gradients to
    FP64 rounding (the adjoint's node sums are atomic)."""
    n = 20000
    w = workloads.config3(seed=151, n=n)
    pos = torch.from_numpy(w.pos).cuda()
    mom = torch.from_numpy(w.mom).cuda()
    gE = torch.ones(1, dtype=torch.float64, device="cuda")
    bh = BarnesHut(n, 1, 16, 0.5, precision, tuning_id=tuning_id)
    ref = BarnesHut(n, 1, 16, 0.5, precision, tuning_id=tuning_id)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # one eager pass before the capture
        bh.build(pos)
        bh.field(mom)
        bh.field_backward(mom, gE=gE)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        bh.build(pos)
        H, E = bh.field(mom)
        dpos, dmom = bh.field_backward(mom, gE=gE)
    for r in range(3):
        w2 = workloads.config3(seed=160 + r, n=n)
        pos.copy_(torch.from_numpy(w2.pos))
        mom.copy_(torch.from_numpy(w2.mom))
        graph.replay()
        torch.cuda.synchronize()
        ref.build(pos)
        Hr, Er = ref.field(mom)
        dpr, dmr = ref.field_backward(mom, gE=gE)
        torch.cuda.synchronize()
        assert torch.equal(H, Hr) and torch.equal(E, Er), r
        for a, b in ((dpos, dpr), (dmom, dmr)):
            err = ((a - b).abs().max() / b.abs().max()).item()
            assert err <= 1e-12, (r, err)
    assert bh.check_status() == 0 and ref.check_status() == 0


def test_autotune_field_mode_has_its_own_cache_entry(tmp_path):
    """field=True times build + field only and is cached under its own key beside the default mode's."""
    import json
    w = workloads.config3(seed=6, n=20000)
    pos = torch.from_numpy(w.pos).cuda()
    mom = torch.from_numpy(w.mom).cuda()
    cache = str(tmp_path / "tune.json")
    a = autotune.autotune(pos, mom, None, 0.5, 16, "fp32_mixed", repeats=2, cache_path=cache)
    f = autotune.autotune(pos, mom, None, 0.5, 16, "fp32_mixed", repeats=2, cache_path=cache, field=True)
    from paper_1212_2934_amd.binding import lib
    assert set(f["times_ms"]) == set(range(int(lib().bh_num_tunings())))
    assert f["key"] != a["key"] and f["key"].endswith("|field")
    with open(cache) as fh:
        assert set(json.load(fh)) == {a["key"], f["key"]}
    with pytest.raises(ValueError):
        autotune.autotune(pos, mom, None, 0.5, 16, "fp32_mixed", md=({}, None), field=True)

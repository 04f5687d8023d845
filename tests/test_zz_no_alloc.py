"""bh_field_noalloc (build + field in a fixed device array, no allocation) against bh_create + bh_build +
bh_field on the same inputs.

Both run the same kernels on the same tree, and the forward field and energy do not depend on the launch
order (every target's sum is taken in one fixed order, the energy reduction is deterministic), so the
results must agree bit for bit, in both precisions.  Two calls in a row, the second on a smaller input,
check that nothing the first call left in the shared array leaks into the second; a third call at the
largest size the array holds and a rejected call just above it check the size limit.  The oracle pins the
handle path's values elsewhere; here it checks the largest call, which no other test covers in this form.
"""
import numpy as np
import pytest
import torch

from paper_1212_2934_amd import binding, workloads
from paper_1212_2934_amd.binding import BarnesHut

from gpu_util import errors

TOL = {"fp64": 1e-12, "fp32_mixed": 1e-5}


def _handle_path(pos, mom, hext, precision, theta=0.5):
    B, _, n = pos.shape
    bh = BarnesHut(n, B, 16, theta, precision)
    bh.build(pos)
    H, E = bh.field(mom, hext)
    assert bh.check_status() == 0
    return H, E


def _batch(n, batch, seed, side, hext):
    pos = np.empty((batch, 3, n))
    mom = np.empty((batch, 3, n))
    for b in range(batch):
        w = workloads.uniform_cube(n, side, seed + b, hext=hext)
        pos[b], mom[b] = w.pos, w.mom
    he = np.tile(np.asarray(hext, float), (batch, 1))
    return (torch.from_numpy(pos).cuda(), torch.from_numpy(mom).cuda(), torch.from_numpy(he).cuda())


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_noalloc_equals_handle_path_twice(precision):
    torch.cuda.set_device(0)
    # first call: two systems of 5000 (ragged against the 64-target waves and the sort tiles)
    pos, mom, he = _batch(5000, 2, 71, 30.0, (0.0, 0.0, 0.5))
    print(f"[noalloc] {precision} call 1: batch 2 x 5000", flush=True)
    H1, E1, F1 = binding.field_noalloc(pos, mom, he, precision=precision)
    Hr, Er = _handle_path(pos, mom, he, precision)
    torch.cuda.synchronize()
    assert int(F1.item()) == 0
    assert torch.equal(H1, Hr)
    assert torch.equal(E1, Er)
    # second call, smaller: one system of 1500, no external field
    pos2, mom2, _ = _batch(1500, 1, 91, 20.0, (0.0, 0.0, 0.0))
    print(f"[noalloc] {precision} call 2: batch 1 x 1500", flush=True)
    H2, E2, F2 = binding.field_noalloc(pos2[0], mom2[0], None, precision=precision)
    Hr2, Er2 = _handle_path(pos2, mom2, None, precision)
    torch.cuda.synchronize()
    assert int(F2.item()) == 0
    assert H2.shape == (3, 1500)
    assert torch.equal(H2, Hr2[0])
    assert torch.equal(E2, Er2)


@pytest.mark.gpu
def test_noalloc_largest_size_and_limit(oracle_mod):
    torch.cuda.set_device(0)
    n = 1 << 16
    params = binding.make_params(n, 1, 16, 0.5, "fp32_mixed")
    assert binding.workspace_bytes(params) <= 64 << 20
    w = workloads.uniform_cube(n, workloads.cube_side(n, 0.05), 1006, hext=(0.0, 0.0, 1.0))
    pos = torch.from_numpy(w.pos).cuda()
    mom = torch.from_numpy(w.mom).cuda()
    he = torch.from_numpy(w.hext).cuda()
    print(f"[noalloc] largest call: 1 x {n}", flush=True)
    H, E, F = binding.field_noalloc(pos, mom, he, precision="fp32_mixed")
    torch.cuda.synchronize()
    assert int(F.item()) == 0
    # sampled targets against the oracle's tree walk (the field of each is computed one by one)
    idx = np.random.default_rng(5).choice(n, 2048, replace=False).astype(np.int64)
    Href, _, _ = oracle_mod.Tree(w.pos, w.mom, 16).field_subset(0.5, idx)
    e = errors(H.cpu().numpy()[:, idx], Href)
    assert e["l2"] <= TOL["fp32_mixed"] and e["p999"] <= TOL["fp32_mixed"], e
    # twice as many particles: refused before anything is enqueued
    big = torch.empty(1, 3, 2 * n, dtype=torch.float64, device="cuda")
    with pytest.raises(binding.BHError) as ex:
        binding.field_noalloc(big, big, None, precision="fp32_mixed")
    assert ex.value.status == binding.BH_EWORKSPACE


def test_noalloc_rejects_oversize_on_host():
    # the size check comes before any pointer check or HIP call, so it needs no device
    import ctypes as C
    params = binding.make_params(1 << 17, 1, 16, 0.5, "fp64")
    assert binding.workspace_bytes(params) > 64 << 20
    st = binding.lib().bh_field_noalloc(C.byref(params), None, None, None, None, None, None, None)
    assert st == binding.BH_EWORKSPACE
    params = binding.make_params(0, 1, 16, 0.5, "fp64")
    assert binding.lib().bh_field_noalloc(C.byref(params), None, None, None, None, None, None, None) == \
        binding.BH_EINVAL


@pytest.mark.gpu
def test_noalloc_replayed_from_a_graph():
    """The entry point captured in a graph (it allocates nothing and records no memset) and replayed on
    new inputs written into the captured buffers: every replay, with eager work and a synchronisation
    between replays, equals the handle path on the same inputs bit for bit."""
    torch.cuda.set_device(0)
    B, n = 2, 3000
    pos, mom, he = _batch(n, B, 131, 26.0, (0.0, 0.0, 0.5))
    H = torch.empty_like(pos)
    E = torch.empty(B, dtype=torch.float64, device="cuda")
    F = torch.zeros(1, dtype=torch.int32, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # one eager call first (the device's array address is looked up once)
        binding.field_noalloc(pos, mom, he, precision="fp32_mixed", out=(H, E, F))
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    print("[noalloc] capture: batch 2 x 3000", flush=True)
    with torch.cuda.graph(graph):
        binding.field_noalloc(pos, mom, he, precision="fp32_mixed", out=(H, E, F))
    for r in range(3):
        p2, m2, _ = _batch(n, B, 140 + r, 26.0, (0.0, 0.0, 0.5))
        pos.copy_(p2)
        mom.copy_(m2)
        print(f"[noalloc] replay {r}", flush=True)
        graph.replay()
        torch.cuda.synchronize()
        Hr, Er = _handle_path(p2, m2, he, "fp32_mixed")
        torch.cuda.synchronize()
        assert int(F.item()) == 0
        assert torch.equal(H, Hr), r
        assert torch.equal(E, Er), r

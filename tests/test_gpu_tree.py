"""GPU tree against the oracle's tree: same sorted order (bitwise), same cells (each run of unary cells
of the oracle's uncollapsed tree appears once on the GPU, at its deepest cell; leaves at the first cell of
their run), same geometric centres (bitwise: same sums in the same order, Eq. magCenter)."""
import numpy as np
import pytest

from paper_1212_2934_amd import workloads
from gpu_util import run_field

pytestmark = pytest.mark.gpu


def _oracle_cells(t):
    keep = {}
    for i in range(t["level"].size):
        if t["nchild"][i] != 1:
            keep[(int(t["first"][i]), int(t["count"][i]))] = (int(t["level"][i]), t["c"][i],
                                                              int(t["nchild"][i]) == 0)
    return keep


def _compare(pos, mom, leaf, oracle_mod, offset=0, gtree=None):
    t = oracle_mod.Tree(pos, mom, leaf).export()
    n = pos.shape[1]
    assert (gtree["perm"][offset:offset + n] - offset == t["perm"]).all()
    ocells = _oracle_cells(t)
    gcells = {}
    for i in range(gtree["first"].size):
        f = int(gtree["first"][i]) - offset
        if 0 <= f < n and f + int(gtree["count"][i]) <= n:
            gcells[(f, int(gtree["count"][i]))] = (int(gtree["level"][i]), gtree["centroid"][i],
                                                   int(gtree["nchild"][i]) == 0)
    assert set(gcells) == set(ocells)
    for k, (lev, c, leafy) in ocells.items():
        glev, gc, gleafy = gcells[k]
        assert glev == lev and gleafy == leafy, k
        assert (gc == c).all(), (k, gc, c)
    return len(ocells)


@pytest.mark.parametrize("n,side,leaf,seed", [(4096, 32.0, 16, 1001), (5000, 36.0, 4, 7),
                                             (777, 20.0, 1, 8), (20000 + 37, 60.0, 16, 9),
                                             (32000 + 11, 80.0, 16, 10), (40000 + 3, 85.0, 16, 11)])
def test_tree_matches_oracle(oracle_mod, n, side, leaf, seed):
    w = workloads.uniform_cube(n, side, seed)
    out = run_field(w.pos, w.mom, leaf=leaf, counters=False)
    assert out["flags"] == 0
    g = out["bh"].export_tree()
    ncells = _compare(w.pos, w.mom, leaf, oracle_mod, gtree=g)
    assert ncells == g["first"].size


def test_tree_chains_and_batch(oracle_mod):
    ws = [workloads.config3(seed=100 + b, n=3000) for b in range(3)]
    pos = np.stack([w.pos for w in ws])
    mom = np.stack([w.mom for w in ws])
    out = run_field(pos, mom, counters=False)
    g = out["bh"].export_tree()
    total = 0
    for b, w in enumerate(ws):
        total += _compare(w.pos, w.mom, 16, oracle_mod, offset=b * 3000, gtree=g)
    assert total == g["first"].size
    assert (g["first"][:3] == np.array([0, 3000, 6000])).all()  # roots are nodes 0..B-1


@pytest.mark.parametrize("n", [1, 2, 3, 16, 17, 64, 65])
def test_tree_small_systems(oracle_mod, n):
    w = workloads.uniform_cube(n, 6.0 + n ** (1 / 3), seed=n)
    out = run_field(w.pos, w.mom, leaf=16, counters=False)
    g = out["bh"].export_tree()
    _compare(w.pos, w.mom, 16, oracle_mod, gtree=g)


def test_tree_dense_cluster_in_a_large_tree(oracle_mod):
    """A tree of more than 2^16 nodes whose cells below level 10 are populated: 2000 of 40000 particles
    packed in a cube 0.01 wide, so cells of levels 10 to about 16 hold more than a leaf.  Those levels
    take the one-workgroup upward launch; their centres must still equal the oracle's bitwise."""
    rng = np.random.default_rng(12)
    w = workloads.uniform_cube(38000, 85.0, seed=12)
    cluster = np.array([[40.0], [41.0], [42.0]]) + 0.01 * rng.random((3, 2000))
    pos = np.concatenate([w.pos, cluster], axis=1)
    mom = np.concatenate([w.mom, workloads.uniform_cube(2000, 85.0, seed=13).mom], axis=1)
    t = oracle_mod.Tree(pos, mom, 16).export()
    assert t["level"].max() >= 14 and (t["level"] >= 10).sum() > 100  # the deep levels are populated
    out = run_field(pos, mom, leaf=16, counters=False)
    assert out["flags"] == 0
    g = out["bh"].export_tree()
    assert g["first"].size > 0
    ncells = _compare(pos, mom, 16, oracle_mod, gtree=g)
    assert ncells == g["first"].size


def test_sort_order_with_runs_of_equal_upper_code_bits(oracle_mod):
    """The tiled sort orders the codes by their bits above the low 32 and then orders each run of equal
    upper bits by the low bits: short runs by insertion, runs of more than 32 by a merge.  Clusters of 24
    and of 80 particles 1e-4 wide (runs of 24 and 80 equal upper parts whose low bits are out of index
    order) and 300 particles at one point (all 63 bits equal: ties stay in index order), inside 6000
    uniform ones: the order must be the oracle's, bit for bit."""
    rng = np.random.default_rng(21)
    w = workloads.uniform_cube(6000, 50.0, seed=21)
    parts = [w.pos]
    for cnt, c in [(24, 11.0), (80, 23.0)]:
        parts.append(np.array([[c], [c + 1.0], [c + 2.0]]) + 1e-4 * rng.random((3, cnt)))
    parts.append(np.tile(np.array([[31.5], [7.25], [19.75]]), (1, 300)))
    pos = np.concatenate(parts, axis=1)
    # interleave the clusters with the uniform particles so that index order and code order differ
    order = rng.permutation(pos.shape[1])
    pos = np.ascontiguousarray(pos[:, order])
    mom = workloads.uniform_cube(pos.shape[1], 50.0, seed=22).mom
    t = oracle_mod.Tree(pos, mom, 16).export()
    out = run_field(pos, mom, leaf=16, counters=False)
    g = out["bh"].export_tree()
    assert (g["perm"] == t["perm"]).all()


@pytest.mark.parametrize("n", [2000, 2048, 2049])
def test_tree_batch_around_the_one_workgroup_sort(oracle_mod, n):
    """Systems of at most 2048 particles sort in one workgroup each (all passes in LDS); 2049 takes the
    multi-workgroup passes.  Both must give the oracle's order and cells for every system of a batch."""
    ws = [workloads.config3(seed=200 + b, n=n) for b in range(3)]
    pos = np.stack([w.pos for w in ws])
    mom = np.stack([w.mom for w in ws])
    out = run_field(pos, mom, counters=False)
    assert out["flags"] == 0
    g = out["bh"].export_tree()
    total = 0
    for b, w in enumerate(ws):
        total += _compare(w.pos, w.mom, 16, oracle_mod, offset=b * n, gtree=g)
    assert total == g["first"].size


def _compare_arrays(pos, mom, leaf, oracle_mod, gtree):
    """_compare for one large system, vectorised: the cells are matched by (first, count) after sorting."""
    t = oracle_mod.Tree(pos, mom, leaf).export()
    assert (gtree["perm"] == t["perm"]).all()
    keep = t["nchild"] != 1
    okey = t["first"][keep].astype(np.int64) * (1 << 32) + t["count"][keep]
    oo = np.argsort(okey)
    gkey = gtree["first"].astype(np.int64) * (1 << 32) + gtree["count"]
    go = np.argsort(gkey)
    assert okey.size == gkey.size
    assert (okey[oo] == gkey[go]).all()
    assert (t["level"][keep][oo] == gtree["level"][go]).all()
    assert ((t["nchild"][keep][oo] == 0) == (gtree["nchild"][go] == 0)).all()
    assert (t["c"][keep][oo] == gtree["centroid"][go]).all()  # bitwise
    return okey.size


@pytest.mark.parametrize("which", ["uniform_2p17", "chains_2p20", "uniform_1310727"])
def test_tree_full_size_bitwise(oracle_mod, which):
    """Radix-sort tiles of several keys per thread: two at 2^17 particles and sixteen at 2^20, both with
    256 tiles per system, the most for which the scatter derives its offsets from the raw tile counts;
    1310727 particles need 321 tiles and take the device-wide scan instead.  The sorted order, the cells
    and their centres must equal the oracle's bit for bit."""
    if which == "uniform_2p17":
        w = workloads.config2()
    elif which == "chains_2p20":
        w = workloads.cached("chains_n1048576_seed1003", lambda: workloads.config3())
    else:
        n = 1310727
        w = workloads.cached("uniform_n1310727_phi0.05",
                             lambda: workloads.uniform_cube(n, workloads.cube_side(n, 0.05), 1007))
    print(f"[tree] {which}: n {w.n}", flush=True)
    out = run_field(w.pos, w.mom, leaf=16, counters=False)
    assert out["flags"] == 0
    g = out["bh"].export_tree()
    ncells = _compare_arrays(w.pos, w.mom, 16, oracle_mod, g)
    assert ncells == g["first"].size


def test_exported_bounding_cubes_of_a_large_batch(oracle_mod):
    """Every system's bounding cube (lo, side, scale) is exported, also beyond the 64th of a batch, and
    equals the oracle's bit for bit (componentwise min and max, one IEEE division)."""
    B, n = 70, 50
    ws = [workloads.uniform_cube(n, 8.0 + 0.05 * b, seed=300 + b) for b in range(B)]
    pos = np.stack([w.pos for w in ws])
    mom = np.stack([w.mom for w in ws])
    out = run_field(pos, mom, counters=False)
    assert out["flags"] == 0
    g = out["bh"].export_tree()
    assert g["bbox"].shape == (B, 5)
    for b, w in enumerate(ws):
        ref = oracle_mod.Tree(w.pos, w.mom, 16).export()["bbox"]
        assert (g["bbox"][b] == ref).all(), (b, g["bbox"][b], ref)

"""Seeded synthetic inputs for the Barnes-Hut dipolar-field path.

This module only draws inputs (positions, unit moments, external fields, MD initial velocities); it holds
none of the method's arithmetic, so both the GPU library's tests and the CPU oracle can consume its output.

Geometry follows the paper's model (Sec. 2): identical hard spheres of diameter d = 1 (reduced units,
R = 1/2), unit moments |m| = 1, volume fraction phi = (4/3) pi R^3 N / V (Eq. phi, Sec. 5).  Centres are
kept at least d/2 from every face of the container so that a wall potential acting at the centre-to-face
distance starts in its repulsive-free region.

Placement is random sequential addition with minimum separation d: candidates are drawn uniformly,
rejected if closer than d to an accepted particle, and conflicts among a batch of candidates are
resolved greedily in draw order (a candidate is accepted iff no earlier accepted candidate is closer than
d).  Chains (the aggregated workload) are rigid straight runs of beads treated as one candidate.

Arrays are float64 structure-of-arrays, shape (3, N) (row 0 = x, row 1 = y, row 2 = z); batches are
(B, 3, N).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.spatial import cKDTree

D = 1.0  # hard-sphere diameter (reduced length unit)


def cube_side(n: int, phi: float) -> float:
    """Side L of a cube holding n spheres of diameter 1 at volume fraction phi (Eq. phi, R = 1/2)."""
    return (n * math.pi / 6.0 / phi) ** (1.0 / 3.0)


def unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    """n unit vectors uniform on the sphere (normalised Gaussian triples), shape (3, n)."""
    g = rng.standard_normal((3, n))
    return g / np.linalg.norm(g, axis=0, keepdims=True)


def _greedy(n_cand: int, pairs: np.ndarray) -> np.ndarray:
    """Sequential greedy acceptance over a conflict graph, vectorised as a fixed point.

    Candidate i is accepted iff no accepted candidate j < i conflicts with it.  ``pairs`` holds (j, i)
    with j < i.  Returns a boolean mask.
    """
    status = np.zeros(n_cand, np.int8)  # 0 undecided, 1 accepted, 2 rejected
    if pairs.size == 0:
        return np.ones(n_cand, bool)
    lo, hi = pairs[:, 0], pairs[:, 1]
    while True:
        und = status == 0
        if not und.any():
            break
        # reject candidates that conflict with an accepted earlier one
        rej = hi[status[lo] == 1]
        status[rej[status[rej] == 0]] = 2
        # accept candidates whose earlier partners are all rejected
        live = status[lo] != 2
        cnt = np.bincount(hi[live], minlength=n_cand)
        acc = (status == 0) & (cnt == 0)
        status[acc] = 1
    return status == 1


def _ordered_pairs(points: np.ndarray, r: float) -> np.ndarray:
    p = cKDTree(points).query_pairs(r, output_type="ndarray")
    if p.size == 0:
        return np.zeros((0, 2), np.int64)
    return np.sort(p, axis=1)


def rsa_uniform(rng: np.random.Generator, n: int, lo, hi, margin: float = 0.5,
                min_sep: float = D) -> np.ndarray:
    """Random sequential addition of n centres in the box [lo+margin, hi-margin], shape (3, n)."""
    lo = np.asarray(lo, float) + margin
    hi = np.asarray(hi, float) - margin
    acc = np.zeros((0, 3))
    while acc.shape[0] < n:
        need = n - acc.shape[0]
        m = int(need * 1.3) + 64
        cand = lo + (hi - lo) * rng.random((m, 3))
        if acc.shape[0]:
            dist, _ = cKDTree(acc).query(cand, k=1, distance_upper_bound=min_sep)
            cand = cand[~(dist < min_sep)]
        keep = _greedy(cand.shape[0], _ordered_pairs(cand, min_sep))
        acc = np.concatenate([acc, cand[keep][:need]], axis=0)
    return np.ascontiguousarray(acc.T)


def rsa_chains(rng: np.random.Generator, n: int, lo, hi, spacing: float = 1.05, lmin: int = 2,
               lmax: int = 20, jitter: float = 0.1, margin: float = 0.5, min_sep: float = D, lengths=None):
    """Straight chains of beads along random axes, lengths uniform in [lmin, lmax], spacing in d.

    Moments are the chain axis plus isotropic Gaussian jitter of standard deviation ``jitter``,
    normalised.  The last accepted chain is truncated so that exactly n beads are returned.
    Returns (pos (3, n), mom (3, n)).  If ``lengths`` is a list, the realised length of every placed chain
    (the truncated one included) is appended to it; the draws are the same either way.
    """
    lo = np.asarray(lo, float) + margin
    hi = np.asarray(hi, float) - margin
    beads = np.zeros((0, 3))
    axes = np.zeros((0, 3))
    rate = 1.0  # beads accepted per bead drawn in the previous batch (sizes the next batch)
    while beads.shape[0] < n:
        need = n - beads.shape[0]
        mc = int(min(need / ((lmin + lmax) / 2.0) * 1.3 / max(rate, 1e-3), 4 * n / lmin)) + 16
        lens = rng.integers(lmin, lmax + 1, size=mc)
        ax = unit_vectors(rng, mc).T
        ctr = lo + (hi - lo) * rng.random((mc, 3))
        cid = np.repeat(np.arange(mc), lens)
        start = np.concatenate([[0], np.cumsum(lens)[:-1]])
        j = np.arange(cid.size) - start[cid]
        off = (j - (lens[cid] - 1) / 2.0) * spacing
        pts = ctr[cid] + off[:, None] * ax[cid]
        inside = np.all((pts >= lo) & (pts <= hi), axis=1)
        bad = np.zeros(mc, bool)
        bad[cid[~inside]] = True
        if beads.shape[0]:
            old_tree = cKDTree(beads)
            # cheap first pass on each chain's end beads, then every bead of the survivors
            for stage in (j == 0, np.ones(cid.size, bool)):
                live = stage & ~bad[cid]
                dist, _ = old_tree.query(pts[live], k=1, distance_upper_bound=min_sep)
                bad[cid[live][dist < min_sep]] = True
        # conflicts among the surviving candidates only (rejected chains cannot block later ones)
        live = np.nonzero(~bad[cid])[0]
        pairs = _ordered_pairs(pts[live], min_sep)
        if pairs.size:
            cp = cid[live[pairs]]
            cp = cp[cp[:, 0] != cp[:, 1]]
            cp = np.unique(np.sort(cp, axis=1), axis=0)
        else:
            cp = np.zeros((0, 2), np.int64)
        ok = _greedy(mc, cp) & ~bad
        sel = np.nonzero(ok)[0]
        rate = max(float(lens[sel].sum()) / float(lens.sum()), 1e-3)
        # accepted chains in draw order; the one that crosses n is truncated to its first beads
        csum = np.cumsum(lens[sel])
        last = int(np.searchsorted(csum, need))  # index of the chain reaching `need` beads
        sel = sel[:last + 1]
        new_b = np.concatenate([pts[start[c]:start[c] + lens[c]] for c in sel], axis=0)[:need] \
            if sel.size else np.zeros((0, 3))
        new_a = np.repeat(ax[sel], lens[sel], axis=0)[:need] if sel.size else np.zeros((0, 3))
        if lengths is not None and sel.size:
            taken = np.minimum(np.cumsum(lens[sel]), need)  # beads placed after each chain
            lengths.extend(int(x) for x in np.diff(np.concatenate([[0], taken])) if x > 0)
        beads = np.concatenate([beads, new_b], axis=0)
        axes = np.concatenate([axes, new_a], axis=0)
    g = rng.standard_normal((n, 3))
    m = axes + jitter * g
    m /= np.linalg.norm(m, axis=1, keepdims=True)
    return np.ascontiguousarray(beads.T), np.ascontiguousarray(m.T)


@dataclasses.dataclass
class Workload:
    """One synthetic input: positions, unit moments, external field, box, and run settings."""
    name: str
    pos: np.ndarray            # (3, N) or (B, 3, N), float64
    mom: np.ndarray            # same shape as pos
    hext: np.ndarray           # (3,) or (B, 3)
    box_lo: np.ndarray         # (3,)
    box_hi: np.ndarray         # (3,)
    theta: float = 0.5
    leaf_size: int = 16
    seed: int = 0

    @property
    def n(self) -> int:
        return self.pos.shape[-1]

    @property
    def batch(self) -> int:
        return 1 if self.pos.ndim == 2 else self.pos.shape[0]


def uniform_cube(n: int, side: float, seed: int, hext=(0.0, 0.0, 0.0), theta: float = 0.5,
                 name: str = "uniform") -> Workload:
    rng = np.random.default_rng(seed)
    pos = rsa_uniform(rng, n, (0.0, 0.0, 0.0), (side, side, side))
    mom = unit_vectors(rng, n)
    return Workload(name, pos, mom, np.asarray(hext, float), np.zeros(3), np.full(3, side), theta,
                    16, seed)


def config1(seed: int = 1001) -> Workload:
    """Plain FP64 single evaluation: N = 4096 uniform in a cube of side 32, theta 0.5, leaf 16."""
    return uniform_cube(4096, 32.0, seed, name="uniform_n4096_cube32")


def config2(seed: int = 1002) -> Workload:
    """Dilute MD workload: N = 2^17 at phi = 0.05, H_ext = (0, 0, 0.5)."""
    n = 1 << 17
    return uniform_cube(n, cube_side(n, 0.05), seed, hext=(0.0, 0.0, 0.5),
                        name="uniform_n131072_phi0.05")


def config3(seed: int = 1003, theta: float = 0.5, n: int = 1 << 20, lengths=None) -> Workload:
    """Aggregated workload: N = 2^20 beads in straight chains (lengths 2-20, spacing 1.05) at phi 0.1.
    lengths: optional list that receives the realised chain lengths (see rsa_chains)."""
    side = cube_side(n, 0.1)
    rng = np.random.default_rng(seed)
    pos, mom = rsa_chains(rng, n, (0.0, 0.0, 0.0), (side, side, side), lengths=lengths)
    return Workload(f"chains_n{n}_phi0.1", pos, mom, np.zeros(3), np.zeros(3), np.full(3, side),
                    theta, 16, seed)


def config4(seed: int = 1004, n: int = 1 << 18) -> Workload:
    """Differentiation workload: N = 2^18 at phi = 0.05, H_ext = (0, 0, 1)."""
    return uniform_cube(n, cube_side(n, 0.05), seed, hext=(0.0, 0.0, 1.0),
                        name=f"uniform_n{n}_phi0.05")


def config5(seed: int = 1005, batch: int = 32, n: int = 1 << 16,
            box=(256.0, 256.0, 8.0)) -> Workload:
    """Batched slab: B realisations of N = 2^16 in a 256 x 256 x 8 slab, H_ext = (0.7, 0, 0).

    Each realisation has its own placement (seed*1000 + r); the thermal noise of realisation r is keyed
    by (noise seed, r) inside the integrator.
    """
    pos = np.empty((batch, 3, n))
    mom = np.empty((batch, 3, n))
    for r in range(batch):
        rng = np.random.default_rng(seed * 1000 + r)
        pos[r] = rsa_uniform(rng, n, (0.0, 0.0, 0.0), box)
        mom[r] = unit_vectors(rng, n)
    hext = np.tile(np.array([0.7, 0.0, 0.0]), (batch, 1))
    return Workload(f"slab_b{batch}_n{n}", pos, mom, hext, np.zeros(3), np.asarray(box, float),
                    0.5, 16, seed)


def fig2_cube(seed: int = 2001, batch: int = 1, n: int = 20000, side: float = 75.0) -> Workload:
    """Cubic confinement of the paper's Fig. 2(a): N = 20000 in a cube of edge 150 R = 75 d (phi = 2.5 %),
    isotropic moments, no external field; one placement per realisation (seed*1000 + r)."""
    return _batched(f"fig2_cube_n{n}", seed, batch, n, (side, side, side))


def fig2_monolayer(seed: int = 2002, batch: int = 1, n: int = 300, side: float = 75.0,
                   height: float = 1.05) -> Workload:
    """Monolayer of the paper's Fig. 2(b): N = 300 in a flat box of height 2.1 R = 1.05 d.  The paper gives
    no lateral size; the cube's edge (150 R = 75 d) is taken, an area fraction of 4.2 %.  Centres start at
    mid-height (the d/2 margin leaves a 0.05 d band)."""
    return _batched(f"fig2_monolayer_n{n}", seed, batch, n, (side, side, height))


def _batched(name: str, seed: int, batch: int, n: int, box) -> Workload:
    pos = np.empty((batch, 3, n))
    mom = np.empty((batch, 3, n))
    for r in range(batch):
        rng = np.random.default_rng(seed * 1000 + r)
        pos[r] = rsa_uniform(rng, n, (0.0, 0.0, 0.0), box)
        mom[r] = unit_vectors(rng, n)
    if batch == 1:
        pos, mom = pos[0], mom[0]
    return Workload(name, pos, mom, np.zeros(3) if batch == 1 else np.zeros((batch, 3)), np.zeros(3),
                    np.asarray(box, float), 0.5, 16, seed)


def maxwell_boltzmann(rng: np.random.Generator, shape, kT: float, mass: float) -> np.ndarray:
    """Gaussian velocities (or angular velocities with mass -> inertia) at temperature kT."""
    return rng.standard_normal(shape) * math.sqrt(kT / mass)


def nearest_to_centre(pos: np.ndarray, k: int) -> np.ndarray:
    """Indices of the k particles nearest the centre of their bounding box (a standalone subset)."""
    c = 0.5 * (pos.min(axis=1) + pos.max(axis=1))
    d2 = ((pos - c[:, None]) ** 2).sum(axis=0)
    return np.sort(np.argsort(d2, kind="stable")[:k])


def cache_file(name: str) -> str:
    """Path of workload `name` in the on-disk cache (npz under $FFBH_CACHE or the temp dir)."""
    import os
    import tempfile
    d = os.environ.get("FFBH_CACHE", os.path.join(tempfile.gettempdir(), "ffbh_cache"))
    os.makedirs(d, exist_ok=True)
    return os.path.join(d, name + ".npz")


def cached(name: str, make):
    """Workload `name` from the on-disk cache (cache_file), else make() it and store it there."""
    import os
    f = cache_file(name)
    if os.path.exists(f):
        z = np.load(f)
        return Workload(str(z["name"]), z["pos"], z["mom"], z["hext"], z["box_lo"], z["box_hi"],
                        float(z["theta"]), int(z["leaf_size"]), int(z["seed"]))
    w = make()
    tmp = f + ".tmp.npz"
    np.savez(tmp, name=w.name, pos=w.pos, mom=w.mom, hext=w.hext, box_lo=w.box_lo, box_hi=w.box_hi,
             theta=w.theta, leaf_size=w.leaf_size, seed=w.seed)
    os.replace(tmp, f)
    return w


def chain_length_table(n: int = 1 << 20, seed: int = 1003) -> str:
    """Markdown histogram of the realised chain lengths of the chain workload (drawn uniform in [2, 20];
    chains that overlap earlier ones or leave the box are redrawn whole, which favours short chains)."""
    lengths = []
    w = config3(seed=seed, n=n, lengths=lengths)
    ln = np.asarray(lengths)
    assert ln.sum() == w.n
    rows = ["| length | chains | fraction of chains | fraction of beads |", "|---|---|---|---|"]
    for L in range(1, 21):
        k = int((ln == L).sum())
        if k:
            rows.append(f"| {L} | {k} | {k / ln.size:.4f} | {k * L / ln.sum():.4f} |")
    rows.append(f"\n{ln.size} chains, {int(ln.sum())} beads; mean length {ln.mean():.2f} (drawn: 11.0), "
                f"bead-weighted mean {float((ln * ln).sum() / ln.sum()):.2f}.")
    return "\n".join(rows) + "\n"

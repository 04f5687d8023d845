"""Reference Langevin MD step (TEST INFRASTRUCTURE ONLY; same rules as the rest of the oracle package).

Equations of motion of Sec. 2 in vector form, integrated with the explicit Euler-Maruyama scheme named in
Sec. 4 (all updates from the state at the start of the step):
    v' = v + dt/M (F - gamma_t v) + sqrt(2 gamma_t kT dt)/M xi_t
    r' = r + dt v
    w' = w + dt/I (m x H_eff - gamma_r w) + sqrt(2 gamma_r kT dt)/I xi_r
    m' = rotation of m by the angle |w| dt about w (Rodrigues), renormalised
F = -dE/dr + short-range pair and wall forces (WCA, or with p["sr_kind"] = 1 the paper's form of Eq. LJ),
H_eff = -dE/dm, E the Barnes-Hut energy (frozen-structure
gradient from the C oracle).  Readings (the paper's angle equations are garbled and its noise variance
for rotations reads 3 kT G_r): vector form, variance 2 gamma kT dt per component.

Thermal noise: Philox4x32-10 (J. Salmon et al., "Parallel random numbers: as easy as 1, 2, 3", SC'11),
written here from its definition; key (seed low 32 bits, seed high 32 bits XOR system index), counter
(step low, step high, particle index, draw 0 or 1); each 32-bit word x maps to u = (x + 1/2) / 2^32 and
pairs of words to two normals by the Box-Muller transform.  Six of the eight normals are used: three
translational, then three rotational.
"""
from __future__ import annotations

import numpy as np

from . import Tree

_MASK = np.uint64(0xFFFFFFFF)
_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds on arrays of 32-bit counters (as uint64); returns four word arrays."""
    c = [np.asarray(x, np.uint64) & _MASK for x in (c0, c1, c2, c3)]
    k0 = np.asarray(k0, np.uint64) & _MASK
    k1 = np.asarray(k1, np.uint64) & _MASK
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c[0]  # 32 x 32 -> 64 bits, exact in uint64
        p1 = _M1 * c[2]
        c = [((p1 >> np.uint64(32)) ^ c[1] ^ k0) & _MASK, p1 & _MASK,
             ((p0 >> np.uint64(32)) ^ c[3] ^ k1) & _MASK, p0 & _MASK]
    return c


def _u01(x):
    return (x.astype(np.float64) + 0.5) / 4294967296.0


def normals(seed: int, system: int, step: int, n: int) -> np.ndarray:
    """The (6, n) normals of one system at one step: rows 0-2 translational, 3-5 rotational."""
    i = np.arange(n, dtype=np.uint64)
    k0 = np.uint64(seed & 0xFFFFFFFF)
    k1 = np.uint64(((seed >> 32) & 0xFFFFFFFF) ^ system)
    s0 = np.uint64(step & 0xFFFFFFFF)
    s1 = np.uint64((step >> 32) & 0xFFFFFFFF)
    words = []
    for draw in (0, 1):
        words += philox4x32_10(np.full(n, s0), np.full(n, s1), i, np.full(n, draw, np.uint64), k0, k1)
    out = []
    for a, b in ((0, 1), (2, 3), (4, 5), (6, 7)):
        r = np.sqrt(-2.0 * np.log(_u01(words[a])))
        t = 2.0 * np.pi * _u01(words[b])
        out += [r * np.cos(t), r * np.sin(t)]
    return np.array(out[:6])


def wca_forces(pos, sigma=1.0, eps=1.0):
    """WCA pair forces by brute force over all pairs: 24 eps [2 (s/r)^12 - (s/r)^6] r_ij / r^2, r < 2^(1/6) s."""
    n = pos.shape[1]
    F = np.zeros_like(pos)
    if eps == 0.0:
        return F
    rc2 = (2.0 ** (1.0 / 6.0) * sigma) ** 2
    for i0 in range(0, n, 512):
        i1 = min(n, i0 + 512)
        d = pos[:, i0:i1, None] - pos[:, None, :]  # (3, b, n)
        r2 = (d * d).sum(axis=0)
        idx = np.arange(i0, i1)
        r2[idx - i0, idx] = np.inf
        sel = r2 < rc2
        sr6 = np.where(sel, (sigma * sigma / np.where(sel, r2, 1.0)) ** 3, 0.0)
        f = np.where(sel, 24.0 * eps * (2.0 * sr6 * sr6 - sr6) / np.where(sel, r2, 1.0), 0.0)
        F[:, i0:i1] = (f[None] * d).sum(axis=2)
    return F


def lj_forces(pos, sigma=1.0, eps=1.0, cut=0.0):
    """The paper's short-range force (Eq. LJ, Sec. 2) by brute force over all pairs:
    24 eps [(s/r)^12 - (s/r)^6] r_ij / r^2, which vanishes at r = s, repels below it and attracts above it
    (potential 2 eps (s/r)^12 - 4 eps (s/r)^6, depth 2 eps at r = s); cut at `cut` (default 2.5 s)."""
    n = pos.shape[1]
    F = np.zeros_like(pos)
    if eps == 0.0:
        return F
    rc = cut if cut > 0.0 else 2.5 * sigma
    rc2 = rc * rc
    for i0 in range(0, n, 512):
        i1 = min(n, i0 + 512)
        d = pos[:, i0:i1, None] - pos[:, None, :]  # (3, b, n)
        r2 = (d * d).sum(axis=0)
        idx = np.arange(i0, i1)
        r2[idx - i0, idx] = np.inf
        sel = r2 < rc2
        sr6 = np.where(sel, (sigma * sigma / np.where(sel, r2, 1.0)) ** 3, 0.0)
        f = np.where(sel, 24.0 * eps * (sr6 * sr6 - sr6) / np.where(sel, r2, 1.0), 0.0)
        F[:, i0:i1] = (f[None] * d).sum(axis=2)
    return F


def short_range_forces(pos, p):
    """Pair forces of the short-range law selected by p["sr_kind"]: 0 WCA (default), 1 the paper's form."""
    if p.get("sr_kind", 0) == 1:
        return lj_forces(pos, p["wca_sigma"], p["wca_eps"], p.get("sr_cut", 0.0))
    return wca_forces(pos, p["wca_sigma"], p["wca_eps"])


def wall_forces(pos, box_lo, box_hi, sigma=1.0, eps=1.0, kind=0, cut=0.0):
    """Walls on the centre-to-face distance with sigma_w = sigma / 2 (distance floored at sigma_w / 10):
    kind 0 the WCA form, cut at 2^(1/6) sigma_w; kind 1 the paper's form (a wall "of the same type" as the
    pair force), cut at half the pair cut-off."""
    if eps == 0.0:
        return np.zeros_like(pos)
    sw = 0.5 * sigma
    if kind == 1:
        c12, rcw = 1.0, 0.5 * (cut if cut > 0.0 else 2.5 * sigma)
    else:
        c12, rcw = 2.0, 2.0 ** (1.0 / 6.0) * sw

    def mag(d):
        dd = np.maximum(d, 0.1 * sw)
        s6 = (sw / dd) ** 6
        return np.where(d < rcw, 24.0 * eps * (c12 * s6 * s6 - s6) / dd, 0.0)

    lo = np.asarray(box_lo, float)[:, None]
    hi = np.asarray(box_hi, float)[:, None]
    return mag(pos - lo) - mag(hi - pos)


def rodrigues(m, w, dt):
    wl = np.linalg.norm(w, axis=0)
    out = m.copy()
    nz = wl > 0
    u = w[:, nz] / wl[nz]
    ph = wl[nz] * dt
    mm = m[:, nz]
    ud = (u * mm).sum(axis=0)
    out[:, nz] = mm * np.cos(ph) + np.cross(u.T, mm.T).T * np.sin(ph) + u * ud * (1.0 - np.cos(ph))
    return out / np.linalg.norm(out, axis=0)


def md_step(state: dict, p: dict, step: int, theta=0.5, leaf=16, field=True, order=1):
    """One step for every system of state (arrays (B, 3, n)); returns the new state (copies).

    p: dt, kT, gamma_t, gamma_r, mass, inertia, wca_eps, wca_sigma, box_lo, box_hi, hext (B, 3), seed, and
    optionally sr_kind (0 WCA, 1 the paper's Eq. LJ form) and sr_cut (its cut-off; 0 = 2.5 sigma).
    field=False drops the dipolar forces and torques (non-interacting particles in H_ext only).  order: the
    cells of the dipolar energy (1: the paper's pseudo-particles; 2: with first moments).
    """
    pos, vel, mom, om = (np.array(state[k], dtype=np.float64) for k in ("pos", "vel", "mom", "omega"))
    B, _, n = pos.shape
    hext = np.zeros((B, 3)) if p.get("hext") is None else np.asarray(p["hext"], float).reshape(B, 3)
    out = {k: np.empty_like(pos) for k in ("pos", "vel", "mom", "omega")}
    for b in range(B):
        if field:
            _, _, dr, dm = Tree(pos[b], mom[b], leaf).energy_grad(theta, hext[b], order=order)
        else:
            dr, dm = np.zeros((3, n)), -np.repeat(hext[b][:, None], n, axis=1)
        F = -dr + short_range_forces(pos[b], p) + \
            wall_forces(pos[b], p["box_lo"], p["box_hi"], p["wca_sigma"], p["wca_eps"], p.get("sr_kind", 0),
                        p.get("sr_cut", 0.0))
        He = -dm
        tq = np.cross(mom[b].T, He.T).T
        xi = normals(p["seed"], b, step, n)
        dt, M, I = p["dt"], p["mass"], p["inertia"]
        at = np.sqrt(2.0 * p["gamma_t"] * p["kT"] * dt) / M
        ar = np.sqrt(2.0 * p["gamma_r"] * p["kT"] * dt) / I
        out["vel"][b] = vel[b] + (dt / M) * (F - p["gamma_t"] * vel[b]) + at * xi[:3]
        out["pos"][b] = pos[b] + dt * vel[b]
        out["omega"][b] = om[b] + (dt / I) * (tq - p["gamma_r"] * om[b]) + ar * xi[3:]
        out["mom"][b] = rodrigues(mom[b], om[b], dt)
    return out


def langevin(alpha):
    """L(a) = coth(a) - 1/a (Eq. Langevin of Sec. 5)."""
    a = np.asarray(alpha, float)
    return 1.0 / np.tanh(a) - 1.0 / a

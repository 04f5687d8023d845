"""Chain formation at strong dipolar coupling: the runs behind the paper's Fig. 2 (Sec. 5), cubic
confinement (N = 20000, edge 150 R) and a monolayer (N = 300, height 2.1 R), with the paper's short-range
law (Eq. LJ) between particles and against the walls, integrated by md_step (HIP-graph replay).

Units.  The paper states its Fig. 2 parameters in SI (T = 300 K, saturation magnetisation 3.1e5 A/m,
density 5000 kg/m^3, R = 10 nm) and its frictions and time step in its own reduced units (lengths in R,
mass V D, time T_ch = (R / M_s) sqrt(3 D / (4 mu0)), Sec. 2).  This package works with d = 2R = 1,
|m| = 1, the particle mass as mass unit and the energy unit e0 = mu0 m^2 / (4 pi d^3), so its time unit is
t0 = sqrt(M d^2 / e0) = 8 sqrt(2) T_ch.  Hence

    kT  = k_B T / e0                      (lambda of Eq. lambda equals 2 / kT)
    gamma_t = Gamma_t * (t0 / T_ch)       (translational friction, per mass)
    gamma_r = Gamma_r * (t0 / T_ch) / 4   (rotational friction; the paper's unit is M R^2, ours M d^2)
    dt  = dtau / (t0 / T_ch)
    inertia = (2/5) M R^2 = 0.1 M d^2

The paper does not give the strength E of its short-range law; eps = kT (well depth 2 kT) is taken, with
the force zero at contact (s = d) and the cut-off at 2.5 s.

Chains are read off a configuration by a bond criterion: two particles are bonded when closer than 1.3 d
and their dipolar pair energy [m_i.m_j - 3 (m_i.r^)(m_j.r^)] / r^3 is below -1 (half the head-to-tail
contact energy).  Clusters are the connected components of the bond graph.

Usage: python -m paper_1212_2934_amd.aggregation [--geometry cube|monolayer] [--steps 100000] ...
"""
import argparse
import ctypes
import math

import numpy as np
import torch
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components
from scipy.spatial import cKDTree

from . import workloads
from .autotune import autotune
from .binding import BarnesHut, md_params

KB = 1.380649e-23       # J/K
MU0 = 4e-7 * math.pi    # T m / A (the pre-2019 exact value; the present one differs by 1e-10)


def reduced_units(T=300.0, Ms=3.1e5, R=10e-9, Gamma_t=0.1, Gamma_r=0.1, dtau=1e-3):
    """Map the paper's SI parameters and reduced frictions / time step to this package's units."""
    m = Ms * 4.0 / 3.0 * math.pi * R ** 3
    d = 2.0 * R
    e0 = MU0 * m * m / (4.0 * math.pi * d ** 3)
    kT = KB * T / e0
    t_ratio = 8.0 * math.sqrt(2.0)  # t0 / T_ch
    return {"kT": kT, "lambda": 2.0 / kT, "gamma_t": Gamma_t * t_ratio, "gamma_r": Gamma_r * t_ratio / 4.0,
            "dt": dtau / t_ratio, "mass": 1.0, "inertia": 0.1, "t0_over_Tch": t_ratio}


def clusters(pos, mom, rcut=1.3, ecut=-1.0):
    """Bond statistics of one configuration (pos, mom of shape (3, n)); see the module docstring."""
    p, m = pos.T, mom.T
    n = p.shape[0]
    pairs = cKDTree(p).query_pairs(rcut, output_type="ndarray")
    if pairs.size:
        r = p[pairs[:, 0]] - p[pairs[:, 1]]
        r2 = (r * r).sum(axis=1)
        mi, mj = m[pairs[:, 0]], m[pairs[:, 1]]
        u = ((mi * mj).sum(axis=1) - 3.0 * (mi * r).sum(axis=1) * (mj * r).sum(axis=1) / r2) / r2 ** 1.5
        bonds = pairs[u < ecut]
    else:
        bonds = np.zeros((0, 2), np.int64)
    g = coo_matrix((np.ones(len(bonds)), (bonds[:, 0], bonds[:, 1])), shape=(n, n))
    _, lab = connected_components(g, directed=False)
    sizes = np.bincount(lab)
    multi = sizes[sizes >= 2]
    deg = np.bincount(bonds.ravel(), minlength=n) if len(bonds) else np.zeros(n, np.int64)
    return {"bonded_fraction": float((deg > 0).mean()), "bonds_per_particle": 2.0 * len(bonds) / n,
            "clusters": int(multi.size), "mean_cluster_size": float(multi.mean()) if multi.size else 0.0,
            "largest_cluster": int(sizes.max()), "branch_fraction": float((deg > 2).mean())}


def temperatures(st, mass, inertia):
    """Translational and rotational kinetic temperatures, M <v^2> / 3 and I <omega^2> / 3."""
    v2 = (st["vel"] ** 2).sum(dim=1).mean().item()
    w2 = (st["omega"] ** 2).sum(dim=1).mean().item()
    return mass * v2 / 3.0, inertia * w2 / 3.0


def run(geometry="cube", batch=1, steps=100000, report=10000, precision="fp32_mixed", theta=0.5, seed=11,
        eps_over_kT=1.0, tuning="auto", **si):
    """Integrate the geometry from random placement; yields one dict of statistics per report interval
    (and one for the initial state).  tuning: a launch shape, or "auto" for the autotuner's choice."""
    u = reduced_units(**si)
    w = workloads.fig2_cube(batch=batch) if geometry == "cube" else workloads.fig2_monolayer(batch=batch)
    pos = w.pos if w.pos.ndim == 3 else w.pos[None]
    mom = w.mom if w.mom.ndim == 3 else w.mom[None]
    n = pos.shape[-1]
    rng = np.random.default_rng(seed)
    kT = u["kT"]
    dev = torch.device("cuda", torch.cuda.current_device())
    st = {"pos": torch.from_numpy(np.ascontiguousarray(pos)).to(dev),
          "vel": torch.from_numpy(workloads.maxwell_boltzmann(rng, pos.shape, kT, u["mass"])).to(dev),
          "mom": torch.from_numpy(np.ascontiguousarray(mom)).to(dev),
          "omega": torch.from_numpy(workloads.maxwell_boltzmann(rng, pos.shape, kT, u["inertia"])).to(dev),
          "step": torch.zeros(1, dtype=torch.int64, device=dev)}
    C3 = ctypes.c_double * 3
    mdp = md_params(u["dt"], kT, u["gamma_t"], u["gamma_r"], u["mass"], u["inertia"], eps_over_kT * kT, 1.0,
                    C3(*w.box_lo), C3(*w.box_hi), None, seed)
    mdp.sr_kind, mdp.sr_cut = 1, 0.0
    if tuning == "auto":
        tuning = autotune(st["pos"], st["mom"], None, theta, 16, precision, md=(st, mdp))["tuning_id"]
    sim = BarnesHut(n, batch, 16, theta, precision, tuning_id=int(tuning))
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()

    def stats(k, ms):
        p, m = st["pos"].cpu().numpy(), st["mom"].cpu().numpy()
        per = [clusters(p[b], m[b]) for b in range(batch)]
        out = {key: float(np.mean([c[key] for c in per])) for key in per[0]}
        tt, tr = temperatures(st, u["mass"], u["inertia"])
        out.update(step=k, time_t0=k * u["dt"], time_Tch=k * u["dt"] * u["t0_over_Tch"], T_trans=tt / kT,
                   T_rot=tr / kT, ms_per_step=ms, z_min=float(p[:, 2].min()), z_max=float(p[:, 2].max()))
        return out

    yield {**stats(0, float("nan")), **{"kT": kT, "lambda": u["lambda"], "dt": u["dt"], "n": n, "batch": batch,
                                        "tuning_id": int(tuning)}}
    graph = sim.capture_md_graph(st, mdp, stream)
    done = 0
    while done < steps:
        k = min(report, steps - done)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(k):
            graph.launch(stream)
        t1.record(stream)
        stream.synchronize()
        done += k
        s = stats(done, t0.elapsed_time(t1) / k)
        s["status_flags"] = sim.check_status()
        yield s


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--geometry", choices=["cube", "monolayer"], default="cube")
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100000)
    ap.add_argument("--report", type=int, default=10000)
    ap.add_argument("--precision", default="fp32_mixed")
    ap.add_argument("--dtau", type=float, default=1e-3, help="time step in the paper's units (T_ch)")
    ap.add_argument("--T", type=float, default=300.0, help="temperature in K")
    ap.add_argument("--eps-over-kT", type=float, default=1.0)
    a = ap.parse_args()
    print("| step | t / T_ch | bonded frac. | bonds/particle | clusters | mean size | largest | branched | "
          "T_t / T | T_r / T | z range | ms/step |")
    print("|---|---|---|---|---|---|---|---|---|---|---|---|")
    for s in run(a.geometry, a.batch, a.steps, a.report, a.precision, eps_over_kT=a.eps_over_kT, T=a.T,
                 dtau=a.dtau):
        if s["step"] == 0:
            print(f"<!-- kT {s['kT']:.5f} (lambda {s['lambda']:.3f}), dt {s['dt']:.4g} t0, N {s['n']}, "
                  f"{s['batch']} realisation(s), tuning {s['tuning_id']} -->")
        print(f"| {s['step']} | {s['time_Tch']:.1f} | {s['bonded_fraction']:.3f} | {s['bonds_per_particle']:.3f} | "
              f"{s['clusters']:.0f} | {s['mean_cluster_size']:.2f} | {s['largest_cluster']:.0f} | "
              f"{s['branch_fraction']:.3f} | {s['T_trans']:.3f} | {s['T_rot']:.3f} | "
              f"{s['z_min']:.3f}-{s['z_max']:.3f} | {s['ms_per_step']:.3f} |"
              + (f" flags {s['status_flags']}" if s.get("status_flags") else ""), flush=True)


if __name__ == "__main__":
    main()

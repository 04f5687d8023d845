"""CPU baseline timings of the oracle (TEST INFRASTRUCTURE; run by the benchmark's CPU-baseline leg only).

Usage: FFBH_ORACLE_NATIVE=1 OMP_NUM_THREADS=<k> python -m oracle.timing <workload.npz> <theta> <leg> [out.npz]

Legs, each one warm-up run and then the median of three (time.perf_counter, wall clock):
- "force": the force evaluation of one MD step on every particle: tree build (Sec. 3.2 kernels 1-4),
  Barnes-Hut field (kernel 5) and the frozen-structure adjoint, FP64; the tree build is also timed alone.
  With out.npz the energy gradient is written there (the benchmark's reference for the GPU gradients).
- "field_sample": tree build plus the Barnes-Hut field of 2^14 sampled targets; the field of all n targets
  is extrapolated as (build + field of the sample * n / 2^14).
- "allpairs_sample": the exact all-pairs field (Eq. H_dip) of 2^12 sampled targets, extrapolated by
  n / 2^12.
Prints one JSON object.
"""
from __future__ import annotations

import json
import statistics
import sys
import time

import numpy as np

from . import Tree, allpairs_field_subset, num_threads

SAMPLE = 1 << 14      # targets of the Barnes-Hut field sample
AP_SAMPLE = 1 << 12   # targets of the all-pairs sample


def _median3(f):
    f()  # warm-up
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        f()
        ts.append(time.perf_counter() - t0)
    return statistics.median(ts), ts


def main():
    path, theta, leg = sys.argv[1], float(sys.argv[2]), sys.argv[3]
    out_path = sys.argv[4] if len(sys.argv) > 4 else None
    z = np.load(path)
    pos, mom = np.ascontiguousarray(z["pos"]), np.ascontiguousarray(z["mom"])
    hext = np.asarray(z["hext"], float).reshape(-1)[:3]
    n = pos.shape[1]
    idx = np.sort(np.random.default_rng(14).choice(n, min(SAMPLE, n), replace=False)).astype(np.int64)
    ap_idx = np.sort(np.random.default_rng(12).choice(n, min(AP_SAMPLE, n), replace=False)).astype(np.int64)
    res = {"leg": leg, "threads": num_threads(), "n": n,
           "sample_targets": int(ap_idx.size if leg == "allpairs_sample" else idx.size)}
    if leg == "force":
        keep = {}

        def force():
            keep["g"] = Tree(pos, mom, 16).energy_grad(theta, hext)

        res["build_s"], res["build_samples_s"] = _median3(lambda: Tree(pos, mom, 16))
        res["force_s"], res["force_samples_s"] = _median3(force)
        if out_path:
            _, E, dr, dm = keep["g"]
            np.savez(out_path, dr=dr, dm=dm, E=E)
    elif leg == "field_sample":
        def field():
            Tree(pos, mom, 16).field_subset(theta, idx)

        res["build_s"], _ = _median3(lambda: Tree(pos, mom, 16))
        res["sample_s"], res["sample_samples_s"] = _median3(field)
        res["field_s_extrapolated"] = res["build_s"] + (res["sample_s"] - res["build_s"]) * n / idx.size
    elif leg == "allpairs_sample":
        res["sample_s"], res["sample_samples_s"] = _median3(lambda: allpairs_field_subset(pos, mom, ap_idx))
        res["field_s_extrapolated"] = res["sample_s"] * n / ap_idx.size
    else:
        raise SystemExit(f"unknown leg {leg}")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

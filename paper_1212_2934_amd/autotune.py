"""Autotuner for the traversal launch shape (tuning_id of bh_params).

Every candidate shape must give the same result as the default shape -- identical per-target interaction
counts and the same field to the last bit (the traversal of one target does not depend on the shape),
and the same adjoint to rounding (its scatters are reduced in a shape-dependent order) -- before its
time counts.  The fastest accepted candidate is cached in a JSON file keyed by device, system
size, batch, theta, leaf size and precision.  The time is that of build + field + adjoint on the given
state, or, when MD parameters are given, of MD steps from it (each step rebuilds the tree from moved
particles, which is what a launch shape that learns from the previous launch meets in a simulation), or,
with field=True, of field evaluations (build + field; only the forward walk's shape matters there).
"""
from __future__ import annotations

import json
import os
import time

import torch

from .binding import BarnesHut, lib


def _key(n, batch, theta, leaf, precision, md=False, field=False):
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    return (f"{dev}|n={n}|b={batch}|theta={theta}|leaf={leaf}|{precision}" + ("|md" if md else "") +
            ("|field" if field else ""))


def autotune(pos, mom, hext=None, theta=0.5, leaf=16, precision="fp32_mixed", repeats=3,
             cache_path=None, verbose=False, md=None, field=False) -> dict:
    """Pick the fastest result-invariant tuning_id for build + forward + adjoint on this input, for
    MD steps when md = (state, md_params) is given (state: pos, vel, mom, omega, step tensors; it is
    copied, not advanced), or for build + field when field is True.

    pos, mom: (B, 3, n) or (3, n) float64 CUDA tensors.  Returns {"tuning_id", "times_ms", "key"}.
    """
    batch = 1 if pos.dim() == 2 else pos.shape[0]
    n = pos.shape[-1]
    if md is not None and field:
        raise ValueError("time either MD steps or field evaluations")
    key = _key(n, batch, theta, leaf, precision, md is not None, field)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]
    ones = torch.ones(batch, dtype=torch.float64, device=pos.device)
    tol = 1e-12 if precision == "fp64" else 1e-6  # the adjoint's reduction order differs between shapes
    ref = None
    ref_grad = None
    times = {}
    for tid in range(int(lib().bh_num_tunings())):
        bh = BarnesHut(n, batch, leaf, theta, precision, tuning_id=tid)
        bh.build(pos)
        cnt = bh.enable_counters()
        H = bh.field(mom, hext, energy=False)
        counts = (cnt[0].clone(), cnt[1].clone())
        bh.disable_counters()
        if ref is None:
            ref = (H.clone(), counts)
        elif not (torch.equal(H, ref[0]) and torch.equal(counts[0], ref[1][0]) and
                  torch.equal(counts[1], ref[1][1])):
            raise RuntimeError(f"tuning {tid} changed the result; refusing it")
        dr, _ = bh.field_backward(mom, hext, gE=ones)
        if ref_grad is None:
            ref_grad = dr.clone()
        elif ((dr - ref_grad).norm() / ref_grad.norm()).item() > tol:
            raise RuntimeError(f"tuning {tid} changed the adjoint beyond rounding; refusing it")
        torch.cuda.synchronize()
        best = float("inf")
        if md is not None:
            st = {k: v.clone() for k, v in md[0].items()}
            bh.md_step(st, md[1])  # the first step has no previous launch to learn from
            torch.cuda.synchronize()
        for _ in range(repeats):
            t0 = time.perf_counter()
            if md is not None:
                bh.md_step(st, md[1])
            elif field:
                bh.build(pos)
                bh.field(mom, hext)
            else:
                bh.build(pos)
                bh.field_backward(mom, hext, gE=ones)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        times[tid] = best * 1e3
        if verbose:
            print(f"tuning {tid}: {best * 1e3:.3f} ms")
    tid = min(times, key=times.get)
    out = {"tuning_id": tid, "times_ms": times, "key": key}
    if cache_path:
        cache[key] = out
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    return out

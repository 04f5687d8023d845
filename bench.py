"""Benchmark: Barnes-Hut dipolar field evaluations and MD-path steps at N = 2^20, theta = 0.5, on one
MI355X, FP32-mixed and FP64, with the dominant kernel's roofline and the FP64 CPU oracle beside it.

Workload: 2^20 particles in straight chains (lengths 2-20, spacing 1.05 d, moments along the chain axis
with N(0, 0.1) jitter) at volume fraction 0.1 in a cube of side 176.41 d, theta = 0.5, leaf size 16,
H_ext = 0 (synthetic, seeded).  A timed step is one MD step (md_step) on that input, i.e. one pass of
the whole hot path: tree build (bounding cube, Morton codes, radix sort, octree, centroids), upward
moment pass, forward field and energy, the adjoint (dE/dr, dE/dm) by re-traversal, WCA pair and wall
forces (partners from a cell grid cut from the build's Morton codes), and the Euler-Maruyama update with
Philox noise (dt 1e-3, kT 1, gamma 0.1, M 1, I 0.1), replayed from a captured HIP graph.  value = MD steps/s in FP32-mixed
precision; field evaluations/s (tree build + field), eager MD steps/s, FP64 figures and the batched slab
workload (32 realisations x 2^16 particles in 256 x 256 x 8, graph-replayed MD steps) are reported beside
it, each precision and workload in the launch shape the autotuner picks for its MD steps (the field
evaluations in the shape it picks for them: build + field).  The gradients
dE/dr and dE/dm of both precisions are compared with the FP64 oracle's (computed by the CPU-baseline leg):
relative L2, 99.9th percentile and maximum per-particle error.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BH dipolar field evals/s + MD steps/s at N=2^20 θ=0.5, FP32 vs FP64 GPU"
PEAK_FP32_VECTOR = 157.3e12   # published MI355X FP32 vector peak (packed FMA)
PEAK_FP32_UNPACKED = 78.6e12  # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz, one FMA per lane
# algorithmic flops per interaction, fixed from the kernel source (FMA = 2, rsqrt = 1):
FLOPS_FWD = 30   # 3 FP64 offset subtractions + 27 for the dipole field and its accumulation
FLOPS_ADJ = 75   # 3 offset + 69 for g, T(x)Hbar and the field T(x)m + 3 gather accumulation


def kernel_source_sha1():
    """Hash of the sources that define the fused traversal kernel (to match committed counter data)."""
    import hashlib
    h = hashlib.sha1()
    for f in ("adjoint.hip", "traverse.h", "ffbh_internal.h"):
        with open(os.path.join(ROOT, "paper_1212_2934_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_traffic(kernel_key):
    """HBM bytes per launch from profiles/traffic.json (rocprofv3 FETCH_SIZE + WRITE_SIZE scaled by a
    plain-copy calibration), or None when the kernel sources changed since the counters were taken."""
    f = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        d = json.load(fh)
    e = d.get(kernel_key)
    if not e or e.get("source_sha1") != kernel_source_sha1():
        return None
    return e["fetch_bytes"] + e["write_bytes"]


def committed_valu_issue(kernel_key):
    """Fraction of the device's VALU issue slots the kernel used, from profiles/valu_issue.json (rocprofv3
    SQ_INSTS_VALU over 256 wave64 instructions per cycle), or None when the kernel sources changed since
    the counters were taken."""
    f = os.path.join(ROOT, "profiles", "valu_issue.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        d = json.load(fh)
    e = d.get(kernel_key)
    if not e or e.get("source_sha1") != kernel_source_sha1():
        return None
    return e["valu_issue_frac"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class HipEvents:
    """Raw hipEvent_t pairs (the library records them around its kernels on the caller's stream)."""

    def __init__(self, count):
        import ctypes as C
        self.C = C
        self.hip = C.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.hip.hipEventSynchronize.argtypes = [C.c_void_p]
        self.hip.hipEventDestroy.argtypes = [C.c_void_p]
        self.ev = []
        for _ in range(count):
            e = C.c_void_p()
            assert self.hip.hipEventCreate(C.byref(e)) == 0
            self.ev.append(e)

    def seconds(self, a, b):
        C = self.C
        assert self.hip.hipEventSynchronize(self.ev[b]) == 0
        ms = C.c_float(0.0)
        assert self.hip.hipEventElapsedTime(C.byref(ms), self.ev[a], self.ev[b]) == 0
        return ms.value * 1e-3

    def __del__(self):
        for e in self.ev:
            self.hip.hipEventDestroy(e)


def table1(args, workloads, BarnesHut, allpairs, md_params):
    """Per-step time of the all-pairs and Barnes-Hut paths for N = 10^3 .. 10^6 (the shape of the paper's
    Table 1): random sequential addition at volume fraction 0.1 in a cube, theta 0.5, leaf 16.  AP step =
    all-pairs field and energy gradient (one kernel); BH step = md_step (build, field, adjoint, WCA,
    integrator) replayed from a HIP graph in the launch shape the autotuner picks for MD steps; field =
    all-pairs field alone vs bh_build + bh_field (eager calls, same shape)."""
    from paper_1212_2934_amd.autotune import autotune
    import ctypes
    import math
    import numpy as np
    import torch
    dev = torch.device("cuda", 0)
    C3 = ctypes.c_double * 3
    print("| N | AP field FP32-mixed ms | AP field FP64 ms | AP step FP32-mixed ms | AP step FP64 ms | "
          "BH field FP32-mixed ms | BH field FP64 ms | BH step FP32-mixed ms | BH step FP64 ms | "
          "AP/BH step FP32-mixed | BH tuning FP32-mixed, FP64 |")
    print("|---|---|---|---|---|---|---|---|---|---|---|")
    for n in (1000, 10000, 100000, 1000000):
        side = (n * math.pi / 6.0 / 0.1) ** (1.0 / 3.0)
        w = workloads.cached(f"uniform_phi0.1_n{n}_seed{3000 + n}",
                             lambda: workloads.uniform_cube(n, side, seed=3000 + n))
        pos = torch.from_numpy(w.pos).to(dev)
        mom = torch.from_numpy(w.mom).to(dev)
        reps = 3 if n >= 100000 else 20

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / reps * 1e3

        row, tun = {}, {}
        for p in ("fp32_mixed", "fp64"):
            row["apf", p] = timed(lambda: allpairs(pos, mom, precision=p))
            row["aps", p] = timed(lambda: allpairs(pos, mom, precision=p, want_dEdr=True))
            st = {"pos": pos.clone(), "vel": torch.zeros_like(pos), "mom": mom.clone(),
                  "omega": torch.zeros_like(pos), "step": torch.zeros(1, dtype=torch.int64, device=dev)}
            mdp = md_params(1e-3, 1.0, 0.1, 0.1, 1.0, 0.1, 1.0, 1.0, C3(0.0, 0.0, 0.0), C3(side, side, side),
                            None, 7)
            tun[p] = autotune(pos, mom, None, 0.5, 16, p, md=(st, mdp))["tuning_id"]
            bh = BarnesHut(n, 1, 16, 0.5, p, tuning_id=tun[p])
            row["bhf", p] = timed(lambda: (bh.build(pos), bh.field(mom)))
            stream = torch.cuda.Stream()
            torch.cuda.synchronize()
            graph = bh.capture_md_graph(st, mdp, stream)
            row["bhs", p] = timed(lambda: graph.launch(stream))
            assert bh.check_status() == 0
            del graph, bh
        f = lambda k, p: f"{row[k, p]:.3f}"
        print(f"| {n} | {f('apf', 'fp32_mixed')} | {f('apf', 'fp64')} | {f('aps', 'fp32_mixed')} | "
              f"{f('aps', 'fp64')} | {f('bhf', 'fp32_mixed')} | {f('bhf', 'fp64')} | {f('bhs', 'fp32_mixed')} | "
              f"{f('bhs', 'fp64')} | {row['aps', 'fp32_mixed'] / row['bhs', 'fp32_mixed']:.2f} | "
              f"{tun['fp32_mixed']}, {tun['fp64']} |", flush=True)


def accuracy(args, workloads, BarnesHut, allpairs, md_params):
    """Field accuracy against cost at N = 2^20 (the benchmark's chain workload): for each theta, the
    paper's pseudo-particles (order 1) and cells with their first moment (order 2).  Error = relative L2
    and 99.9th percentile per particle against the FP64 all-pairs sum; time = build + field (eager calls,
    synchronised, best of 5) and the forward traversal kernel alone (HIP events around it).  Then the
    forces (dE/dr) against the all-pairs energy gradient and the eager MD step time, FP32-mixed."""
    import torch
    dev = torch.device("cuda", 0)
    w = workloads.cached("chains_n1048576_seed1003", lambda: workloads.config3())
    n = w.n
    pos = torch.from_numpy(w.pos).to(dev)
    mom = torch.from_numpy(w.mom).to(dev)
    ref, ref_f, _ = allpairs(pos, mom, precision="fp64", want_dEdr=True)
    import ctypes
    side = float(w.box_hi[0])
    C3 = ctypes.c_double * 3
    mdp = md_params(1e-3, 1.0, 0.1, 0.1, 1.0, 0.1, 1.0, 1.0, C3(0.0, 0.0, 0.0), C3(side, side, side), None, 11)

    def err(H):
        d = torch.linalg.vector_norm(H - ref, dim=0)
        r = torch.linalg.vector_norm(ref, dim=0)
        per = d / torch.clamp(r, min=1e-3 * torch.sqrt(torch.mean(r * r)))
        return ((torch.linalg.vector_norm(H - ref) / torch.linalg.vector_norm(ref)).item(),
                torch.quantile(per[torch.randperm(per.numel(), device=dev)[:1 << 16]], 0.999).item())

    print("| theta | cells | precision | rel. L2 error | 99.9th pct error | build + field ms | traversal ms |")
    print("|---|---|---|---|---|---|---|")
    rows_md = []
    for theta in (0.3, 0.4, 0.5, 0.6, 0.7, 0.8):
        for order in (1, 2):
            for precision in ("fp32_mixed", "fp64"):
                bh = BarnesHut(n, 1, 16, theta, precision, expansion=order)
                ev = HipEvents(4)
                bh.set_raw_timing_events(ev.ev)
                bh.build(pos)
                H = bh.field(mom, energy=False)
                torch.cuda.synchronize()
                best, kern = float("inf"), float("inf")
                for _ in range(5):
                    t0 = time.perf_counter()
                    bh.build(pos)
                    bh.field(mom, energy=False)
                    torch.cuda.synchronize()
                    best = min(best, (time.perf_counter() - t0) * 1e3)
                    kern = min(kern, ev.seconds(0, 1) * 1e3)
                bh.set_raw_timing_events(None)
                assert bh.check_status() == 0
                e2, e999 = err(H)
                print(f"| {theta} | {'order ' + str(order)} | {precision} | {e2:.3e} | {e999:.3e} | {best:.3f} | "
                      f"{kern:.3f} |", flush=True)
                if precision == "fp32_mixed":
                    # forces: dE/dr of the MD step against the all-pairs gradient, and the MD step time
                    dr, _ = bh.field_backward(mom, None, gE=torch.ones(1, dtype=torch.float64, device=dev))
                    fe = (torch.linalg.vector_norm(dr - ref_f) / torch.linalg.vector_norm(ref_f)).item()
                    st = {"pos": pos.clone(), "vel": torch.zeros_like(pos), "mom": mom.clone(),
                          "omega": torch.zeros_like(pos), "step": torch.zeros(1, dtype=torch.int64, device=dev)}
                    bh.md_step(st, mdp)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(5):
                        bh.md_step(st, mdp)
                    torch.cuda.synchronize()
                    rows_md.append((theta, order, fe, (time.perf_counter() - t0) / 5 * 1e3))
                    assert bh.check_status() == 0
                del bh, H
    print()
    print("| theta | cells | force rel. L2 error (FP32-mixed) | MD step ms (FP32-mixed, eager) |")
    print("|---|---|---|---|")
    for theta, order, fe, ms in rows_md:
        print(f"| {theta} | order {order} | {fe:.3e} | {ms:.3f} |", flush=True)


def grad_errors(g, ref):
    """Relative L2, 99.9th percentile and maximum of the per-particle error |g_i - ref_i| /
    max(|ref_i|, 1e-3 rms |ref|) of a (3, n) gradient."""
    import numpy as np
    g = g.reshape(3, -1).cpu().numpy()
    d = np.linalg.norm(g - ref, axis=0)
    r = np.linalg.norm(ref, axis=0)
    per = d / np.maximum(r, 1e-3 * np.sqrt(np.mean(r * r)))
    return {"rel_l2": float(np.linalg.norm(g - ref) / np.linalg.norm(ref)),
            "p999": float(np.quantile(per, 0.999)), "max": float(per.max())}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(workload_npz, theta):
    """The FP64 oracle timed on this host's cores (oracle/timing.py, each leg a child process of its own
    thread count; timing build of the oracle compiled here with -O3 -march=native, no contraction):
    the force evaluation of one MD step on all threads (the baseline value), the field on one core and the
    all-pairs field (both extrapolated from sampled targets).  Returns (cpu_baseline dict, oracle gradient)."""
    import subprocess
    import tempfile
    import numpy as np
    env = dict(os.environ, FFBH_ORACLE_NATIVE="1")
    subprocess.run([sys.executable, "-c", "import oracle; oracle.build(force=True)"], cwd=ROOT, env=env, check=True)
    from oracle import NATIVE_CFLAGS

    def leg(name, threads=None, out=None):
        e = dict(env) if threads is None else dict(env, OMP_NUM_THREADS=str(threads))
        cmd = [sys.executable, "-m", "oracle.timing", workload_npz, str(theta), name] + ([out] if out else [])
        r = subprocess.run(cmd, cwd=ROOT, env=e, check=True, capture_output=True, text=True)
        return json.loads(r.stdout.strip().splitlines()[-1])

    with tempfile.TemporaryDirectory() as td:
        gpath = os.path.join(td, "grad.npz")
        force = leg("force", out=gpath)
        z = np.load(gpath)
        ref = {"dr": z["dr"], "dm": z["dm"]}
    one = leg("field_sample", threads=1)
    ap = leg("allpairs_sample")
    n = force["n"]
    cpu = {"value": 1.0 / force["force_s"], "unit": "MD steps/s", "cores": force["threads"], "kind": "oracle",
           "sample": f"the force evaluation of one MD step at N={n} (tree build, Barnes-Hut field and adjoint for "
                     f"every target, FP64; the WCA forces and the integrator are not timed): one warm-up, median "
                     f"of 3 ({force['force_s']:.2f} s)",
           "cpu_model": cpu_model(), "nproc": os.cpu_count(), "build_flags": " ".join(NATIVE_CFLAGS),
           "force_eval_s_samples": force["force_samples_s"], "tree_build_s": force["build_s"],
           "one_core_field_evals_per_s": 1.0 / one["field_s_extrapolated"],
           "one_core_sample": f"tree build + Barnes-Hut field of {one['sample_targets']} sampled targets on "
                              f"{one['threads']} thread, extrapolated to {n} targets "
                              f"({one['field_s_extrapolated']:.2f} s, extrapolated)",
           "allpairs_field_evals_per_s": 1.0 / ap["field_s_extrapolated"],
           "allpairs_sample": f"exact all-pairs field of {ap['sample_targets']} sampled targets on {ap['threads']} "
                              f"threads, extrapolated to {n} targets ({ap['field_s_extrapolated']:.1f} s, "
                              "extrapolated)"}
    return cpu, ref


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-slab", action="store_true")
    ap.add_argument("--table1", action="store_true",
                    help="print the all-pairs vs Barnes-Hut per-step sweep over N (the paper's Table 1) and exit")
    ap.add_argument("--tuning", type=int, nargs=2, metavar=("FP32_MIXED", "FP64"), default=None,
                    help="launch shapes to use instead of running the autotuner")
    ap.add_argument("--accuracy", action="store_true",
                    help="print field error against cost over theta for order-1 and order-2 cells and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="finish with one plain device copy of MIB MiB (a reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1212_2934_amd import workloads
    import ctypes

    from paper_1212_2934_amd.binding import BarnesHut, allpairs, md_params

    if args.table1:
        table1(args, workloads, BarnesHut, allpairs, md_params)
        return
    if args.accuracy:
        accuracy(args, workloads, BarnesHut, allpairs, md_params)
        return

    log("generating workload (2^20 chains, phi 0.1)")
    w = workloads.cached("chains_n1048576_seed1003", lambda: workloads.config3())
    n = w.n
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    pos = torch.from_numpy(w.pos).to(dev)
    mom = torch.from_numpy(w.mom).to(dev)
    hext = torch.zeros(3, dtype=torch.float64, device=dev)
    ones = torch.ones(1, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    rng = np.random.default_rng(2003)
    side = float(w.box_hi[0])
    vel0 = torch.from_numpy(rng.standard_normal(w.pos.shape)).to(dev)              # kT / M = 1
    om0 = torch.from_numpy(rng.standard_normal(w.pos.shape) * np.sqrt(10.0)).to(dev)  # kT / I = 10
    C3 = ctypes.c_double * 3
    mdp = md_params(1e-3, 1.0, 0.1, 0.1, 1.0, 0.1, 1.0, 1.0, C3(0.0, 0.0, 0.0), C3(side, side, side), None, 2003)
    state0 = {"pos": pos, "vel": vel0, "mom": mom, "omega": om0,
              "step": torch.zeros(1, dtype=torch.int64, device=dev)}

    # launch shape per precision: the autotuner's fastest result-invariant candidate for MD steps from this
    # state, or the one given with --tuning (profiler runs, so that only the timed shape's kernels count)
    from paper_1212_2934_amd.autotune import autotune
    tuning = {}
    for precision in ("fp32_mixed", "fp64"):
        if args.tuning is not None:
            tuning[precision] = args.tuning[0 if precision == "fp32_mixed" else 1]
            log(f"launch shape {precision}: tuning {tuning[precision]} (given)")
            continue
        t = autotune(pos, mom, hext, args.theta, 16, precision, repeats=3, md=(state0, mdp))
        tuning[precision] = t["tuning_id"]
        log(f"autotune {precision}: tuning {t['tuning_id']} "
            f"({', '.join(f'{k}: {v:.2f} ms' for k, v in sorted(t['times_ms'].items()))})")

    # the field evaluations' own shape (only the forward walk's waves per workgroup matter there)
    tuning_field = {}
    for precision in ("fp32_mixed", "fp64"):
        if args.tuning is not None:
            tuning_field[precision] = tuning[precision]
            continue
        t = autotune(pos, mom, hext, args.theta, 16, precision, repeats=3, field=True)
        tuning_field[precision] = t["tuning_id"]
        log(f"autotune field {precision}: tuning {t['tuning_id']} "
            f"({', '.join(f'{k}: {v:.2f} ms' for k, v in sorted(t['times_ms'].items()))})")

    def make(precision, field=False):
        return BarnesHut(n, 1, 16, args.theta, precision,
                         tuning_id=(tuning_field if field else tuning)[precision])

    # interaction counts (outside timing): identical for both precisions
    bh = make("fp32_mixed")
    bh.build(pos)
    nf, nr = bh.enable_counters()
    bh.field(mom, hext)
    assert bh.check_status() == 0
    n_far, n_near = int(nf.sum().item()), int(nr.sum().item())
    bh.disable_counters()
    inter = n_far + n_near
    log(f"interactions per evaluation: far {n_far}, near {n_near}")

    res, H_bh, grads = {}, {}, {}
    for precision in ("fp32_mixed", "fp64"):
        bh = make(precision)
        ev = HipEvents(4)
        bh.set_raw_timing_events(ev.ev)
        state = {"pos": pos.clone(), "vel": vel0.clone(), "mom": mom.clone(), "omega": om0.clone(),
                 "step": torch.zeros(1, dtype=torch.int64, device=dev)}

        def step():
            bh.md_step(state, mdp)

        # the graph gets its own handle: one handle's calls share its workspace and must not overlap
        side_stream = torch.cuda.Stream()
        gbh = make(precision)
        gstate = {k: v.clone() for k, v in state.items()}
        torch.cuda.synchronize()
        graph = gbh.capture_md_graph(gstate, mdp, side_stream)

        def gstep():
            graph.launch(side_stream)

        fbh = make(precision, field=True)

        def field_only():
            fbh.build(pos)
            return fbh.field(mom, hext)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        for _ in range(args.warmup):
            gstep()
        torch.cuda.synchronize()
        t_fwd = t_adj = 0.0
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        t_step_eager = (time.perf_counter() - t0) / args.steps
        t0 = time.perf_counter()
        for _ in range(args.steps):
            gstep()
        torch.cuda.synchronize()
        t_step = (time.perf_counter() - t0) / args.steps
        assert gbh.check_status() == 0
        del graph, gbh
        for _ in range(args.steps):  # adjoint kernel time, one step at a time
            step()
            t_adj += ev.seconds(2, 3)
        # field evaluation alone (build + field), on the handle of the field evaluations' shape
        bh.set_raw_timing_events(None)
        fbh.set_raw_timing_events(ev.ev)
        for _ in range(args.warmup):
            field_only()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            field_only()
        torch.cuda.synchronize()
        t_eval = (time.perf_counter() - t0) / args.steps
        for _ in range(args.steps):  # forward traversal kernel time
            field_only()
            t_fwd += ev.seconds(0, 1)
        assert bh.check_status() == 0 and fbh.check_status() == 0
        fbh.set_raw_timing_events(None)
        # the energy gradient of this precision on the benchmark state (compared with the oracle's below)
        grads[precision] = bh.field_backward(mom, hext, gE=ones)
        assert bh.check_status() == 0
        H_bh[precision] = field_only()[0].clone()
        res[precision] = dict(t_step=t_step, t_step_eager=t_step_eager, t_eval=t_eval, t_fwd_kernel=t_fwd / args.steps,
                              t_adj_kernel=t_adj / args.steps)
        log(f"{precision}: md step (graph) {t_step * 1e3:.3f} ms, eager {t_step_eager * 1e3:.3f} ms, field eval {t_eval * 1e3:.3f} ms, forward traversal "
            f"{res[precision]['t_fwd_kernel'] * 1e3:.3f} ms, fused forward+adjoint traversal "
            f"{res[precision]['t_adj_kernel'] * 1e3:.3f} ms")
        del bh, fbh
    torch.cuda.synchronize()

    # all-pairs reference on the same state: its time, and the Barnes-Hut field error against it
    ap_ms, H_ap = {}, {}
    for precision in ("fp32_mixed", "fp64"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H_ap[precision] = allpairs(pos, mom, precision=precision)[0]
        torch.cuda.synchronize()
        ap_ms[precision] = (time.perf_counter() - t0) * 1e3
        log(f"all-pairs {precision}: {ap_ms[precision]:.1f} ms per field evaluation")

    def rel_err(H, ref):
        d = torch.linalg.vector_norm(H - ref, dim=0)
        r = torch.linalg.vector_norm(ref, dim=0)
        per = d / torch.clamp(r, min=1e-3 * torch.sqrt(torch.mean(r * r)))
        return {"rel_l2": (torch.linalg.vector_norm(H - ref) / torch.linalg.vector_norm(ref)).item(),
                "p999": torch.quantile(per[torch.randperm(per.numel(), device=per.device)[:1 << 16]], 0.999).item()}

    fp32_vs_fp64 = rel_err(H_bh["fp32_mixed"], H_bh["fp64"])
    ap_err = {"bh_fp32_mixed": rel_err(H_bh["fp32_mixed"], H_ap["fp64"]),
              "bh_fp64": rel_err(H_bh["fp64"], H_ap["fp64"]),
              "allpairs_fp32_mixed": rel_err(H_ap["fp32_mixed"], H_ap["fp64"])}
    log(f"field error against the FP64 all-pairs sum: {ap_err}")
    del H_ap

    # batched slab: 32 independent realisations of 2^16 particles, graph-replayed MD steps
    slab, slab_tuning = {}, {}
    if not args.no_slab:
        log("generating slab workload (32 x 2^16 in 256 x 256 x 8)")
        ws = workloads.cached("slab_b32_n65536_seed1005", lambda: workloads.config5())
        sp = torch.from_numpy(ws.pos).to(dev)
        sm = torch.from_numpy(ws.mom).to(dev)
        shext = torch.from_numpy(ws.hext).to(dev)
        srng = np.random.default_rng(2005)
        smdp = md_params(1e-3, 1.0, 0.1, 0.1, 1.0, 0.1, 1.0, 1.0, C3(*ws.box_lo), C3(*ws.box_hi),
                         shext.data_ptr(), 2005)
        svel = torch.from_numpy(srng.standard_normal(ws.pos.shape)).to(dev)
        som = torch.from_numpy(srng.standard_normal(ws.pos.shape) * np.sqrt(10.0)).to(dev)
        for precision in ("fp32_mixed", "fp64"):
            sst = {"pos": sp.clone(), "vel": svel.clone(), "mom": sm.clone(), "omega": som.clone(),
                   "step": torch.zeros(1, dtype=torch.int64, device=dev)}
            if args.tuning is not None:
                stun = tuning[precision]
            else:
                t = autotune(sp, sm, shext, 0.5, 16, precision, repeats=3, md=(sst, smdp))
                stun = t["tuning_id"]
                log(f"autotune slab {precision}: tuning {stun} "
                    f"({', '.join(f'{k}: {v:.2f} ms' for k, v in sorted(t['times_ms'].items()))})")
            slab_tuning[precision] = stun
            sbh = BarnesHut(ws.n, ws.batch, 16, 0.5, precision, tuning_id=stun)
            ss = torch.cuda.Stream()
            torch.cuda.synchronize()
            sg = sbh.capture_md_graph(sst, smdp, ss)
            for _ in range(args.warmup):
                sg.launch(ss)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                sg.launch(ss)
            torch.cuda.synchronize()
            ts = (time.perf_counter() - t0) / args.steps
            assert sbh.check_status() == 0
            slab[precision] = ts
            log(f"slab {precision}: {ts * 1e3:.3f} ms per batched MD step ({ws.batch} realisations)")
            del sg, sbh

    r32 = res["fp32_mixed"]
    # dominant kernel of the FP32-mixed step: the fused forward + adjoint walk
    tid = tuning["fp32_mixed"]
    # the instantiation launched: its last argument says whether the acceptance test runs on squared sides
    # scaled by 1 / theta^2 (theta^2 a power of two up to 0.3, theta = 0.5 here)
    th2 = args.theta * args.theta
    scaled = 0.0 < th2 <= 0.3 and math.frexp(th2)[0] == 0.5
    adj_key = f"k_adjoint<true, false, {'true' if scaled else 'false'}>"
    if r32["t_adj_kernel"] >= r32["t_fwd_kernel"]:
        kname, kt, flops = f"{adj_key} (fused forward + adjoint, tuning {tid})", r32["t_adj_kernel"], FLOPS_ADJ * inter
    else:
        kname, kt, flops = "k_field<fp32_mixed>", r32["t_fwd_kernel"], FLOPS_FWD * inter
    achieved = flops / kt
    roofline = {"bound": "alu", "kernel": kname, "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR,
                "frac_of_unpacked_fp32": achieved / PEAK_FP32_UNPACKED,
                "traffic": committed_traffic(adj_key) if "adjoint" in kname else None,
                "valu_issue_frac": committed_valu_issue(adj_key) if "adjoint" in kname else None,
                "flops_per_launch": flops, "avg_kernel_ms": kt * 1e3}

    cpu, grad_err = None, None
    if not args.no_cpu_baseline:
        log("timing the FP64 CPU oracle on the same workload (force evaluation, 1-core field, all-pairs)")
        cpu, ref = cpu_baseline(workloads.cache_file("chains_n1048576_seed1003"), args.theta)
        grad_err = {p: {"dE/dr": grad_errors(g[0], ref["dr"]), "dE/dm": grad_errors(g[1], ref["dm"])}
                    for p, g in grads.items()}
        log(f"gradient error against the FP64 oracle: {grad_err}")

    out = {
        "metric": METRIC,
        "value": 1.0 / r32["t_step"],
        "unit": "MD steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["t_step"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair arithmetic, f64 tree/accumulation",
        "data": "synthetic",
        "config": {"workload": "chains N=2^20 phi=0.1 cube 176.41 theta=0.5 leaf 16, one MD step",
                   "n": n, "theta": args.theta, "leaf_size": 16},
        "field_evals_per_s_fp32": 1.0 / r32["t_eval"],
        "field_evals_per_s_fp64": 1.0 / res["fp64"]["t_eval"],
        "particle_fields_per_s_fp32": n / r32["t_eval"],
        "interactions_per_s_fp32": inter / r32["t_eval"],
        "field_rel_l2_fp32_mixed_vs_fp64": fp32_vs_fp64,
        "md_steps_per_s_fp64": 1.0 / res["fp64"]["t_step"],
        "md_steps_per_s_fp32_eager": 1.0 / r32["t_step_eager"],
        "slab_b32_n65536_md_steps_per_s": {p: 1.0 / t for p, t in slab.items()} or None,
        "slab_tuning_id": slab_tuning or None,
        "speedup_fp32_over_fp64_step": res["fp64"]["t_step"] / r32["t_step"],
        "interactions_per_eval": inter,
        "kernel_ms": {p: {"traversal": r["t_fwd_kernel"] * 1e3, "adjoint": r["t_adj_kernel"] * 1e3}
                      for p, r in res.items()},
        "tuning_id": tuning,
        "tuning_id_field": tuning_field,
        "allpairs_ms": ap_ms,
        "field_rel_error_vs_allpairs_fp64": ap_err,
        "roofline": roofline,
        "grad_error_vs_oracle_fp64": grad_err,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB read, {args.copy_calibration} MiB written")


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark: complex Langevin + adaptive gauge cooling link-updates/s on one
MI355X.

Workload (the paper's SU(3) + theta-term method at the 16^4 production size):
16^4 periodic lattice, beta = 6.0, theta = 1.0, seed 3, perturbed SL(3,C)
start, adaptive Langevin step (eps0 = 1e-2, bound fixed on the first step),
10 adaptive (D_1) gauge-cooling steps with alpha = 1 and eps_c = eps0 after
every update.  One "step" = one CL update of every link + its 10 cooling
steps.  value = 4 V x steps / wall time (link-updates/s), with the links
resident in HBM before the timed region starts.

Prints ONE JSON line.  Also reports the mixed-precision path on the same
workload, the dominant kernel's roofline (average duration from HIP events
recorded around every launch of an instrumented replay of the same steps; the
bytes are the floor of one read and one write of the link field per sweep),
the whole step against the same floor and against the FP64 VALU, the served
request stream (mixed, all-mixed, all-FP64 and one run at a time) and the
FP64 CPU oracle timed on a bounded sample (2 steps) of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CL+cooling link-updates/s at 16^4, FP64 vs mixed; served p50/p99 step latency"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
VALU_FP64_TFLOPS = 78.6        # 256 CU x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz
VALU_FP32_TFLOPS = 78.6        # same rate: the library is compiled without packed FP32 instructions
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1311_1056_amd", "csrc", "kernels.hip")


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--dims", default="16,16,16,16")
    ap.add_argument("--theta", type=float, default=1.0)
    ap.add_argument("--beta", type=float, default=6.0)
    ap.add_argument("--ncool", type=int, default=10)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 32^4, theta-point and cooling-mode legs")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--served-runs", type=int, default=256, help="runs in the served mix (0: skip)")
    ap.add_argument("--served-budget-mb", type=int, default=2048)
    ap.add_argument("--served-steps-per-call", type=int, default=4,
                    help="batch steps per server call (one wait for the GPU per call)")
    ap.add_argument("--chain-only", action="store_true",
                    help="only run the SU(2) Polyakov-chain leg (for profiling its kernel)")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def kernel_src_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def algorithmic_cost(kind, V, rs, theta):
    """Algorithmic bytes and flops of one launch.

    Bytes: every field element the kernel must touch, read or written once.
    Flops: 3x3 complex product = 108 FMA = 216 flops, adjugate = 126 flops,
    Hermitian-times-general product = 162 flops, Hermitian exponential pair
    (square, determinant, two 20-term real series, two polynomials) ~ 500."""
    L = 4 * V
    mat = 18 * rs
    prod, adj, hprod, hexp = 216, 126, 162, 500
    # the even sites' staged transforms in the link type: Omega alone in FP64
    # (the applying kernel inverts it), Omega - 1 and Omega^-1 - 1 in FP32
    om = (V // 2) * (9 if rs == 8 else 18) * rs
    if kind == "cool_omega":
        # read every link once, write the staged transform per even site;
        # per even site: 8 U U^dagger-type Hermitian products (54 flops) + one pair
        return {"bytes": L * mat + om, "flops": (V // 2) * (8 * 54 + hexp)}
    if kind == "cool_apply":
        # read and write every link once, read the staged transforms; per link: even transform,
        # odd transform (Hermitian products), per odd site: G and one exponential pair
        return {"bytes": L * 2 * mat + om,
                "flops": L * 2 * hprod + (V // 2) * (8 * 54 + hexp)}
    if kind == "cool_step":
        # one cooling step in one kernel: every link read and written once (the
        # halo re-reads are served on chip), both exponential pairs per site
        return {"bytes": L * 2 * mat, "flops": L * 2 * hprod + V * (8 * 54 + hexp)}
    if kind == "drift":
        # one walk per loop along the staple P = e1 e2 e3: Wilson part P and
        # adj(P) (2 products, 3 adjugates, 2 complex axpys of 9 entries).  With
        # the theta term: the transported clover X1 + e1 (X2 + e2 X3 e2^-1) e1^-1
        # (four products, two determinant reciprocals with their scalings and
        # additions, 2 x (26 + 54 + 18) flops), the staple products R = e1 e2
        # and P, the two insertions of Q and the scaling of Q; adjugates of the
        # two raw links, of P and, on every other loop, of e3.  Per plane the
        # two signs' P_+ - P_- and P'_+ - P'_- (36 flops) meet X0 in two
        # products after one scaling.  Per link: e0 A + B adj(e0) and the
        # traceless part.
        axpy, scl = 2 * 9 * 8, 9 * 6
        loop = ((8 * prod + (7 * adj) // 2 + 2 * (26 + scl + 18) + axpy + scl) if theta
                else (2 * prod + 3 * adj + axpy))
        plane = (2 * prod + scl + 36) if theta else 0
        byt = L * (mat + mat) + (V * 6 * mat if theta else 0)  # links + K out (+ F in)
        return {"bytes": byt, "flops": L * (6 * loop + 3 * plane + 2 * prod + adj)}
    if kind == "update":
        return {"bytes": L * 3 * mat, "flops": L * (3 * prod + 600)}
    if kind == "clover":
        return {"bytes": L * mat + V * 6 * mat, "flops": V * 6 * (12 * prod + 8 * adj)}
    return None


def floor_bytes(kind, V, rs):
    """The byte floor's share of one launch: every sweep over the lattice (the
    CL update, each cooling step) reads and writes each link once, with
    neighbours reused on chip; the drift, the clover field, the staged Omega and
    the second read of a two-kernel cooling step are overhead above it.  The
    update and the cooling step's applying kernel carry the sweeps' bytes."""
    if kind in ("update", "cool_apply", "cool_step"):
        return 4 * V * 2 * 18 * rs
    return 0


def kernel_roofline(kind, ms_total, n, V, rs, theta, precision, dims):
    """Roofline entry of one kernel from its event-measured average duration.
    HBM-bound kernels are priced at their share of the sweep byte floor when
    they have one (frac), with the kernel's own necessary bytes beside it."""
    c = algorithmic_cost(kind, V, rs, theta)
    t = ms_total / n * 1e-3
    peak_flops = VALU_FP64_TFLOPS if precision == "fp64" else VALU_FP32_TFLOPS
    ridge = peak_flops * 1e12 / (HBM_PEAK_GBS * 1e9)
    if c["flops"] / c["bytes"] < ridge:
        fb = floor_bytes(kind, V, rs) or c["bytes"]
        achieved = fb / t / 1e9
        rf = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
              "frac": round(achieved / HBM_PEAK_GBS, 4), "bytes_counted": fb,
              "kernel_bytes_frac": round(c["bytes"] / t / 1e9 / HBM_PEAK_GBS, 4)}
    else:
        achieved = c["flops"] / t / 1e12
        rf = {"bound": "alu", "achieved": round(achieved, 2), "peak": peak_flops, "unit": "TFLOP/s",
              "frac": round(achieved / peak_flops, 4)}
    rf["kernel"] = "k_" + kind
    rf["avg_us"] = round(1e6 * t, 2)
    rf["alg_bytes_per_launch"] = c["bytes"]
    rf["alg_flops_per_launch"] = c["flops"]
    rf["traffic"] = traffic_for(rf["kernel"], precision, dims)
    return rf


def run_gpu(args, precision, with_timing=True, record=False):
    import torch
    import paper_1311_1056_amd as cl
    dims = tuple(int(x) for x in args.dims.split(","))
    V = dims[0] * dims[1] * dims[2] * dims[3]
    prec = cl.CL_FP64 if precision == "fp64" else cl.CL_MIXED
    lat = cl.Lattice(dims, args.beta, args.theta, prec, seed=3, device="cuda:0")
    lat.init(True, 0.3, 0.05)
    kw = dict(eps0=1e-2, adaptive=True, n_cool=args.ncool, eps_c=1e-2, alpha=1.0, mode=cl.CL_ALPHA_UNORM)
    if record:
        lat.record_enable(True)
    # capture both step graphs (a block of eight steps and a single step) now,
    # so that no capture lands in the timed region whatever --warmup is
    lat.run_prepare(**kw)
    # the capture above left the GPU idle: bring it back to its clocks before
    # the warm-up steps
    settle_gpu(dims, args.beta, args.theta, prec, kw)
    lat.run_steps(args.warmup, **kw)
    torch.cuda.synchronize()
    # timed region: K steps replayed from the captured step graph
    t0 = time.perf_counter()
    lat.run_steps(args.steps, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing = {}
    if with_timing:
        # instrumented replay of K more steps: every kernel bracketed by HIP events
        # on the lattice's stream (individual launches instead of the graph)
        lat.timing_enable(True)
        lat.run_steps(args.steps, **kw)
        timing = lat.timing_read()
        lat.timing_enable(False)
    obs = lat.measure()
    rec = lat.record_read(obs["step"] - args.steps + 1, args.steps) if record else None
    lat.close()
    dt = t1 - t0
    return {"V": V, "dims": dims, "seconds": dt, "ms_per_step": 1e3 * dt / args.steps,
            "value": 4 * V * args.steps / dt, "timing": timing, "obs": obs, "record": rec}


def roofline(res, precision, theta):
    """The dominant kernel's roofline (largest share of the step's kernel time)
    and the per-kernel table."""
    rs = 8 if precision == "fp64" else 4
    V = res["V"]
    timing = res["timing"]
    if not timing:
        return None, {}, []
    total = sum(ms for ms, _ in timing.values())
    kernels = {}
    for k, (ms, n) in timing.items():
        kernels[k] = {"avg_us": round(1e3 * ms / n, 3), "launches": n, "share": round(ms / total, 4)}
    costed = [k for k in timing if algorithmic_cost(k, V, rs, theta)]
    rfs = []
    for k in sorted(costed, key=lambda k: -timing[k][0]):
        rf = kernel_roofline(k, timing[k][0], timing[k][1], V, rs, theta, precision, res["dims"])
        rf["share_of_step"] = round(timing[k][0] / total, 3)
        if rf["bound"] == "hbm":
            # practical ceiling at this size: a plain device copy of the same bytes
            cus = copy_us(rf["alg_bytes_per_launch"])
            rf["copy_same_bytes_us"] = round(cus, 2)
            rf["frac_of_copy"] = round(cus / rf["avg_us"], 4)
        rfs.append(rf)
    return rfs[0], kernels, rfs


def step_roofline(res, precision, theta, n_cool, dims=None):
    """The whole CL step against the byte floor (one read and one write of the
    link field for the update and for each of the n_cool cooling steps) and
    against the VALU (the algorithmic flops of the step's kernels).  With
    counter runs of the current kernels for this lattice, also the bytes the
    step's kernels actually moved (FETCH_SIZE + WRITE_SIZE per launch times
    launches per step, re-fetches included) over the step time."""
    rs = 8 if precision == "fp64" else 4
    V = res["V"]
    t = res["ms_per_step"] * 1e-3
    byt = (1 + n_cool) * 4 * V * 2 * 18 * rs
    kinds = ["drift", "update"] + (["clover"] if theta else [])
    flops = sum(algorithmic_cost(k, V, rs, theta)["flops"] for k in kinds)
    flops += n_cool * (algorithmic_cost("cool_omega", V, rs, theta)["flops"] +
                       algorithmic_cost("cool_apply", V, rs, theta)["flops"])
    peak = VALU_FP64_TFLOPS if precision == "fp64" else VALU_FP32_TFLOPS
    t_hbm, t_valu = byt / (HBM_PEAK_GBS * 1e9), flops / (peak * 1e12)
    return {"floor_bytes_per_step": byt, "achieved_GBs": round(byt / t / 1e9, 1), "peak_GBs": HBM_PEAK_GBS,
            "frac_hbm": round(byt / t / 1e9 / HBM_PEAK_GBS, 4), "flops_per_step": flops,
            "achieved_TFLOPs": round(flops / t / 1e12, 2), "peak_TFLOPs": peak,
            "hbm_bound_ms": round(1e3 * t_hbm, 4), "valu_bound_ms": round(1e3 * t_valu, 4),
            "binding_roof": "hbm" if t_hbm >= t_valu else "valu",
            "frac_of_binding_roof": round(max(t_hbm, t_valu) / t, 4), "ms_per_step": round(1e3 * t, 4),
            **measured_step_traffic(precision, dims, theta, n_cool, t)}


def measured_step_traffic(precision, dims, theta, n_cool, t):
    """Counter-measured bytes per step and their rate, or nulls when a kernel
    of the step has no counter run on the current source."""
    out = {"traffic_bytes_per_step": None, "traffic_GBs": None, "frac_hbm_traffic": None}
    if dims is None:
        return out
    launches = {"k_drift": 1, "k_update": 1, "k_cool_omega": n_cool, "k_cool_apply": n_cool}
    if theta:
        launches["k_clover"] = 1
    total = 0
    for k, n in launches.items():
        b = traffic_for(k, precision, dims)
        if b is None:
            return out
        total += n * b
    return {"traffic_bytes_per_step": total, "traffic_GBs": round(total / t / 1e9, 1),
            "frac_hbm_traffic": round(total / t / 1e9 / HBM_PEAK_GBS, 4)}


_COPY_CACHE = {}


def copy_us(total_bytes):
    """Best-of-20 event-timed duration of a plain device copy (torch copy_)
    that reads and writes total_bytes / 2 each."""
    if total_bytes in _COPY_CACHE:
        return _COPY_CACHE[total_bytes]
    import torch
    n = max(1, int(total_bytes // 16))
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(20):
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, 1e3 * e0.elapsed_time(e1))
    del a, b
    _COPY_CACHE[total_bytes] = best
    return best


def traffic_for(kernel, precision, dims):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they
    were taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            tab = json.load(f)
    except (OSError, ValueError):
        return None
    key = f"{kernel}/{precision}/{'x'.join(map(str, dims))}"
    ent = tab.get(key)
    if not ent or ent.get("src_sha") != kernel_src_hash():
        return None
    return ent.get("bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args):
    """The FP64 oracle timed on the host: a bounded sample of the bench workload
    on all threads, plus the two small configurations (4^4 fixed-eps D_0 and
    8^4 adaptive D_1) on all threads and on one thread."""
    import numpy as np
    import oracle
    dims = tuple(int(x) for x in args.dims.split(","))
    V = int(np.prod(dims))
    threads = oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    U = oracle.init_links(dims, 3, 0.3, 0.05)
    t0 = time.perf_counter()
    oracle.run(dims, U, args.beta, args.theta, 3, args.cpu_steps, 1e-2, True, args.ncool, 1e-2, 1.0, 1)
    dt = time.perf_counter() - t0
    small = {}
    for name, (cd, beta, seed, nst, eps0, adaptive, nc, mode) in {
            "4x4x4x4_fixed_eps_D0": ((4, 4, 4, 4), 5.7, 1, 20, 1e-3, False, 5, 0),
            "8x8x8x8_adaptive_D1": ((8, 8, 8, 8), 6.0, 2, 3, 1e-2, True, 10, 1)}.items():
        rec = {}
        for nth in (threads, 1):
            oracle.set_threads(nth)
            Uc = oracle.init_links(cd, seed, 0.3, 0.05)
            t1 = time.perf_counter()
            oracle.run(cd, Uc, beta, 0.0, seed, nst, eps0, adaptive, nc, eps0, 1.0, mode)
            rec[f"threads_{nth}"] = round(4 * int(np.prod(cd)) * nst / (time.perf_counter() - t1), 1)
        small[name] = rec
    oracle.set_threads(threads)
    return {"value": 4 * V * args.cpu_steps / dt, "unit": "link-updates/s", "cores": threads, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"{args.cpu_steps} steps (CL update + {args.ncool} cooling steps + measurement each) of the "
                      f"same {'x'.join(map(str, dims))} workload, FP64, {threads} OpenMP threads, {dt:.1f} s",
            "small_configs_link_updates_per_s": small}


SERVED_SHAPES = [(6, 6, 6, 6), (8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 16), (8, 8, 8, 16), (24, 24, 24, 8)]


def served_mix(n, seed=6):
    """The served request mix: lattice uniform over six shapes, beta ~ U[5.7, 6.2],
    theta ~ U[0, 2], 50..500 steps, 1..20 cooling steps per update, eps0 ~ U[1e-3, 1e-2],
    FP64 or mixed with probability 1/2; run seed 1000 + index."""
    import numpy as np
    rng = np.random.default_rng(seed)
    runs = []
    for i in range(n):
        runs.append(dict(dims=SERVED_SHAPES[int(rng.integers(6))], beta=float(rng.uniform(5.7, 6.2)),
                         theta=float(rng.uniform(0.0, 2.0)), n_steps=int(rng.integers(50, 501)),
                         n_cool=int(rng.integers(1, 21)), eps0=float(rng.uniform(1e-3, 1e-2)),
                         prec=int(rng.integers(2)), seed=1000 + i))
    return runs


def served_stream(capacity_lus, n_runs, load, prec=None):
    """The request mix and its Poisson arrival times at `load` x the single-run
    FP64 capacity (arrival seed 5); prec = 0 / 1 makes every run FP64 / mixed."""
    import numpy as np
    runs = served_mix(n_runs)
    if prec is not None:
        for r in runs:
            r["prec"] = prec
    work = np.array([4 * np.prod(r["dims"]) * r["n_steps"] for r in runs], dtype=float)
    rate = load * capacity_lus / work.mean()  # runs per second
    arrivals = np.cumsum(np.random.default_rng(5).exponential(1.0 / rate, len(runs)))
    return runs, arrivals, rate


PREC_NAMES = {None: "FP64 or mixed with probability 1/2", 0: "all FP64", 1: "all mixed"}


def served(args, capacity_lus, n_runs, load, prec=None):
    """Continuous batching of the request mix arriving as a Poisson stream at
    `load` x the single-run FP64 capacity, under a fixed HBM budget (above 1x
    the queue grows and admission waits for memory to free up)."""
    import numpy as np
    import paper_1311_1056_amd as cl
    runs, arrivals, rate = served_stream(capacity_lus, n_runs, load, prec)
    srv = cl.Server(args.served_budget_mb << 20)
    results = []
    i = 0
    t0 = time.perf_counter()
    while len(results) < len(runs):
        now = time.perf_counter() - t0
        while i < len(runs) and arrivals[i] <= now:
            r = runs[i]
            srv.submit(r["dims"], r["beta"], r["theta"], r["prec"], r["seed"], r["n_steps"], r["eps0"], True,
                       r["n_cool"], r["eps0"], 1.0, cl.CL_ALPHA_UNORM, tag=i)
            i += 1
        a, p = srv.step(args.served_steps_per_call)
        results += srv.poll()
        if a == 0 and p == 0 and i < len(runs):
            time.sleep(max(0.0, min(arrivals[i] - (time.perf_counter() - t0), 0.01)))
    makespan = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    lu = sum(r["link_updates"] for r in results)
    bad = sum(1 for r in results if r["status"] != 0)
    return {"value": round(lu / makespan, 1), "unit": "link-updates/s", "runs": len(runs), "failed_runs": bad,
            "step_ms_p50": round(st["step_ms_p50"], 3), "step_ms_p99": round(st["step_ms_p99"], 3),
            "queue_wait_s_p50": round(st["wait_s_p50"], 3), "queue_wait_s_p99": round(st["wait_s_p99"], 3),
            "makespan_s": round(makespan, 2), "gpu_busy_s": round(st["busy_s"], 2),
            "batch_steps": st["batch_steps"], "load": load, "arrival_rate_runs_per_s": round(rate, 3),
            "budget_bytes": args.served_budget_mb << 20, "steps_per_call": args.served_steps_per_call,
            "mix": "6^4, 8^4, 12^4, 16^4, 8^3x16, 24^3x8; beta U[5.7,6.2]; theta U[0,2]; 50-500 steps; "
                   f"1-20 D1 cooling steps; eps0 U[1e-3,1e-2]; {PREC_NAMES[prec]}; Poisson arrivals"}


def served_one_at_a_time(args, capacity_lus, n_runs, load, prec=0):
    """The same request stream without batching: each run, in arrival order,
    on its own lattice (the lattice API's graph-replayed steps) once the
    previous one has finished.  A run's per-step latency is its run time over
    its steps."""
    import numpy as np
    import torch
    import paper_1311_1056_amd as cl
    runs, arrivals, rate = served_stream(capacity_lus, n_runs, load, prec)
    step_ms, waits, lu = [], [], 0
    t0 = time.perf_counter()
    for i, r in enumerate(runs):
        now = time.perf_counter() - t0
        if arrivals[i] > now:
            time.sleep(arrivals[i] - now)
        t_start = time.perf_counter() - t0
        waits.append(t_start - arrivals[i])
        lat = cl.Lattice(r["dims"], r["beta"], r["theta"], r["prec"], r["seed"])
        lat.init(True, 0.3, 0.05)
        lat.run_steps(r["n_steps"], r["eps0"], True, r["n_cool"], r["eps0"], 1.0, cl.CL_ALPHA_UNORM)
        lat.measure()
        lat.close()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0 - t_start
        step_ms += [1e3 * dt / r["n_steps"]] * r["n_steps"]
        lu += 4 * int(np.prod(r["dims"])) * r["n_steps"]
    makespan = time.perf_counter() - t0
    return {"value": round(lu / makespan, 1), "unit": "link-updates/s", "runs": len(runs),
            "step_ms_p50": round(float(np.percentile(step_ms, 50)), 3),
            "step_ms_p99": round(float(np.percentile(step_ms, 99)), 3),
            "queue_wait_s_p50": round(float(np.percentile(waits, 50)), 3),
            "queue_wait_s_p99": round(float(np.percentile(waits, 99)), 3),
            "makespan_s": round(makespan, 2), "load": load, "arrival_rate_runs_per_s": round(rate, 3),
            "mix": f"the served stream, {PREC_NAMES[prec]}, one run at a time"}


def with_args(args, **kw):
    d = dict(vars(args))
    d.update(kw)
    return argparse.Namespace(**d)


def large_lattice(args):
    """32^4 FP64: 604 MB of links, more than the 256 MB Infinity Cache, so every
    sweep streams from HBM."""
    a = with_args(args, dims="32,32,32,32", steps=5, warmup=2)
    res = run_gpu(a, "fp64")
    rf, kernels, rfs = roofline(res, "fp64", args.theta)
    out = {"lattice": "32x32x32x32", "value": round(res["value"], 1), "unit": "link-updates/s",
           "ms_per_step": round(res["ms_per_step"], 4), "steps": a.steps, "roofline": rf, "rooflines": rfs,
           "step_roofline": step_roofline(res, "fp64", args.theta, args.ncool, (32, 32, 32, 32))}
    # one GPU's share of a 32^4 lattice split in two along x3 (the kernels at
    # that shape, periodic here; the halo exchange of a real split is not built)
    b = with_args(args, dims="32,32,32,16", steps=10, warmup=2)
    rb = run_gpu(b, "fp64")
    rfb, _, _ = roofline(rb, "fp64", args.theta)
    out["half_share_32x32x32x16"] = {"value": round(rb["value"], 1), "unit": "link-updates/s",
                                     "ms_per_step": round(rb["ms_per_step"], 4), "steps": b.steps, "roofline": rfb}
    return out


def mixed_vs_fp64(args, n_steps=300):
    """Mixed precision against FP64 over whole trajectories at 24^4 and 32^4
    (theta 1, seed 4, adaptive eps0 = 1e-2, 10 D_1 cooling steps per update):
    both start from the same FP32-representable links and draw the same
    Philox noise; each records P, Q and d at every step on the device.  The
    first step's error is the per-step accuracy of the mixed path (gated at
    1e-6 in the tests); later steps show how the CL dynamics amplify it."""
    import numpy as np
    import torch
    import paper_1311_1056_amd as cl
    kw = (1e-2, True, 10, 1e-2, 1.0, cl.CL_ALPHA_UNORM)
    out = {"steps": n_steps, "theta": 1.0, "seed": 4,
           "err": "|mixed - FP64| / max(1, |FP64|) of the recorded observable at that step"}
    for L in (24, 32):
        dims = (L, L, L, L)
        mx = cl.Lattice(dims, 6.0, 1.0, cl.CL_MIXED, seed=4)
        mx.init(True, 0.3, 0.05)
        fp = cl.Lattice(dims, 6.0, 1.0, cl.CL_FP64, seed=4)
        fp.set_links(mx.get_links())
        recs, ms = [], {}
        for name, lat in (("mixed", mx), ("fp64", fp)):
            lat.record_enable(True)
            lat.run_prepare(*kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lat.run_steps(n_steps, *kw)
            torch.cuda.synchronize()
            ms[name] = round(1e3 * (time.perf_counter() - t0) / n_steps, 4)
            recs.append(lat.record_read(1, n_steps))
            lat.close()
        a, b = recs
        cols = {"plaq": (3, 4), "q": (5, 6), "d": (2, None)}

        def err(i, c):
            re, im = cols[c]
            va = a[i, re] + (1j * a[i, im] if im else 0)
            vb = b[i, re] + (1j * b[i, im] if im else 0)
            return float(abs(va - vb) / max(1.0, abs(vb)))
        at = {}
        for k in (1, 10, 100, n_steps):
            if k <= n_steps:
                at[str(k)] = {c: float(f"{err(k - 1, c):.3e}") for c in cols}
        first_over = {c: next((i + 1 for i in range(n_steps) if err(i, c) > 1e-6), None) for c in cols}
        out[f"{L}x{L}x{L}x{L}"] = {"err_at_step": at, "first_step_over_1e-6": first_over, "ms_per_step_recorded": ms,
                                   "final_fp64": {"plaq": float(b[-1, 3]), "q": [float(b[-1, 5]), float(b[-1, 6])],
                                                  "d": float(b[-1, 2])}}
    return out


def theta_series(args, n_steps=500):
    """The 16^4 workload as a Langevin-time series: 500 CL steps at theta =
    0.5, 1 and 2 (seed 3, adaptive eps, 10 D_1 cooling steps), P, Q, S and
    d recorded on the device at every step and summarised here: the running
    mean of Q (the paper's observable), P and d over the second half, the
    step sizes, and the time per recorded step."""
    import numpy as np
    import torch
    import paper_1311_1056_amd as cl
    kw = (1e-2, True, args.ncool, 1e-2, 1.0, cl.CL_ALPHA_UNORM)
    out = {"steps": n_steps, "dims": "16x16x16x16", "seed": 3}
    for th in (0.5, 1.0, 2.0):
        lat = cl.Lattice((16, 16, 16, 16), args.beta, th, cl.CL_FP64, seed=3)
        lat.init(True, 0.3, 0.05)
        lat.record_enable(True)
        lat.run_prepare(*kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.run_steps(n_steps, *kw)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / n_steps
        r = lat.record_read(1, n_steps)
        lat.close()
        half = r[n_steps // 2:]
        q = r[:, 5] + 1j * r[:, 6]
        run_q = np.cumsum(q) / np.arange(1, n_steps + 1)
        out[f"theta_{th}"] = {
            "ms_per_step": round(1e3 * dt, 4),
            "running_mean_Q": {str(k): [round(float(run_q[k - 1].real), 4), round(float(run_q[k - 1].imag), 4)]
                               for k in (50, 100, 250, n_steps)},
            "plaq_second_half": [round(float(half[:, 3].mean()), 6), round(float(half[:, 3].std()), 6)],
            "d_after_cooling_second_half": [float(f"{half[:, 2].mean():.4e}"), float(f"{half[:, 2].max():.4e}")],
            "d_before_cooling_second_half": float(f"{half[:, 1].mean():.4e}"),
            "eps_mean": float(f"{r[:, 9].mean():.4e}"),
            "langevin_time": round(float(r[:, 9].sum()), 4),
        }
    return out


def theta_points(args):
    """The 16^4 workload at theta = 0, 0.5 and 2 (theta = 1 is the main line)."""
    out = {}
    for th in (0.0, 0.5, 2.0):
        a = with_args(args, theta=th, steps=30, warmup=3)
        res = run_gpu(a, "fp64")
        rf, kernels, rfs = roofline(res, "fp64", th)
        out[f"theta_{th}"] = {"value": round(res["value"], 1), "ms_per_step": round(res["ms_per_step"], 4),
                              "roofline": rf}
    return out


def pure_gauge_links(dims, seed, sx=0.4, sy=0.3):
    """Host-layout links of a cold configuration rotated by a random SL(3,C)
    gauge transformation, U_mu(x) = O_x O_{x+mu}^-1 with O_x = exp(A_x),
    A_x = i sum_a lambda_a (a + i b), a ~ N(0, sx), b ~ N(0, sy): gauge
    equivalent to the identity, so cooling can bring d to 0."""
    import numpy as np
    rng = np.random.default_rng(seed)
    lam = np.zeros((8, 3, 3), complex)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7] = np.diag([1, 1, -2]) / np.sqrt(3)
    V = int(np.prod(dims))
    c = rng.normal(0, sx, (V, 8)) + 1j * rng.normal(0, sy, (V, 8))
    A = 1j * np.einsum("va,aij->vij", c, lam)

    def expm(M):
        # scaling and squaring of a 20-term Taylor series
        k = max(0, int(np.ceil(np.log2(max(np.abs(M).sum(axis=(1, 2)).max(), 1e-300)))) + 1)
        M = M / 2.0 ** k
        E = np.broadcast_to(np.eye(3, dtype=complex), M.shape).copy()
        T = E.copy()
        for n in range(1, 21):
            T = T @ M / n
            E = E + T
        for _ in range(k):
            E = E @ E
        return E

    O = expm(A).reshape(dims[3], dims[2], dims[1], dims[0], 3, 3)
    Oi = expm(-A).reshape(dims[3], dims[2], dims[1], dims[0], 3, 3)
    U = np.zeros((dims[3], dims[2], dims[1], dims[0], 4, 3, 3), complex)
    for mu in range(4):
        U[..., mu, :, :] = O @ np.roll(Oi, -1, axis=3 - mu)
    U = U.reshape(V, 4, 3, 3)
    out = np.zeros((V, 4, 18))
    out[..., 0::2] = U.real.reshape(V, 4, 9)
    out[..., 1::2] = U.imag.reshape(V, 4, 9)
    return out


def cooling_modes(args):
    """D_0 / D_1 / D_2 adaptive cooling of pure-gauge SL(3,C) starts at 16^4
    (eps_c = 1e-2, alpha = 1): the distance d after every 50 cooling steps and
    the time per cooling step, from a mild and a strong gauge rotation."""
    import torch
    import paper_1311_1056_amd as cl
    dims = tuple(int(x) for x in args.dims.split(","))
    out = {"start": "cold links under a random SL(3,C) gauge transformation exp(i lambda_a (a + i b))",
           "eps_c": 1e-2, "alpha": 1.0}
    for start, (sx, sy) in (("mild", (0.3, 0.15)), ("strong", (0.4, 0.3))):
        U0 = pure_gauge_links(dims, 7, sx, sy)
        rec = {"a_sigma": sx, "b_sigma": sy}
        for name, mode in (("D0", cl.CL_ALPHA_FIXED), ("D1", cl.CL_ALPHA_UNORM), ("D2", cl.CL_ALPHA_GRAD)):
            lat = cl.Lattice(dims, args.beta, 0.0, cl.CL_FP64, seed=7)
            lat.set_links(U0)
            d = [lat.unitarity_norm()]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            status = "ok"
            try:
                for _ in range(4):
                    lat.gauge_cool(50, 1e-2, 1.0, mode, sync=False)
                    d.append(lat.unitarity_norm())
            except cl.ClError as e:
                status = "diverged" if e.status == cl.CL_ENONFINITE else f"error {e.status}"
            dt = time.perf_counter() - t0
            lat.close()
            rec[name] = {"d_every_50_steps": [float(f"{x:.4e}") for x in d], "status": status,
                         "ms_per_cooling_step": round(1e3 * dt / (50 * max(1, len(d) - 1)), 4)}
        out[start] = rec
    return out


def alone_vs_batched(args, n=32):
    """The first n runs of the served mix, all submitted at once to the server,
    against the same runs one at a time through the lattice API."""
    import torch
    import paper_1311_1056_amd as cl
    runs = served_mix(n)
    srv = cl.Server(args.served_budget_mb << 20)
    t0 = time.perf_counter()
    for i, r in enumerate(runs):
        srv.submit(r["dims"], r["beta"], r["theta"], r["prec"], r["seed"], r["n_steps"], r["eps0"], True,
                   r["n_cool"], r["eps0"], 1.0, cl.CL_ALPHA_UNORM, tag=i)
    res = []
    while len(res) < n:
        srv.step(args.served_steps_per_call)
        res += srv.poll()
    tb = time.perf_counter() - t0
    srv.close()
    lu = sum(r["link_updates"] for r in res)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in runs:
        lat = cl.Lattice(r["dims"], r["beta"], r["theta"], r["prec"], r["seed"])
        lat.init(True, 0.3, 0.05)
        lat.run_steps(r["n_steps"], r["eps0"], True, r["n_cool"], r["eps0"], 1.0, cl.CL_ALPHA_UNORM)
        lat.measure()
        lat.close()
    ta = time.perf_counter() - t0
    return {"runs": n, "batched_link_updates_per_s": round(lu / tb, 1), "alone_link_updates_per_s": round(lu / ta, 1),
            "batched_s": round(tb, 3), "alone_s": round(ta, 3)}


def chain_cost(n_cool, mode):
    """Algorithmic flops of one SU(2)-chain link-update: one CL update of one
    link with its share of the n_cool cooling steps and of the measurement,
    counted for a work-efficient schedule (a 2x2 complex product = 4 complex
    products + 4 complex FMAs = 56 flops; Box-Muller transcendentals not
    counted).  Drift: prefix, suffix and loop product per link (3 products),
    i beta TL(P) and its norm (44).  Update: eps K + noise and the factor i
    (54), the 2x2 exponential (norm, invariant, two 12-term complex series,
    assembly: 274), the product (56), det renormalisation (51).  Two unitarity
    norms (32).  Cooling step: TL(U U^dag - W^dag W) (62), the scale (3), the
    closed Hermitian exponential pair (9-term real series: 60), the two
    Hermitian-times-general products (80), the Omega / Omega^-1 entries (4),
    plus the D_1 norm (16) or the D_2 gradient sum (6).  Measurement: the
    ordered product (56)."""
    prod = 56
    drift = 3 * prod + 44
    update = 54 + 274 + prod + 51
    cool = 62 + 3 + 60 + 80 + 4 + (16 if mode == 1 else 6 if mode == 2 else 0)
    return drift + update + 32 + n_cool * cool + prod


def chain_workload(args):
    """SU(2) Polyakov chain, S = -(beta/2) Tr(U_1 ... U_N), complex beta =
    2 + i, CL with adaptive step and D_2 cooling (alpha = 1, eps_c = eps0),
    unitary start (sigma 0.3 / 0).  Throughput at N = 10, 100 and 1000 links
    (about 10^6 links each; eps0 = 5e-3, 10 cooling steps per update), and
    <S> = -beta <Tr P / 2> (Langevin-time averages, 1024 chains of N = 10)
    against the exact one-link value -beta I_2(beta) / I_1(beta): versus eps0
    with its linear extrapolation to eps = 0 (10 D_2 steps), and versus the
    number of cooling steps for D_0 and D_2 at eps0 = 1e-3."""
    import numpy as np
    import scipy.special
    import torch
    import paper_1311_1056_amd as cl
    beta = 2.0 + 1.0j
    out = {"workload": "SU(2) Polyakov chain, beta = 2 + 1i, adaptive eps0 = 5e-3, 10 D2 cooling steps "
                       "(alpha = 1, eps_c = eps0) per update, FP64", "throughput": []}
    eps = 5e-3
    for n, n_chains, steps in ((10, 102400, 20), (100, 10240, 20), (1000, 1024, 20)):
        ch = cl.Chain(n, n_chains, beta, seed=1)
        ch.init(0.3, 0.0)
        ch.run(2, eps, True, 10, eps, 1.0, cl.CL_ALPHA_GRAD)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ch.run(steps, eps, True, 10, eps, 1.0, cl.CL_ALPHA_GRAD)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        m = ch.measure()
        ch.close()
        lu = n * n_chains * steps
        tflops = chain_cost(10, 2) * lu / (ms * 1e-3) / 1e12
        out["throughput"].append({
            "n_links": n, "chains": n_chains, "steps": steps, "ms": round(ms, 3),
            "link_updates_per_s": round(lu / (ms * 1e-3), 1),
            "roofline": {"bound": "alu", "kernel": "k_chain_run", "achieved": round(tflops, 2),
                         "peak": VALU_FP64_TFLOPS, "unit": "TFLOP/s", "frac": round(tflops / VALU_FP64_TFLOPS, 4),
                         "alg_flops_per_link_update": chain_cost(10, 2), "traffic": None},
            "chains_ok": sum(x["status"] == 0 for x in m)})
        progress(f"chain N={n}: {lu / (ms * 1e-3) / 1e9:.2f} G link-updates/s")
    exact = complex(-beta * scipy.special.iv(2, beta) / scipy.special.iv(1, beta))

    def point(eps0, n_cool, mode, scale):
        ch = cl.Chain(10, 1024, beta, seed=7)
        ch.init(0.3, 0.0)
        ch.run(int(2.5 / eps0), eps0, True, n_cool, eps0, 1.0, mode)        # Langevin time 2.5
        ch.run(int(scale / eps0), eps0, True, n_cool, eps0, 1.0, mode)      # Langevin time `scale`
        m = [x for x in ch.measure() if x["status"] == 0]
        ch.close()
        S = np.array([-beta * x["mean_L"] for x in m])
        k = max(len(S), 1)
        return {"eps0": eps0, "n_cool": n_cool, "chains_ok": len(m),
                "S": [round(S.mean().real, 4), round(S.mean().imag, 4)],
                "err": [round(S.real.std() / np.sqrt(k), 4), round(S.imag.std() / np.sqrt(k), 4)],
                "d": float(f"{np.mean([x['mean_d'] for x in m]):.3e}") if m else None}

    vs_eps = [point(e, 10, cl.CL_ALPHA_GRAD, 15.0) for e in (4e-3, 2e-3, 1e-3, 5e-4)]
    x = np.array([p["eps0"] for p in vs_eps])
    fit = {}
    for c, part in ((0, "re"), (1, "im")):
        y = np.array([p["S"][c] for p in vs_eps])
        w = 1.0 / np.array([max(p["err"][c], 1e-4) for p in vs_eps]) ** 2
        A = np.stack([np.ones_like(x), x], 1)
        cov = np.linalg.inv(A.T @ (A * w[:, None]))
        coef = cov @ (A.T @ (w * y))
        fit[part] = [round(float(coef[0]), 4), round(float(np.sqrt(cov[0, 0])), 4)]
    progress("chain eps extrapolation done")
    vs_cool = []
    for mode, name in ((cl.CL_ALPHA_FIXED, "D0"), (cl.CL_ALPHA_GRAD, "D2")):
        for n_cool in (0, 1, 3, 10, 30):
            if n_cool == 0 and mode != cl.CL_ALPHA_FIXED:
                continue
            p = point(1e-3, n_cool, mode, 15.0)
            p["mode"] = name
            vs_cool.append(p)
    out["cooling_vs_t"] = chain_cooling_curves()
    progress("chain cooling curves done")
    out["convergence"] = {"n_links": 10, "chains": 1024, "langevin_time": {"therm": 2.5, "measured": 15.0},
                          "exact_S": [round(exact.real, 4), round(exact.imag, 4)],
                          "vs_eps_D2_ncool10": vs_eps,
                          "extrapolated_S_eps0": {"re": fit["re"], "im": fit["im"]},
                          "vs_cooling_steps_eps1e-3": vs_cool}
    progress("chain convergence done")
    return out


def gauge_rotated_chains(n_chains, n, seed, sv=0.5, sa=0.3, sb=0.3):
    """Input generator: U_k = Omega_k V_k Omega_{k+1}^-1 on periodic chains,
    V_k = exp(i sigma.x) in SU(2) and Omega_k = exp(i sigma.(a + i b)) in
    SL(2,C), x, a, b independent normals (numpy seed): unitary chains moved off
    SU(2) along their gauge orbits.  (..., n, 8) doubles, row-major 2x2, (re, im)."""
    import numpy as np
    pauli = np.array([[[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]], complex)

    def expm2(A):
        # traceless 2x2: A^2 = w 1, exp(A) = cosh(l) 1 + sinh(l)/l A with l^2 = w
        w = A[..., 0, 0] ** 2 + A[..., 0, 1] * A[..., 1, 0]
        l = np.sqrt(w + 0j)
        small = np.abs(l) < 1e-8
        sh = np.where(small, 1.0 + w / 6.0, np.sinh(l) / np.where(small, 1.0, l))
        return np.cosh(l)[..., None, None] * np.eye(2) + sh[..., None, None] * A

    rng = np.random.default_rng(seed)
    x = rng.normal(0, sv, (n_chains, n, 3))
    c = rng.normal(0, sa, (n_chains, n, 3)) + 1j * rng.normal(0, sb, (n_chains, n, 3))
    Vk = expm2(1j * np.einsum('cka,aij->ckij', x, pauli))
    O = expm2(1j * np.einsum('cka,aij->ckij', c, pauli))
    Oi = expm2(-1j * np.einsum('cka,aij->ckij', c, pauli))
    U = O @ Vk @ np.roll(Oi, -1, axis=1)
    out = np.zeros(U.shape[:-2] + (8,))
    out[..., 0::2] = U.real.reshape(U.shape[:-2] + (4,))
    out[..., 1::2] = U.imag.reshape(U.shape[:-2] + (4,))
    return out


def chain_cooling_curves():
    """Cooling alone on gauge-rotated unitary chains U_k = Omega_k V_k
    Omega_{k+1}^-1 (64 chains, numpy seed 3, eps_c = 1e-3, alpha = 1): d(t)
    for D_0, D_1, D_2 on N = 1000 links with the log-log slope of the last
    decade of D_0 (the paper reports t^(-3/2)), and D_0 for N = 1 ... 1000
    (the slowing down with the chain length)."""
    import numpy as np
    import paper_1311_1056_amd as cl
    ts = (1, 3, 10, 30, 100, 300, 1000, 3000, 10000, 30000)

    def curve(n, mode):
        ch = cl.Chain(n, 64, 1.0)
        ch.set_links(gauge_rotated_chains(64, n, 3))
        d, t = [float(np.mean([x["d"] for x in ch.measure()]))], 0
        for T in ts:
            ch.cool(T - t, 1e-3, 1.0, mode)
            t = T
            m = ch.measure()
            d.append(float(np.mean([x["d"] for x in m])))
        ok = sum(x["status"] == 0 for x in m)
        ch.close()
        return {"d": [float(f"{v:.4e}") for v in d], "chains_ok": ok}

    out = {"eps_c": 1e-3, "alpha": 1.0, "chains": 64, "t": [0] + list(ts), "n1000": {}, "D0_vs_n": {}}
    for mode, name in ((0, "D0"), (1, "D1"), (2, "D2")):
        out["n1000"][name] = curve(1000, mode)
    d0 = out["n1000"]["D0"]["d"]
    out["n1000"]["D0_slope_3000_to_30000"] = round(float(np.log(d0[-1] / d0[-3]) / np.log(10.0)), 3)
    for n in (1, 2, 10, 100):
        out["D0_vs_n"][f"n{n}"] = curve(n, 0)
    return out


def copy_calibration(mib):
    import torch
    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 4, "bytes_written": n * 4, "launches": 3}), flush=True)


def settle_gpu(dims, beta, theta, prec, kw, seconds=0.1):
    """Run the leg's own kernels for about `seconds` on a separate scratch
    lattice (seed 9, discarded) just before the measured lattice's warm-up
    steps.  An idle GPU clocks down and needs about 10 ms of this load to come
    back; a few warm-up steps are not enough.  Measured on one box (16^4,
    ms per step of a 20-step call right after 5 warm-up steps / of 100 steps):
    FP64 0.504 / 0.462 with nothing before, 0.487 / 0.461 after plain device
    copies, 0.463 / 0.461 after this; mixed 0.392 / 0.370, 0.389 / 0.369,
    0.370 / 0.369.  The measured lattice still takes exactly the warm-up and
    timed steps it is asked for; nothing here is timed."""
    import torch
    import paper_1311_1056_amd as cl
    s = cl.Lattice(dims, beta, theta, prec, seed=9, device="cuda:0")
    s.init(True, 0.3, 0.05)
    s.run_prepare(**kw)
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        s.run_steps(8, **kw)
        torch.cuda.synchronize()
    s.close()


_T0 = time.perf_counter()


def progress(msg):
    """One line per finished leg on stderr (the JSON line is the only stdout)."""
    print(f"bench.py [{time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE={world}); "
              "independent runs shard across GPUs with no exchange, so the per-GPU figure is the N=1 line",
              file=sys.stderr, flush=True)
        sys.exit(2)
    if args.copy_calib:
        copy_calibration(args.copy_calib)
        return
    if args.chain_only:
        print(json.dumps({"chain": chain_workload(args)}), flush=True)
        return
    dims = tuple(int(x) for x in args.dims.split(","))
    res = run_gpu(args, args.precision)
    rf, kernels, rfs = roofline(res, args.precision, args.theta)
    progress(f"main workload: {res['value'] / 1e6:.1f} M link-updates/s")
    prec_name = "FP64" if args.precision == "fp64" else "mixed FP32/FP64"
    out = {
        "metric": METRIC,
        "value": round(res["value"], 1),
        "unit": "link-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.dims.replace(',', 'x')} SU(3)+theta CL, {prec_name}, {args.ncool} D1 "
                               f"cooling steps/update, beta={args.beta}, theta={args.theta}, adaptive eps0=1e-2, "
                               f"alpha=1, eps_c=1e-2, seed 3, periodic Wilson action",
                   "lattice": args.dims.replace(",", "x"), "precision": args.precision,
                   "parallelism": "single GPU"},
        "roofline": rf,
        "step_roofline": step_roofline(res, args.precision, args.theta, args.ncool, dims),
        "rooflines": rfs,
        "kernels": kernels,
        "observables_after": {"plaq": [res["obs"]["plaq"].real, res["obs"]["plaq"].imag],
                              "q": [res["obs"]["q"].real, res["obs"]["q"].imag], "d": res["obs"]["d"]},
    }
    if args.precision == "fp64" and not args.no_mixed:
        mx = run_gpu(args, "mixed")
        progress(f"mixed precision: {mx['value'] / 1e6:.1f} M link-updates/s")
        mrf, mk, mrfs = roofline(mx, "mixed", args.theta)
        out["mixed"] = {"value": round(mx["value"], 1), "ms_per_step": round(mx["ms_per_step"], 4),
                        "dtype": "f32 links/drift/cooling, f64 det renorm, reductions, measurement and control",
                        "roofline": mrf, "step_roofline": step_roofline(mx, "mixed", args.theta, args.ncool, dims),
                        "rooflines": mrfs}
        # the same workload recording every step's observables on the device
        rc = run_gpu(args, "fp64", with_timing=False, record=True)
        recd = rc["record"]
        out["recorded"] = {"value": round(rc["value"], 1), "ms_per_step": round(rc["ms_per_step"], 4),
                           "cost_vs_unrecorded": round(rc["ms_per_step"] / res["ms_per_step"] - 1.0, 4),
                           "what": "P, Q, S, d before/after cooling, eps, Kmax, alpha_ad of every step, "
                                   "device ring, no host synchronisation",
                           "last_steps": {"step": recd[-3:, 0].tolist(), "plaq_re": recd[-3:, 3].tolist(),
                                          "q_re": recd[-3:, 5].tolist(), "q_im": recd[-3:, 6].tolist(),
                                          "d": recd[-3:, 2].tolist()}}
        progress(f"recorded: {rc['value'] / 1e6:.1f} M link-updates/s")
    if args.precision == "fp64" and not args.no_extra:
        out["large_lattice"] = large_lattice(args)
        progress("32^4 leg done")
        out["theta_points"] = theta_points(args)
        progress("theta points done")
        out["mixed_vs_fp64"] = mixed_vs_fp64(args)
        progress("mixed vs FP64 trajectories done")
        out["theta_series"] = theta_series(args)
        progress("theta series done")
        out["cooling_modes"] = cooling_modes(args)
        progress("cooling modes done")
        out["chain"] = chain_workload(args)
    if args.served_runs > 0 and args.precision == "fp64":
        out["served"] = served(args, res["value"], args.served_runs, 0.7)
        progress("served mix at 0.7x done")
        # one stream three ways: batched all-mixed, batched all-FP64, FP64 one run at a time
        nv = max(1, args.served_runs // 2)
        out["served_all_mixed"] = served(args, res["value"], nv, 0.7, prec=1)
        progress("served all-mixed done")
        out["served_all_fp64"] = served(args, res["value"], nv, 0.7, prec=0)
        progress("served all-FP64 done")
        out["served_fp64_one_at_a_time"] = served_one_at_a_time(args, res["value"], nv, 0.7, prec=0)
        progress("served one at a time done")
        out["served_overload"] = served(args, res["value"], max(1, args.served_runs // 2), 1.5)
        progress("served mix at 1.5x done")
        out["served_alone_vs_batched"] = alone_vs_batched(args)
        progress("alone vs batched done")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args)
        progress("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

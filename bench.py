#!/usr/bin/env python3
"""Throughput of the DPD step (particle-steps/s) on one MI355X.

Workload: the large single-species fluid, L = 96 periodic, rho = 3
(2,654,208 particles), a = 25, gamma = 4.5, sigma = 3, dt = 0.04, FP32 forces
and velocities with FP64 positions, uniform random start (seeded, synthetic).

One step is the whole hot path: integrate-1, cell binning, pair force
F^C + F^D + F^R with Philox noise, bonds (none here), integrate-2.  The timed
region runs `--steps` consecutive steps with the state resident in HBM,
bracketed by HIP events on the library's stream.

Prints one JSON line: metric, value (median of five timed runs), roofline of
the dominant kernel and the CPU baseline (the FP64 oracle on the host cores, on
a bounded sample).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per particle-step in mixed precision: the persistent
# state (FP64 position 24 B, FP32 velocity 12 B and force 12 B, tag 4 B,
# type 4 B) read once and written once.
B_ALG_MIXED = 112.0
B_ALG_FP64 = 160.0
# Plain 32-bit VALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (lane-ops/s).
SIMDS = 256 * 4
CLOCK_HZ = 2.4e9
VALU_PEAK = SIMDS * 16 * CLOCK_HZ
# Algorithmic lane-op slots per particle of the gather formulation at rho = 3:
# 81 candidates x 8 (three differences, three 32x32->64 multiply-adds, one
# compare, one accumulate) + 12.57 in-range pairs x 86 (Philox4x32-10 40,
# uniforms and Box-Muller 18 with log/sqrt/cos at quarter rate, geometry and
# force 28).
OPS_PER_PARTICLE = 81 * 8 + 12.57 * 86
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_force_fluid_L96_traffic.md")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_force_fluid_L96_counters.md")
KERNEL_SOURCES = ["paper_1804_06205_amd/csrc/dpd_kernels.hip",
                  "paper_1804_06205_amd/csrc/dpd_device.hpp",
                  "paper_1804_06205_amd/csrc/dpd_kernels.hpp"]


def _profiled(path, key, variant):
    """`key` of a committed rocprofv3 summary of the fused kernel, if it was
    taken on these kernel sources and this brick."""
    import hashlib
    import re
    try:
        txt = open(path).read()
    except OSError:
        return None
    m = re.search(key + r"=([0-9.]+) variant=(\d+) sources_sha256=([0-9a-f]+)", txt)
    if not m:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != m.group(3) or int(m.group(2)) != variant:
        return None
    return float(m.group(1))


def measured_traffic(variant):
    """HBM bytes per launch of the fused kernel (FETCH_SIZE and WRITE_SIZE)."""
    return _profiled(TRAFFIC_FILE, "traffic_bytes_per_launch", variant)


def measured_valu(variant):
    """Issued VALU wave instructions per particle of the fused kernel (SQ_INSTS_VALU)."""
    return _profiled(COUNTERS_FILE, "valu_insts_per_particle", variant)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="fluid_L96",
                    choices=["fluid_L96", "fluid_L10", "melt_L32", "peptide_L40",
                             "replica_stream", "paper_sweep", "configs"])
    ap.add_argument("--window", type=int, default=100,
                    help="replica_stream: steps per batch window")
    ap.add_argument("--budget-gib", type=float, default=64.0,
                    help="replica_stream: device memory budget of the batch")
    ap.add_argument("--requests", type=int, default=512,
                    help="replica_stream: requests replayed")
    ap.add_argument("--no-serial", action="store_true",
                    help="replica_stream: skip the one-at-a-time baseline")
    ap.add_argument("--no-serving", action="store_true",
                    help="fluid_L96: skip the serving leg (the replica stream, batched "
                         "and one at a time)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--variant", type=int, default=None,
                    help="use this brick variant instead of autotuning")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many steps (for rocprofv3), print nothing else")
    return ap.parse_args()


def make_workload(name):
    from paper_1804_06205_amd import workloads as W
    return {"fluid_L96": W.cfg_fluid_L96, "fluid_L10": W.cfg_fluid_L10,
            "melt_L32": W.cfg_melt_L32, "peptide_L40": W.cfg_peptide_L40}[name]()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, budget_s):
    """The oracle (FP64, OpenMP) on the host cores, stepped until budget_s."""
    import oracle
    st = oracle.State.from_workload(w)
    steps = 0
    t0 = time.perf_counter()
    while True:
        st.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 1000:
            break
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": w.n * steps / el, "unit": "particle-steps/s", "cores": threads,
            "kind": "oracle", "host_cpu": _cpu_model(), "host_nproc": os.cpu_count(),
            "sample": f"{steps} step(s) of the same {w.name} box ({w.n} particles) after its "
                      f"initial force, FP64, {threads} OpenMP threads, {el:.1f} s"}


SERVING_KEYS = ("requests", "makespan_s", "particle_steps", "particle_steps_per_s",
                "replica_steps_per_s", "latency_p50_s", "latency_p99_s", "latency_max_s")


def serving_leg(args):
    """The serving half of the metric: the 512-request replica stream (Poisson
    arrivals at 200/s, L in 6..12, one 10-40 bead chain each, 1000-10000
    steps) served by continuous batching, and the same trace one replica at a
    time through dpd_step (first come first served).  The stream's batched
    throughput is its offered load while requests arrive; the same requests
    all present at once (`saturated`) give what the batch sustains."""
    from paper_1804_06205_amd import serve
    from paper_1804_06205_amd import workloads as W

    reqs = W.replica_stream()[: args.requests]
    budget = int(args.budget_gib * (1 << 30))
    serve.serve_batched(W.replica_stream(nreq=4, steps_range=(50, 100)), budget,
                        window=args.window, realtime=False)
    _, summ = serve.serve_batched(reqs, budget, window=args.window)
    out = {"workload": "replica_stream", "arrival_rate_per_s": 200.0, "L": [6, 12],
           "chain_beads": [10, 40], "steps": [1000, 10000], "window": args.window,
           "batched": {k: summ[k] for k in SERVING_KEYS}}
    out["batched"]["variant"] = summ["variant"]
    out["batched"]["graph_captures"] = summ["graph_captures"]
    _, sat = serve.serve_batched(reqs, budget, window=args.window, realtime=False)
    out["saturated"] = {k: sat[k] for k in ("requests", "makespan_s", "particle_steps_per_s",
                                            "replica_steps_per_s")}
    if not args.no_serial:
        _, s1 = serve.serve_one_at_a_time(reqs)
        out["one_at_a_time"] = {k: s1[k] for k in SERVING_KEYS}
        out["speedup_particle_steps"] = (summ["particle_steps_per_s"] /
                                         s1["particle_steps_per_s"])
        out["p99_ratio_one_at_a_time_over_batched"] = (s1["latency_p99_s"] /
                                                       summ["latency_p99_s"])
    return out


def replica_stream(args):
    """Continuous batching of the replica request stream (Poisson arrivals at
    200/s, L in 6..12, one 10-40 bead chain each, 1000-10000 steps), against
    the same trace served one replica at a time."""
    from paper_1804_06205_amd import serve
    from paper_1804_06205_amd import workloads as W

    reqs = W.replica_stream()[: args.requests]
    budget = int(args.budget_gib * (1 << 30))
    # Warm-up: the kernels' first launches and graph instantiation.
    serve.serve_batched(W.replica_stream(nreq=4, steps_range=(50, 100)), budget,
                        window=args.window, realtime=False)
    _, summ = serve.serve_batched(reqs, budget, window=args.window)
    line = {
        "metric": "particle-steps/s (batched replicas, rho=3)",
        "value": summ["particle_steps_per_s"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": int(sum(r.steps for r in reqs)),
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "replica_stream", "requests": len(reqs), "arrival_rate": 200.0,
                   "L": [6, 12], "chain_beads": [10, 40], "steps": [1000, 10000],
                   "precision": "FP32 forces/velocities, FP64 positions",
                   "window": args.window, "budget_bytes": budget},
        "serving": summ,
        "roofline": None,
    }
    _, sat = serve.serve_batched(reqs, budget, window=args.window, realtime=False)
    line["saturated"] = {k: sat[k] for k in ("requests", "makespan_s", "particle_steps_per_s",
                                             "replica_steps_per_s")}
    if not args.no_serial:
        _, s1 = serve.serve_one_at_a_time(reqs)
        line["one_at_a_time"] = s1
        line["speedup_vs_one_at_a_time"] = summ["particle_steps_per_s"] / s1["particle_steps_per_s"]
    print(json.dumps(line), flush=True)


# CAMUS times from the paper's performance section (ms per step, 2x Xeon
# E5-2640, rho = 3, a = 25): one thread, and the best thread count with that
# count.  Table 1: the fluid; Table 3: the same boxes with the alpha-helix
# model's 1-3 and 1-5 terms.
PAPER_TABLE1 = {5000: (10.1, 2.8, 12), 10000: (20.5, 5.1, 16), 50000: (99.0, 24.8, 12),
                100000: (194.5, 48.7, 8)}
PAPER_TABLE3 = {5000: (10.2, 2.8, 12), 10000: (20.8, 5.2, 8), 50000: (104.9, 25.9, 8),
                100000: (194.7, 49.4, 8)}


def cpu_baseline_ms(w, nthreads, gomp):
    """CPU baseline: the oracle (FP64, OpenMP) on nthreads host threads, ms per
    step after its initial force (at least 3 steps and 1 s)."""
    import oracle
    gomp.omp_set_num_threads(nthreads)
    st = oracle.State.from_workload(w)
    st.step(1)
    steps = 0
    t0 = time.perf_counter()
    while steps < 3 or time.perf_counter() - t0 < 1.0:
        st.step(1)
        steps += 1
    return (time.perf_counter() - t0) * 1e3 / steps


def _gpu_ms_per_step(g, steps, stream):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    g.step(steps)
    e1.record(stream)
    g.sync()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def paper_sweep(args):
    """The paper's benchmark boxes (rho = 3, a = 25, N = 5k..100k), each as the
    plain fluid (Table 1) and with ceil(0.03 N / 60) chains of the alpha-helix
    deck's bonds (Table 3): GPU ms/step through dpd_step and through a
    one-replica batch (graph-captured windows), and the oracle at one and at
    all host threads, with the paper's CAMUS times beside them.
    Acc = 100 T1 / T and Par = Acc / threads as in the paper's Eqs. 9-10,
    T1 = the oracle on one thread."""
    import ctypes
    import torch
    import oracle
    from paper_1804_06205_amd import dpd
    from paper_1804_06205_amd import workloads as W

    oracle.lib()                      # loads the OpenMP runtime the oracle uses
    gomp = ctypes.CDLL("libgomp.so.1")
    nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    stream = torch.cuda.Stream()
    rows = []
    for N in sorted(PAPER_TABLE1):
        for chains in (False, True):
            w = W.sweep_box(N, chains=chains)
            g = dpd.System.from_workload(w, stream=stream)
            g.step(args.warmup)
            g.sync()
            variant, _ = g.autotune(3)
            ms = _gpu_ms_per_step(g, args.steps, stream)
            g.close()
            # One replica through the batch path: K-step windows replayed as a graph.
            K = 100
            g = dpd.System.from_workload(w)
            with dpd.Batch(1 << 40, 1, variant=variant) as b:
                b.admit(g, 10 ** 7)
                b.advance(K)
                b.poll()
                t0 = time.perf_counter()
                nwin = max(1, args.steps // K)
                for _ in range(nwin):
                    b.advance(K)
                b.poll()
                ms_graph = (time.perf_counter() - t0) * 1e3 / (nwin * K)
            g.close()
            t_or = {nt: cpu_baseline_ms(w, nt, gomp) for nt in (1, nthreads)}
            gomp.omp_set_num_threads(nthreads)
            p1, pbest, pth = (PAPER_TABLE3 if chains else PAPER_TABLE1)[N]
            best = min(ms, ms_graph)
            rows.append({"N": N, "L": w.L[0], "table": 3 if chains else 1,
                         "chains": int(w.types.sum() // 60), "bonds": w.nbonds, "dt": w.dt,
                         "brick": list(dpd.variants()[variant][:3]),
                         "gpu_ms_per_step": ms, "gpu_graph_ms_per_step": ms_graph,
                         "gpu_particle_steps_per_s": N / best * 1e3,
                         "oracle_ms_1thread": t_or[1], "oracle_ms_all": t_or[nthreads],
                         "oracle_threads": nthreads,
                         "acc_gpu": 100.0 * t_or[1] / best,
                         "acc_oracle": 100.0 * t_or[1] / t_or[nthreads],
                         "par_oracle": 100.0 * t_or[1] / t_or[nthreads] / nthreads,
                         "paper_camus_ms_1thread": p1, "paper_camus_ms_best": pbest,
                         "paper_camus_best_threads": pth})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    top = [r for r in rows if r["table"] == 1][-1]
    line = {"metric": "particle-steps/s (paper box sizes, rho=3)",
            "value": top["gpu_particle_steps_per_s"], "unit": "particle-steps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": min(top["gpu_ms_per_step"], top["gpu_graph_ms_per_step"]),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "paper_sweep", "N": sorted(PAPER_TABLE1), "rho": 3, "a": 25.0,
                       "gamma": 4.5, "sigma": 3.0, "dt": [0.04, 0.02],
                       "precision": "FP32 forces/velocities, FP64 positions"},
            "sweep": rows, "roofline": None}
    print(json.dumps(line), flush=True)


CONFIG_SET = (("fluid_L10", 100), ("melt_L32", 1000), ("peptide_L40", 2000),
              ("fluid_L96", 500))


def configs(args):
    """Every benchmark workload at its full step count: time per step through
    dpd_step (eager launches) and, for the mixed-precision ones, through a
    one-replica batch whose windows of 100 steps replay a captured HIP graph;
    the fused kernel's share of the step (per-launch device times)."""
    import torch
    from paper_1804_06205_amd import dpd

    rows = []
    for name, steps in CONFIG_SET:
        w = make_workload(name)
        stream = torch.cuda.Stream()
        g = dpd.System.from_workload(w, stream=stream)
        g.step(args.warmup)
        g.sync()
        if w.precision == "mixed":
            variant, _ = g.autotune(3)
        else:
            variant = g.info().get("variant", None)
        ms = _gpu_ms_per_step(g, steps, stream)
        kt = g.step_profiled(min(steps, 200))
        obs = g.observables()
        g.close()
        row = {"workload": name, "particles": w.n, "steps": steps, "precision": w.precision,
               "us_per_step": ms * 1e3, "particle_steps_per_s": w.n / ms * 1e3,
               "fused_kernel_us": kt["ms_fused"] / max(1, kt["n_fused"]) * 1e3,
               "begin_kernel_us": kt["ms_begin"] / max(1, kt["n_begin"]) * 1e3,
               "fused_share": (kt["ms_fused"] / max(1, kt["n_fused"])) / ms,
               "final_kT": obs["kT"], "final_pressure": obs["pressure"]}
        if w.precision == "mixed":
            row["brick"] = list(dpd.variants()[variant][:3])
            K = 100
            g = dpd.System.from_workload(w)
            with dpd.Batch(1 << 40, 1, variant=variant) as b:
                b.admit(g, 10 ** 7)
                b.advance(K)
                b.poll()
                nwin = max(1, steps // K)
                t0 = time.perf_counter()
                for _ in range(nwin):
                    b.advance(K)
                b.poll()
                ms_graph = (time.perf_counter() - t0) * 1e3 / (nwin * K)
            g.close()
            row["graph_us_per_step"] = ms_graph * 1e3
            row["graph_gain"] = ms / ms_graph
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    line = {"metric": "particle-steps/s (DPD step, rho=3)", "value": rows[-1]["particle_steps_per_s"],
            "unit": "particle-steps/s", "n_gpus": 1, "steps": None, "warmup": args.warmup,
            "ms_per_step": rows[-1]["us_per_step"] / 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "configs", "set": [r["workload"] for r in rows]},
            "rows": rows, "roofline": None}
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    # The brick variant the autotuner picks is kept per class of system
    # (the library's DPD_TUNE_CACHE); a repeated run on a machine reuses it.
    os.environ.setdefault("DPD_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "dpd_tune.json"))
    os.makedirs(os.path.dirname(os.environ["DPD_TUNE_CACHE"]), exist_ok=True)
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is described, not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1804_06205_amd import dpd

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "replica_stream":
        replica_stream(args)
        return
    if args.workload == "paper_sweep":
        paper_sweep(args)
        return
    if args.workload == "configs":
        configs(args)
        return
    w = make_workload(args.workload)
    stream = torch.cuda.Stream()
    g = dpd.System.from_workload(w, stream=stream)
    if args.variant is not None:
        g.set_variant(args.variant)
    if args.profile_steps:
        g.step(args.profile_steps)
        g.sync()
        print(f"profiled {args.profile_steps} steps of {w.name}", flush=True)
        return

    g.step(args.warmup)
    g.sync()
    # The autotuner picks the brick shape (every shape gives bitwise the same
    # trajectory); it only times kernels on the current state.
    if args.variant is None:
        variant, _ = g.autotune(3)
    else:
        variant = args.variant
    torch.cuda.synchronize()
    # The timed region: `steps` consecutive steps, five times; the median run
    # is reported (the runs continue one trajectory).
    runs = []
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        g.step(args.steps)
        e1.record(stream)
        g.sync()
        torch.cuda.synchronize()
        runs.append(e0.elapsed_time(e1))
    ms = sorted(runs)[2]
    ms_step = ms / args.steps
    value = w.n * args.steps / (ms / 1e3)

    # Per-kernel device time of the same step sequence (events around each
    # launch, same stream).
    kt = g.step_profiled(args.steps)
    fused_ms = kt["ms_fused"] / max(1, kt["n_fused"])
    b_alg = B_ALG_FP64 if w.precision == "fp64" else B_ALG_MIXED
    achieved = b_alg * w.n / (fused_ms / 1e3) / 1e9
    alu = OPS_PER_PARTICLE * w.n / (fused_ms / 1e3)
    traffic = measured_traffic(variant) if w.name == "fluid_L96" else None
    valu = measured_valu(variant) if w.name == "fluid_L96" else None
    info = g.info()
    obs = g.observables()
    g.close()

    line = {
        "metric": "particle-steps/s (DPD step, rho=3)",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if w.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "particles": w.n, "box": list(w.L), "rho": 3,
                   "a": float(w.a[0, 0]), "gamma": w.gamma, "sigma": w.sigma, "dt": w.dt,
                   "precision": "FP32 forces/velocities, FP64 positions"
                   if w.precision == "mixed" else "FP64",
                   "cell_capacity": info["cell_capacity"],
                   "brick": list(dpd.variants()[variant][:3]),
                   "threads_per_block": dpd.variants()[variant][3]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "k_force (fused)", "kernel_ms": fused_ms,
                     "bytes_per_particle_step": b_alg,
                     "binding_roof": "alu: VALU issue (roofline_alu)"},
        "roofline_alu": {"bound": "alu", "achieved": alu / 1e12, "peak": VALU_PEAK / 1e12,
                         "unit": "Tlane-op/s", "frac": alu / VALU_PEAK,
                         "ops_per_particle_step": OPS_PER_PARTICLE,
                         # Issued VALU work (committed counter summary): the share of all
                         # SIMD issue slots the kernel's VALU instructions take.
                         "issued_valu_insts_per_particle": valu,
                         "valu_issue_frac": None if valu is None else
                         valu * 4 * w.n / (SIMDS * CLOCK_HZ * fused_ms / 1e3)},
        "kernel_ms": {"begin": kt["ms_begin"] / max(1, kt["n_begin"]), "fused": fused_ms,
                      "finish": kt["ms_finish"] / max(1, kt["n_finish"])},
        "final_kT": obs["kT"],
        "ms_per_step_runs": [r / args.steps for r in runs],
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    if w.name == "fluid_L96" and not args.no_serving:
        line["serving"] = serving_leg(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark of the 3D FD-LB solver on one MI355X.  Prints one JSON line.

Headline (`value`): MLUPS of the time step on the 256x128x128 shock-bubble
problem (planar shock of seeded Mach number into quiescent gas, a bubble or
droplet of seeded density ratio, inflow/outflow in x, reflecting walls in y
and z), FP32 storage and bulk arithmetic with the moments, temperature and
equilibrium in FP64,
synthetic seeded input already resident on the device.  A step is one time
step of the whole grid: the fused moments + equilibrium + NND convection +
dissipation + BGK update kernel and the boundary-layer kernel, replayed from
a captured graph.

Beside it:
  roofline      the fused step kernel's algorithmic HBM rate (15 reads + 15
                writes of f per node) over its mean launch time, measured with
                HIP events that each launch's dispatch records at its start
                and end, against the 8 TB/s peak;
                `traffic` is the counter-measured HBM bytes per launch from
                the committed rocprofv3 summary when it was taken on this
                kernel source, else null;
  copy_ceiling  the rate of a plain copy of the same bytes between two
                alternating buffers, the practical ceiling of such a kernel;
  accuracy_2000_steps  the headline problem over its full 2000 steps in
                FP64, FP32 with FP64 moments and equilibrium, and FP32: the
                FP32 modes' per-field error against the FP64 run;
  periodic_riemann  the 128^3 periodic 3D Riemann problem over its 1000
                steps in FP64, FP32 and FP32 with FP64 moments and
                equilibrium: MLUPS, kernel GB/s, the drift of the
                conserved totals and the FP32 modes' error against the
                FP64 run;
  batch         64 solves of uneven size, 500 steps each, in one persistent
                launch per step vs the same solves stepped one after another,
                and vs the plain one-at-a-time FP64 loop (with the batched
                results' error against it);
  serving       an open Poisson stream of 200 mixed solves through the
                continuous-batching server vs the plain one-at-a-time FP64
                loop: capacities and their ratio (also against the same
                loop in the served precision), and at 50%, 80% and 95% of
                the served capacity solves/s, p50/p99 time to solution
                (overall and per grid size), the server's tick counters and
                the served results' error against FP64 (top-level figures:
                80%);
  cpu_baseline  the FP64 oracle on the host cores (model, clock, count
                stated), median of three timings on a bounded sample.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--seed S]
                  [--no-batch] [--no-serve] [--no-cpu-baseline] [--copy-check]
                  [--batch-only] [--serve-requests N] [--stores auto|non-temporal|plain]
                  [--grid NX NY NZ]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, vendor figure
BYTES_PER_SITE = {"fp64": 240, "fp32": 120, "fp32_t64": 120}  # 15 reads + 15 writes of f
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_hbm_traffic.txt")
HEADLINE_GRID = (256, 128, 128)
KERNEL_SOURCES = ["lbm3d_tile.h", "lbm3d_model.h", "lbm3d_device.hip", "lbm3d_internal.h", "lbm3d_layout.cpp"]


def kernel_source_hash() -> str:
    """Hash of the step kernel's code: comments and whitespace are dropped,
    so only a change of the code itself invalidates the counter figures."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1010_4135_amd", "csrc", name)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update("".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(precision: str, stores: str):
    """Counter-measured HBM bytes per step-kernel launch from the committed
    summary, if it was taken on the current kernel source with the same
    precision and store kind."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if (kv.get("kernel_source_hash") != kernel_source_hash() or kv.get("precision") != precision
            or kv.get("stores") != stores):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_cpu():
    """Model, clock and core counts of the host this runs on."""
    model, mhz = "unknown", None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name") and model == "unknown":
                model = line.split(":", 1)[1].strip()
            elif line.startswith("cpu MHz") and mhz is None:
                mhz = float(line.split(":", 1)[1])
    except OSError:
        pass
    return {"cpu_model": model, "cpu_mhz": mhz, "nproc": os.cpu_count(),
            "affinity_cores": len(os.sched_getaffinity(0))}


def cpu_baseline(case, steps: int = 3, reps: int = 3):
    """The FP64 oracle on the host cores this process may use (its CPU
    affinity, capped by OMP_NUM_THREADS when set), on the same grid: one
    warm-up step, then `reps` timings of `steps` steps, median; and the same
    oracle on one thread (median of `reps` single steps)."""
    import oracle

    threads = len(os.sched_getaffinity(0))
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        threads = min(threads, int(os.environ["OMP_NUM_THREADS"]))
    used = oracle.set_threads(threads)
    o = oracle.Oracle(case.params)
    o.init(*case.fields)
    o.step(1)  # warm-up
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        o.step(steps)
        times.append(time.perf_counter() - t0)
    oracle.set_threads(1)
    times1 = []
    for _ in range(reps):
        t0 = time.perf_counter()
        o.step(1)
        times1.append(time.perf_counter() - t0)
    oracle.set_threads(used)
    out = {"value": round(case.sites * steps / float(np.median(times)) / 1e6, 3), "unit": "MLUPS", "cores": used,
           "kind": "oracle",
           "sample": f"{case.grid[0]}x{case.grid[1]}x{case.grid[2]} full grid, FP64, 1 warm-up step then "
                     f"{steps} steps timed {reps} times (median)",
           "single_thread_value": round(case.sites / float(np.median(times1)) / 1e6, 3),
           "timings_s": [round(t, 3) for t in times]}
    out.update(host_cpu())
    return out


def accuracy_full_length(lbm3d, inputs, metrics, seed: int, steps: int = 2000):
    """The headline problem run for its full 2000 steps in FP64, FP32 with
    FP64 moments and equilibrium, and plain FP32: per-field relative L1
    distance of the FP32 modes to the FP64 run (the FP64 mode itself is held
    to the FP64 oracle by the parity tests), health of each run."""
    case = inputs.shock_bubble(seed, precision="fp64")
    ref = None
    out = {"workload": f"shock_bubble {case.grid[0]}x{case.grid[1]}x{case.grid[2]}", "steps": steps}
    for prec in ("fp64", "fp32_t64", "fp32"):
        with lbm3d.Solver(dict(case.params, precision=prec)) as s:
            s.init(*case.fields)
            s.step(steps)
            m = s.moments(allow_nonfinite=True)
            health, _ = s.status()
        row = {"health": health}
        if prec == "fp64":
            ref = m
        else:
            row["rel_l1_vs_fp64"] = {k: float(f"{v:.3e}") for k, v in metrics.rel_l1(m, ref).items()}
        out[prec] = row
    return out


def batch_bench(lbm3d, inputs, metrics, seed: int, count: int = 64, steps: int = 500):
    """64 uneven solves: one persistent launch per step vs one solve at a time,
    both in FP32 with FP64 temperature recovery, and vs the plain FP64 loop
    (one solve at a time), with the batched results' error against it."""
    cases = inputs.batch_cases(seed, count=count, steps=steps, precision="fp32_t64")
    sites = sum(c.sites for c in cases)

    def fresh(precision=None):
        out = []
        for c in cases:
            s = lbm3d.Solver(c.params if precision is None else dict(c.params, precision=precision))
            s.init(*c.fields)
            out.append(s)
        return out

    solvers = fresh()
    tz = lbm3d.lbm3d_batch_tune([s.h for s in solvers], 5)  # tile depth from the autotuner
    lbm3d.lbm3d_batch_step([s.h for s in solvers], [1] * count)  # warm-up (plan, graph, code)
    t0 = time.perf_counter()
    lbm3d.lbm3d_batch_step([s.h for s in solvers], [steps] * count)
    t_batch = time.perf_counter() - t0
    f_batch = [s.get_f() for s in solvers[:4]]
    m_batch = [s.moments() for s in solvers]
    for s in solvers:
        s.close()
    solvers = fresh()
    for s in solvers:
        s.step(1)
        s.sync()
    t0 = time.perf_counter()
    for s in solvers:
        s.step(steps)
        s.sync()
    t_seq = time.perf_counter() - t0
    same = all(np.array_equal(a, s.get_f()) for a, s in zip(f_batch, solvers[:4]))
    for s in solvers:
        s.close()
    # the plain FP64 loop: each solve alone, the same steps (1 + steps, as above)
    solvers = fresh("fp64")
    for s in solvers:
        s.step(1)
        s.sync()
    t0 = time.perf_counter()
    for s in solvers:
        s.step(steps)
        s.sync()
    t_f64 = time.perf_counter() - t0
    err = max(metrics.max_rel_l1(a, s.moments()) for a, s in zip(m_batch, solvers))
    for s in solvers:
        s.close()
    return {"solves": count, "steps_each": steps, "sites_total": sites, "precision": "fp32_t64",
            "tile": [64, 8, tz], "tile_from": "autotuner",
            "batched_s": round(t_batch, 4), "sequential_s": round(t_seq, 4),
            "batched_mlups": round(sites * steps / t_batch / 1e6, 1),
            "sequential_mlups": round(sites * steps / t_seq / 1e6, 1),
            "speedup": round(t_seq / t_batch, 3), "first4_bitwise_equal_alone": bool(same),
            "fp64_loop_s": round(t_f64, 4), "speedup_vs_fp64_loop": round(t_f64 / t_batch, 3),
            "max_rel_l1_batched_vs_fp64": float(f"{err:.3e}")}


def conservation_drift(c0, c1) -> dict:
    """Change of the domain totals (mass, momentum, energy) between two
    reads: mass and energy relative to their first value, the largest
    momentum component's change per unit of the first mass (a velocity)."""
    return {"mass_relative": float(f"{(c1[0] - c0[0]) / c0[0]:.3e}"),
            "momentum_per_mass": float(f"{np.abs(c1[1:4] - c0[1:4]).max() / c0[0]:.3e}"),
            "energy_relative": float(f"{(c1[4] - c0[4]) / c0[4]:.3e}")}


def periodic_riemann_bench(lbm3d, inputs, metrics, seed: int, steps: int = 1000):
    """128^3 periodic 3D Riemann problem in each precision: MLUPS, the step
    kernel's algorithmic GB/s, the drift of the conserved totals over the
    run (on a periodic box every flux telescopes, so only rounding moves
    them), and the FP32 modes' per-field relative L1 distance to the FP64
    run after the same steps (the FP64 mode itself is held to the FP64
    oracle by the parity tests)."""
    out = {"workload": "riemann_3d 128^3 periodic", "steps": steps}
    ref = None
    for prec in ("fp64", "fp32", "fp32_t64"):
        case = inputs.riemann_3d(seed, precision=prec)
        s = lbm3d.Solver(case.params)
        s.init(*case.fields)
        s.tune(5)
        c0 = s.conserved()
        ms = s.step_timed(steps)
        c1 = s.conserved()
        m = s.moments()  # after exactly `steps` steps in every precision
        _, kms = s.step_profiled(20)
        bps = BYTES_PER_SITE[prec]
        s.close()
        row = {"mlups": round(case.sites * steps / (ms / 1e3) / 1e6, 1),
               "kernel_gbs": round(case.sites * bps / (kms / 1e3) / 1e9, 1),
               "conservation_drift": conservation_drift(c0, c1)}
        if prec == "fp64":
            ref = m
        else:
            row["rel_l1_vs_fp64"] = {k: float(f"{v:.3e}") for k, v in metrics.rel_l1(m, ref).items()}
        out[prec] = row
    return out


def _pct(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else None


def serve_bench(lbm3d, inputs, metrics, seed: int, count: int = 200):
    """Open Poisson stream of `count` mixed solves (one draw of requests for
    every load level; only the arrival times scale with the rate).

    - served capacity: every request submitted at once to the
      continuous-batching server (FP32 with FP64 moments and equilibrium);
    - baseline: the plain one-at-a-time FP64 loop over the same requests
      back to back (create, init, step, read back, free), which gives each
      request's service time, the FP64 results and the baseline capacity;
      the same loop in the served precision gives the capacity ratio at
      equal precision, and each of its results is compared bit for bit
      with the served one;
    - at 50%, 80% and 95% of the served capacity: the served path on the
      open stream, measured; the baseline's latencies are its measured
      service times replayed through the FIFO queue of the same arrival
      times (the loop serves one request at a time, so that replay is its
      schedule).  p50/p99 time to solution overall and per grid size,
      solves/s, and the server's tick counters."""
    base_trace = inputs.serve_trace(seed, count=count, rate=1.0)
    budget = int(200e9)

    def served(rate):
        with lbm3d.Server(budget, 64, tick_steps=32) as srv:
            t_start = time.perf_counter()
            tickets = []
            for t_arr, c in base_trace:
                delay = t_arr / rate - (time.perf_counter() - t_start)
                if delay > 0:
                    time.sleep(delay)
                tickets.append((srv.submit(c.params, c.fields, c.steps), c))
            res, lat = [], []
            for t, c in tickets:
                nx, ny, nz = c.grid
                rc, fields, tm = srv.wait(t, (nz, ny, nx))
                res.append(fields)
                lat.append(tm["t_done"] - tm["t_submit"])
            wall = time.perf_counter() - t_start
            st = srv.stats()
        return res, lat, wall, st

    # baseline: FP64, one request at a time, back to back
    service, base = [], []
    for _, c in base_trace:
        t0 = time.perf_counter()
        with lbm3d.Solver(dict(c.params, precision="fp64")) as s:
            s.init(*c.fields)
            s.step(c.steps)
            base.append(s.moments())
        service.append(time.perf_counter() - t0)
    base_capacity = count / sum(service)
    res_cap, _, w_cap, st_cap = served(1e12)
    capacity = count / w_cap
    # the same loop in the served precision, to separate what serving gains
    # from what FP32 storage gains; each result is compared bit for bit with
    # the served one (outside the loop's timing)
    t_same, same_bits = 0.0, 0
    for k, (_, c) in enumerate(base_trace):
        t0 = time.perf_counter()
        with lbm3d.Solver(dict(c.params, precision="fp32_t64")) as s:
            s.init(*c.fields)
            s.step(c.steps)
            m = s.moments()
        t_same += time.perf_counter() - t0
        same_bits += all(np.array_equal(a, b) for a, b in zip(m, res_cap[k]))
    del res_cap
    same_capacity = count / t_same
    out = {"requests": count, "served_precision": "fp32_t64",
           "baseline": "one solve at a time, FP64, arrival order; latencies from its measured service times "
                       "replayed through the FIFO queue of the arrival trace",
           "served_capacity_solves_per_s": round(capacity, 3),
           "baseline_capacity_solves_per_s": round(base_capacity, 3),
           "capacity_ratio": round(capacity / base_capacity, 3),
           "same_precision_loop_capacity_solves_per_s": round(same_capacity, 3),
           "capacity_ratio_same_precision": round(capacity / same_capacity, 3),
           "served_bitwise_equal_alone": f"{same_bits}/{count}",
           "capacity_run_busy_frac": round(st_cap["busy_s"] / max(w_cap, 1e-9), 3)}
    grids = sorted({c.grid for _, c in base_trace})
    levels = []
    for load in (0.5, 0.8, 0.95):
        rate = load * capacity
        res, lat_s, wall_s, st = served(rate)
        arr = [t / rate for t, _ in base_trace]
        lat_b, fin = [], 0.0
        for a, sv in zip(arr, service):
            fin = max(a, fin) + sv
            lat_b.append(fin - a)
        wall_b = fin
        err = max(metrics.max_rel_l1(a, b) for a, b in zip(res, base))
        row = {"load": load, "arrival_rate_per_s": round(rate, 3),
               "served_solves_per_s": round(count / wall_s, 3), "baseline_solves_per_s": round(count / wall_b, 3),
               "throughput_ratio": round(wall_b / wall_s, 3),
               "served_p50_s": round(_pct(lat_s, 50), 4), "served_p99_s": round(_pct(lat_s, 99), 4),
               "baseline_p50_s": round(_pct(lat_b, 50), 4), "baseline_p99_s": round(_pct(lat_b, 99), 4),
               "max_rel_l1_served_vs_fp64": float(f"{err:.3e}"),
               "server": {"ticks": st["ticks"], "rebuilds": st["rebuilds"], "evicted": st["evicted"],
                          "busy_frac": round(st["busy_s"] / max(st["wall_s"], 1e-9), 3),
                          "plan_s": round(st["plan_s"], 3), "admit_s": round(st["admit_s"], 3),
                          "finish_s": round(st["finish_s"], 3)}}
        by_grid = {}
        for g in grids:
            idx = [k for k, (_, c) in enumerate(base_trace) if c.grid == g]
            by_grid["x".join(map(str, g))] = {
                "n": len(idx),
                "served_p50_s": round(_pct([lat_s[k] for k in idx], 50), 4),
                "served_p99_s": round(_pct([lat_s[k] for k in idx], 99), 4),
                "baseline_p50_s": round(_pct([lat_b[k] for k in idx], 50), 4),
                "baseline_p99_s": round(_pct([lat_b[k] for k in idx], 99), 4)}
        row["by_grid"] = by_grid
        if load == 0.8:
            out.update({k: v for k, v in row.items() if k not in ("load", "by_grid")})
        levels.append(row)
    out["by_load"] = levels
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="fp32_t64", choices=["fp64", "fp32", "fp32_t64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--copy-check", action="store_true",
                    help="also run the checkpoint pack (a plain copy of 15 x nodes elements) for counter calibration")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--stores", choices=["auto", "non-temporal", "plain"], default="auto",
                    help="store kind of the headline's tiled step: the autotuner's choice (default), or "
                         "pinned after tuning (for profiles taken with a known kind)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched step of the 64-solve mix (--steps steps) and print its rate")
    ap.add_argument("--grid", type=int, nargs=3, default=list(HEADLINE_GRID), metavar=("NX", "NY", "NZ"),
                    help="grid of the shock-bubble workload (default: the headline 256 128 128); other grids "
                         "are for shape studies: no counter traffic and no CPU baseline are reported for them")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is a design note, not implemented", file=sys.stderr)
        sys.exit(2)

    from paper_1010_4135_amd import inputs, lbm3d, metrics

    if args.batch_only:
        # the batched step alone (for a profiler): the 64-solve mix, the
        # tuner's tile depth, one warm-up step, then --steps batched steps
        cases = inputs.batch_cases(args.seed, count=64, steps=args.steps, precision="fp32_t64")
        sites = sum(c.sites for c in cases)
        solvers = []
        for c in cases:
            s = lbm3d.Solver(c.params)
            s.init(*c.fields)
            solvers.append(s)
        tz = lbm3d.lbm3d_batch_tune([s.h for s in solvers], 5)
        lbm3d.lbm3d_batch_step([s.h for s in solvers], [1] * len(solvers))
        t0 = time.perf_counter()
        lbm3d.lbm3d_batch_step([s.h for s in solvers], [args.steps] * len(solvers))
        dt = time.perf_counter() - t0
        for s in solvers:
            s.close()
        print(json.dumps({"batch_only": True, "solves": len(cases), "sites_total": sites, "steps": args.steps,
                          "tile": [64, 8, tz], "batched_mlups": round(sites * args.steps / dt / 1e6, 1)}), flush=True)
        return

    headline = tuple(args.grid) == HEADLINE_GRID
    case = inputs.shock_bubble(args.seed, grid=tuple(args.grid), precision=args.precision)
    nx, ny, nz = case.grid
    s = lbm3d.Solver(case.params)
    s.init(*case.fields)
    # launch shape from the autotuner (state unchanged; outside the timed region)
    t_tune = time.perf_counter()
    s.tune(10)
    t_tune = time.perf_counter() - t_tune
    if args.stores != "auto":
        s.set_streaming(args.stores == "non-temporal")
    s.step(args.warmup)
    # runs of 32 steps replay a captured graph: capture it here, outside the
    # timed region (the state advances 32 more steps, untimed)
    graph_prep = 32 if args.steps >= 32 else 0
    if graph_prep:
        s.step(graph_prep)
    s.sync()
    # timed region: K steps replayed from captured graphs, HIP events on the
    # solver's stream, host clock around it
    t0 = time.perf_counter()
    ms = s.step_timed(args.steps)
    wall = time.perf_counter() - t0
    ms_per_step = ms / args.steps
    mlups = case.sites * args.steps / (ms / 1e3) / 1e6
    # per-launch duration of the fused step kernel (events recorded by each
    # launch's dispatch)
    _, kernel_ms = s.step_profiled(min(200, args.steps))
    health, done = s.status()
    if args.copy_check:
        for _ in range(3):
            s.get_f()
    by, tz = s.get_tile()
    stores = "non-temporal" if s.streaming() else "plain"
    bps = BYTES_PER_SITE[args.precision]
    achieved = case.sites * bps / (kernel_ms / 1e3) / 1e9
    out = {
        "metric": "MLUPS (lattice-site updates per second, 1e6) of the FD-LB time step",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"shock_bubble {nx}x{ny}x{nz}, {args.precision}" +
                        (" (FP32 f, FP64 moments, temperature and equilibrium)" if args.precision == "fp32_t64"
                         else ""),
            "grid": [nx, ny, nz], "precision": args.precision, "seed": args.seed,
            "mach": round(case.meta["mach"], 4), "density_ratio": round(case.meta["ratio"], 4),
            "tile": [64, by, tz], "tile_from": "autotuner", "tune_s": round(t_tune, 3),
            "stores": stores,
            "graph_capture_steps": graph_prep,
            "wall_s_timed_region": round(wall, 4), "health": health, "steps_done": done,
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": measured_traffic(args.precision, stores) if headline else None,
            "kernel": "k_step_tiled", "kernel_ms": round(kernel_ms, 5), "bytes_per_site": bps,
            "sites_per_launch": case.sites,
        },
    }
    s.close()
    # practical ceiling: a plain copy of the step's bytes (the f read per
    # step), alternating between two buffers as the step does
    copy_gbs = lbm3d.lbm3d_stream_copy_rate(case.sites * bps // 2, 10)
    out["copy_ceiling"] = {
        "what": "plain float4 copy of the bytes one step reads, alternating between two buffers",
        "GBps": round(copy_gbs, 1), "frac_of_peak": round(copy_gbs / PEAK_HBM_GBS, 4),
        "step_kernel_frac_of_copy": round(achieved / copy_gbs, 4),
    }
    if not args.no_batch:
        out["accuracy_2000_steps"] = accuracy_full_length(lbm3d, inputs, metrics, args.seed)
        out["periodic_riemann"] = periodic_riemann_bench(lbm3d, inputs, metrics, args.seed, steps=1000)
        out["batch"] = batch_bench(lbm3d, inputs, metrics, args.seed)
    if not args.no_serve:
        out["serving"] = serve_bench(lbm3d, inputs, metrics, args.seed, count=args.serve_requests)
    if not args.no_cpu_baseline and headline:
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

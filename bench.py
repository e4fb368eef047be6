"""Benchmark: Bellman (state,input) row-updates per second on one MI355X.

A step is one whole solve of the hot path on one synthetic problem already
resident on the device: labels, the per-solve 1-D tables, T_d Bellman
sweeps (rows recomputed on the fly; the first also takes the FP64 cut-off
tail) and the FP64 readout.  The headline workload is the 5-D room ring
(20^5 = 3.2M states, 10 heater levels, horizon 32, safety) solved with the
FP32 path; the plain FP64 path is timed beside it, both are checked against
the oracle at sampled states, and the 3-D unicycle reach-avoid workload
(100 x 100 x 60 states, 45 inputs, horizon 16) is timed after it.

Prints one JSON line (rank 0).  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

PEAK_FP32_TFLOPS = 157.3     # MI355X vector FP32 (packed), published
PEAK_FP64_TFLOPS = 78.6      # MI355X vector FP64, published
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E, published
C_ERFC = 20                  # flops charged per 1-D erfc evaluation

# HBM bytes per launch of the dominant sweep, from two profiler counter
# passes (FETCH_SIZE, WRITE_SIZE) scaled by what the same counters read for a
# 1 GiB device copy (x2.000 and x1.000), and the FP32 flops it executes per
# row (SQ_INSTS_VALU_FLOPS_FP32 x 64 / rows); recorded with a hash of the
# kernel's sources and reported only while the sources still hash to it.
TRAFFIC = {
    ("unicycle3d", "otf", "factored"): {"read": 4.276e+06, "write": 3.6e+06, "exec_flops_per_row": 44.91,
                                        "sha": "ebf5a84873e37ee5", "sources": ('amy_fixed.hip', 'amy_device.hpp', 'amy_plan.hpp')},
    ("unicycle3d-intersect", "otf", "factored"): {"read": 4.494e+06, "write": 3.6e+06, "exec_flops_per_row": 72.71,
                                                  "sha": "ebf5a84873e37ee5", "sources": ('amy_fixed.hip', 'amy_device.hpp', 'amy_plan.hpp')},
    ("room5d", "otf", "fixed"): {"read": 1.047e+08, "write": 2.68e+07, "exec_flops_per_row": 735.8,
                                 "sha": "ebf5a84873e37ee5", "sources": ('amy_fixed.hip', 'amy_device.hpp', 'amy_plan.hpp')},
    ("vehicle7d", "otf", "fixed"): {"read": 3.587e+07, "write": 1.258e+07, "exec_flops_per_row": 2831.1,
                                    "sha": "ebf5a84873e37ee5", "sources": ('amy_fixed.hip', 'amy_device.hpp', 'amy_plan.hpp')},
}


def _profiled(workload, mode, variant):
    """The profiler figures of this workload's sweep, if its sources still
    hash to the ones they were taken from."""
    import hashlib
    t = TRAFFIC.get((workload, mode, variant))
    if t is None:
        return None
    h = hashlib.sha256()
    for f in t["sources"]:
        with open(os.path.join(ROOT, "paper_2005_06191_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return t if h.hexdigest()[:16] == t["sha"] else None


def traffic_for(workload, mode, variant):
    t = _profiled(workload, mode, variant)
    return None if t is None else t["read"] + t["write"]


WORKLOADS = {
    "unicycle3d": lambda prec, mode: W.unicycle3d(precision=prec, mode=mode),
    "room5d": lambda prec, mode: W.room5d(precision=prec, mode=mode),
    "vehicle7d": lambda prec, mode: W.vehicle7d(precision=prec, mode=mode),
    "linear2d": lambda prec, mode: W.linear2d(precision=prec, mode=mode),
    # the robot of Sec. 7 with its disturbance (11 points): max over inputs of the min over disturbances
    "robot2d": lambda prec, mode: W.robot2d(precision=prec).with_(mode=mode),
    # the unicycle workload with the intersect window (no cell meeting [mu - x*, mu + x*] dropped)
    "unicycle3d-intersect": lambda prec, mode: W.unicycle3d(precision=prec, mode=mode).with_(window="intersect"),
    # the road traffic ring of Sec. 8.3.1 given as source text (compiled at run time), quantisation 0.74;
    # one lane per state (measured 4x faster here than the 64-lanes-per-state sweep AUTO takes for
    # windows of this size)
    "traffic5d-text": lambda prec, mode: W.traffic5d(q=0.74, precision=prec, text=True).with_(mode=mode,
                                                                                                variant="lanes"),
    # the room ring with beta(2, 2) noise on [-0.05, 0.05] (cells meeting the support)
    "room5d-beta": lambda prec, mode: W.room5d(precision=prec, mode=mode).with_(
        noise="beta", noise_a=(-0.05,) * 5, noise_b=(0.05,) * 5, noise_alpha=(2.0,) * 5, noise_beta=(2.0,) * 5),
}


def contraction_flops_per_row(plan) -> float:
    """Flops of one row's window sum done dimension by dimension (innermost
    first): a multiply-add per cell of each partial contraction,
    2 (W + W/L_n + W/(L_n L_{n-1}) + ... + L_1).  This is what the row
    must execute once its 1-D mass tables exist (the sweeps build those once
    per solve and share them between rows), so it is the per-row work the
    roofline fraction is priced on."""
    L = [x for x in plan["window"] if x > 0]
    f, w = 0.0, float(plan["W"])
    for l in reversed(L):
        f += 2.0 * w
        w /= l
    return f


def factored_flops_per_row(plan, n_fast) -> float:
    """The factored sweep's contraction per row: for each state and
    combination of the slow inputs, the outer dimensions' windows are
    contracted once for the U innermost cells that the fast input's windows
    can reach (2 (U W' + U W'/L_{n-2} + ... + U L_0) flops with
    W' = L_0 ... L_{n-2}, dimension by dimension), and each of the n_fast
    inputs then sums its own L_{n-1} of those U partial sums (2 L_{n-1}
    flops).  U = L_{n-1} + 3 for the compiled shapes (a fast-digit drift of
    at most two cells, plus one for rounding)."""
    L = [x for x in plan["window"] if x > 0]
    U = L[-1] + 3
    outer, w = 0.0, float(U * math.prod(L[:-1]))
    for l in reversed(L[:-1]):
        outer += 2.0 * w
        w /= l
    return outer / n_fast + 2.0 * L[-1]


def row_equivalent_flops_per_row(plan) -> float:
    """3W + C_erfc * edges: the per-row count of a sweep that builds every
    row's 1-D tables itself and multiplies each cell's mass out (a
    multiply-add with V and a mass product per window cell, one erfc per
    window edge, sum_i (L_i + 1) edges).  Sweeps that share tables or
    partial sums between rows execute fewer; reported beside the roofline,
    never as its fraction."""
    L = [x for x in plan["window"] if x > 0]
    edges = sum(l + 1 for l in L)
    return 3.0 * plan["W"] + C_ERFC * edges


def stored_bytes_per_row(plan, f64: bool) -> float:
    """Stored sweep: the row's W masses plus its int32 window origin."""
    return plan["W"] * (8 if f64 else 4) + 4


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q
    f, c = math.floor(k), math.ceil(k)
    return xs[f] + (xs[c] - xs[f]) * (k - f)


def run_solves(solver, steps, warmup):
    import torch
    for _ in range(warmup):
        solver.solve(policy=True, info=True)
    torch.cuda.synchronize()
    lat, main, sweeps, n_main = [], [], [], 0
    t0 = time.perf_counter()
    for _ in range(steps):
        r = solver.solve(policy=True, info=True)
        lat.append(r.info["t_total_ms"])
        main.append(r.info["t_main_sweeps_ms"])
        sweeps.append(r.info["t_sweeps_ms"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return dict(wall=wall, lat=lat, main=main, sweeps=sweeps, info=r.info, V=r.V)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(p, threads, budget_s):
    """Row-updates/s of the oracle's one-step routine at `threads` threads on
    about budget_s seconds of strided states (calibrated on a short run)."""
    import numpy as np

    import oracle
    n_cal = max(64, 200 * threads)
    st = np.linspace(0, p.n_x - 1, min(n_cal, p.n_x)).astype(np.int64)
    t = time.perf_counter()
    oracle.step(p, st, threads=threads)
    dt = max(time.perf_counter() - t, 1e-3)
    n = int(min(p.n_x, max(len(st), len(st) * budget_s / dt)))
    st = np.linspace(0, p.n_x - 1, n).astype(np.int64)
    t = time.perf_counter()
    oracle.step(p, st, threads=threads)
    dt = time.perf_counter() - t
    return n, dt


def cpu_baseline(p, budget_s=15.0, budget_1core_s=8.0):
    """The FP64 oracle, unchanged, on a bounded sample: one Bellman step
    (k = T_d) at evenly strided states, all inputs of each state, on every
    CPU this process may run on (capped by OMP_NUM_THREADS when it is set:
    the GPU job's CPU share), and again on one core."""
    cpus = len(os.sched_getaffinity(0))
    threads = cpus
    env = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    if env > 0:
        threads = min(threads, env)
    n, dt = _oracle_rate(p, threads, budget_s)
    n1, dt1 = _oracle_rate(p, 1, budget_1core_s)
    return {"value": n * p.n_u / dt, "unit": "row-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"one Bellman step from the terminal values at {n} evenly strided states x "
                      f"{p.n_u} inputs ({n * p.n_u} row-updates) of the same problem, {dt:.1f} s, "
                      f"FP64 oracle with {threads} OpenMP threads",
            "value_1core": n1 * p.n_u / dt1,
            "sample_1core": f"{n1} states x {p.n_u} inputs, {dt1:.1f} s, one thread",
            "host_cpus": cpus, "cpu_model": _cpu_model()}


def oracle_check_sampled(p32, V32, n_states=1000, seed=5, user=None):
    """Max |V - V_oracle| of the FP32 and FP64 solves at sampled states: the
    plain FP64 GPU path solves the same problem with one step fewer (its V
    at k = 1 is V_2 of the full horizon), the oracle takes the last Bellman
    step from it at the sampled states on its own, and both GPU results at
    k = 1 are compared with that."""
    import numpy as np

    import oracle
    import paper_2005_06191_amd as A
    T = p32.horizon
    p64 = p32.with_(precision="fp64")
    V64 = A.Solver(p64, user=user).solve(policy=False, info=False).V.cpu().numpy()
    Vn = A.Solver(p64.with_(horizon=T - 1), user=user).solve(policy=False, info=False).V.cpu().numpy()
    rng = np.random.default_rng(seed)
    st = np.unique(np.concatenate([rng.integers(0, p32.n_x, n_states), [0, p32.n_x - 1]]))
    Vr, _, _ = oracle.step(p32.with_(precision="fp64"), st, V_next=Vn)
    e32 = float(np.abs(V32[st] - Vr).max())
    e64 = float(np.abs(V64[st] - Vr).max())
    return {"fp32": e32, "fp64": e64, "states": int(len(st)), "tol_fp32": 1e-5, "tol_fp64": 1e-12,
            "ok": bool(e32 <= 1e-5 and e64 <= 1e-12),
            "how": "oracle's last Bellman step from the GPU FP64 V_2 at sampled states vs the GPU V_1"}


def bench_batch(args):
    """The 64-system batch in one persistent launch (FP32); value counts
    every system's rows x horizon."""
    import torch

    import paper_2005_06191_amd as A
    torch.cuda.set_device(0)
    ps = W.batch_systems()
    bs = A.BatchSolver(ps)
    tuned = None
    if args.tune:
        tuned = bs.tune()
    for _ in range(args.warmup):
        bs.solve(info=True)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = bs.solve(info=True)
        lat.append(res[0].info["t_total_ms"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    work = sum(p.rows * p.horizon for p in ps)
    flops = 0.0
    for p, r in zip(ps, res):
        flops += p.rows * p.horizon * contraction_flops_per_row(r.info)
    kms = statistics.mean(lat)
    achieved = flops / (kms * 1e-3) / 1e12
    variants = {}
    for r in res:
        variants[r.info["variant"]] = variants.get(r.info["variant"], 0) + 1
    # the alternative: the same systems solved one after another on one
    # stream, each with its own AUTO variant and its workspace allocated once
    solvers = [A.Solver(p) for p in ps]
    for _ in range(args.warmup):
        for sv in solvers:
            sv.solve(policy=False, info=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        for sv in solvers:
            sv.solve(policy=False, info=False)
    torch.cuda.synchronize()
    seq_ms = 1e3 * (time.perf_counter() - t1) / args.steps
    out = {
        "metric": "Bellman (state,input) row-updates/sec FP32 vs FP64 at <=1e-5 err; p50/p99",
        "value": work * args.steps / wall, "unit": "row-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch of {len(ps)} systems (2-D linear / 3-D unicycle), one persistent launch",
                   "systems": len(ps), "row_updates": work, "variants": variants, "tuned": tuned},
        "p50_ms": percentile(lat, 0.5), "p99_ms": percentile(lat, 0.99),
        "sequential_ms_per_pass": round(seq_ms, 3),
        "batch_speedup_vs_sequential": round(seq_ms / (1e3 * wall / args.steps), 3),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
                     "kernel": "k_batch_persistent (FP32)", "kernel_avg_ms": round(kms, 4)},
    }
    print(json.dumps(out), flush=True)


def copy_calibration(mib):
    """A plain device-to-device copy of known size (reads and writes mib MiB
    each), for scaling the HBM fetch/write counters of a profiler run."""
    import torch
    torch.cuda.set_device(0)
    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(10):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "launches": 10}), flush=True)


def _serve_run(srv, reqs, times, phase=""):
    """Submit reqs at the given offsets (s) and collect every result on a
    waiter thread; returns (wall_s, per-request latencies in ms).  Progress
    goes to stderr every 10 results."""
    import threading
    tickets, lat, err = [None] * len(reqs), [0.0] * len(reqs), []
    ready = threading.Semaphore(0)
    t_start = time.perf_counter()

    def waiter():
        for i in range(len(reqs)):
            ready.acquire()
            try:
                _, _, info = srv.wait(tickets[i], timeout_ms=-1)
                lat[i] = info["t_total_ms"]
            except Exception as e:  # noqa: BLE001 - reported below
                err.append(f"{reqs[i].name}: {e}")
            if (i + 1) % 10 == 0 or i + 1 == len(reqs):
                print(f"[serve] {phase}: {i + 1}/{len(reqs)} done at {time.perf_counter() - t_start:.1f} s",
                      file=sys.stderr, flush=True)

    th = threading.Thread(target=waiter)
    th.start()
    t0 = time.perf_counter()
    for i, (p, t) in enumerate(zip(reqs, times)):
        d = t0 + t - time.perf_counter()
        if d > 0:
            time.sleep(d)
        tickets[i] = srv.submit(p)
        ready.release()
    th.join()
    wall = time.perf_counter() - t0
    if err:
        raise RuntimeError("serving requests failed: " + "; ".join(err[:3]))
    return wall, lat


def bench_serve(args):
    """The serving stream: Poisson arrivals of FP32 solve requests (2-D
    linear, 3-D unicycle and 5-D room families with log-uniform state counts
    in [1e3, 2e6], plus 7-D vehicles at 2.1e6 states for 10%) into the
    continuous-batching server.  One request set is replayed three times:
    closed-loop (all queued at once) for the capacity, then open-loop with the
    stream's exponential gaps rescaled to 0.5 and 0.8 of that capacity.
    value = row-updates/s at load 0.8."""
    import numpy as np
    import torch

    import paper_2005_06191_amd as A
    torch.cuda.set_device(0)
    n, n_warm = args.requests, 10
    stream = W.serving_stream(count=n + n_warm)
    warm = [p for _, p in stream[:n_warm]]
    sample = [p for _, p in stream[n_warm:]]
    gaps = np.diff([stream[n_warm - 1][0]] + [t for t, _ in stream[n_warm:]])
    work = sum(p.rows * p.horizon for p in sample)
    budget = int(args.hbm_budget_gb * (1 << 30))
    loads = []
    with A.Server(hbm_budget_bytes=budget, max_slots=args.slots) as srv:
        _serve_run(srv, warm, [0.0] * len(warm), "warm-up")
        srv.reset_stats()
        wall, lat = _serve_run(srv, sample, [0.0] * n, "capacity")
        st = srv.stats()
        cap_qps = n / wall
        cap = {"wall_s": wall, "qps": cap_qps, "row_updates_per_s": work / wall,
               "p50_ms": percentile(lat, 0.5), "p99_ms": percentile(lat, 0.99),
               "max_active": st["max_active"], "hbm_peak_gb": st["hbm_peak"] / 2 ** 30}
        for rho in (0.5, 0.8):
            times = np.cumsum(gaps) - gaps[0]
            times = times / times[-1] * (n - 1) / (rho * cap_qps) if n > 1 else times
            srv.reset_stats()
            wall, lat = _serve_run(srv, sample, times.tolist(), f"load {rho}")
            st = srv.stats()
            loads.append({"load": rho, "offered_qps": rho * cap_qps, "wall_s": wall,
                          "row_updates_per_s": work / wall, "p50_ms": percentile(lat, 0.5),
                          "p99_ms": percentile(lat, 0.99), "mean_ms": statistics.mean(lat),
                          "max_active": st["max_active"], "steps": st["steps"],
                          "busy_frac": st["busy_s"] / wall})
    hi = loads[-1]
    fams = {}
    for p in sample:
        f = p.name.split("-")[1]
        fams[f] = fams.get(f, 0) + 1
    out = {
        "metric": "Bellman (state,input) row-updates/sec FP32 vs FP64 at <=1e-5 err; p50/p99",
        "value": hi["row_updates_per_s"], "unit": "row-updates/s", "n_gpus": 1, "steps": n,
        "warmup": n_warm, "ms_per_step": 1e3 * hi["wall_s"] / n, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serving stream: Poisson arrivals of FP32 requests, families 2-D/3-D/5-D "
                               "(n_x logU[1e3,2e6]) + 10% 7-D vehicle (2.1e6 states); value at load 0.8",
                   "requests": n, "row_updates": work, "families": fams,
                   "hbm_budget_gb": args.hbm_budget_gb, "max_slots": args.slots},
        "p50_ms": hi["p50_ms"], "p99_ms": hi["p99_ms"],
        "serve": {"capacity": cap, "loads": loads},
    }
    print(json.dumps(out), flush=True)


METRIC = "Bellman (state,input) row-updates/sec FP32 vs FP64 at <=1e-5 err; p50/p99"


def bench_solve(workload, mode, variant, steps, warmup, fp64=True, check=True):
    """Time `steps` whole FP32 solves of one workload (after `warmup`), the
    plain FP64 path beside it, and the roofline of the dominant sweep."""
    import torch

    import paper_2005_06191_amd as A
    p32 = WORKLOADS[workload]("fp32", mode)
    user = A.UserDynamics(p32.rhs, p32.n, p32.m, p32.p_dist) if p32.dyn == "user" else None
    s32 = A.Solver(p32, variant=variant if variant != "auto" else p32.variant, user=user)
    plan = s32.plan
    rows, T = p32.rows, p32.horizon
    r32 = run_solves(s32, steps, warmup)
    out = {"value": rows * T * steps / r32["wall"], "ms_per_step": 1e3 * r32["wall"] / steps,
           "p50_ms": percentile(r32["lat"], 0.5), "p99_ms": percentile(r32["lat"], 0.99),
           "config": {"workload": f"{p32.name} {p32.spec} {mode} (n_x={p32.n_x}, n_u={p32.n_u}, "
                                  + (f"n_w={p32.n_w}, " if p32.n_w > 1 else "") + f"T_d={T}, W={plan['W']})",
                      "states": p32.n_x, "inputs": p32.n_u, "horizon": T, "rows": rows,
                      "window": plan["window"][:p32.n], "W": plan["W"], "mode": mode,
                      "variant": plan["variant"]},
           "tail_bound_E": r32["info"]["tail_bound_E"]}
    # dominant kernel: the working-precision sweep alone, steps T_d - 1 .. 2
    # (T_d - 2 launches per solve), timed by HIP events on the solve's stream
    n_main = max(T - 2, 1)
    sweep_ms = statistics.mean(r32["main"]) / n_main
    prof = _profiled(workload, mode, plan["variant"])
    if mode == "otf":
        factored = plan["variant"] == "factored"
        fl = factored_flops_per_row(plan, p32.u_count[-1]) if factored else contraction_flops_per_row(plan)
        achieved = fl * rows / (sweep_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": traffic_for(workload, mode, plan["variant"]),
                "kernel": f"sweep {plan['variant']} (FP32)", "kernel_avg_ms": round(sweep_ms, 4),
                "launches_timed": n_main * steps, "flops_per_row": fl, "rows_per_launch": rows,
                "work": ("factored contraction: the outer windows once per state and slow-input "
                         "combination for the U cells the fast input reaches, 2 L_0 U (L_1 + 1) / n_fast "
                         "+ 2 L_2 flops per row" if factored else
                         "per-row window contraction done dimension by dimension, "
                         "2 (W + W/L_n + ... + L_1) flops; the 1-D tables are built once per solve"),
                "peak_without_packed_fp32": PEAK_FP64_TFLOPS,
                "frac_without_packed_fp32": round(achieved / PEAK_FP64_TFLOPS, 4),
                "row_equivalent": {"flops_per_row": row_equivalent_flops_per_row(plan),
                                   "tflops": round(row_equivalent_flops_per_row(plan) * rows
                                                   / (sweep_ms * 1e-3) / 1e12, 3)}}
        if prof is not None and "exec_flops_per_row" in prof:
            ex = prof["exec_flops_per_row"] * rows / (sweep_ms * 1e-3) / 1e12
            roof["executed"] = {"flops_per_row": prof["exec_flops_per_row"], "tflops": round(ex, 3),
                                "frac": round(ex / PEAK_FP32_TFLOPS, 4)}
            if prof["exec_flops_per_row"] < fl:
                # the sweep shares partial sums between rows: price on what runs
                roof["achieved"] = round(ex, 3)
                roof["frac"] = round(ex / PEAK_FP32_TFLOPS, 4)
                roof["frac_without_packed_fp32"] = round(ex / PEAK_FP64_TFLOPS, 4)
                roof["work"] = ("executed FP32 flops per row from the profiler's counters (the sweep "
                                "shares partial sums between inputs, so it runs fewer than the "
                                "per-row contraction)")
    else:
        by = stored_bytes_per_row(plan, False)
        achieved = by * rows / (sweep_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": traffic_for(workload, mode, plan["variant"]),
                "kernel": "k_sweep_stored (FP32)", "kernel_avg_ms": round(sweep_ms, 4),
                "launches_timed": n_main * steps, "bytes_per_row": by, "rows_per_launch": rows}
    out["roofline"] = roof
    if fp64:
        s64 = A.Solver(p32.with_(precision="fp64"), variant=variant if variant != "auto" else p32.variant, user=user)
        k64 = max(3, steps // 2)
        r64 = run_solves(s64, k64, 1)
        v64 = rows * T * k64 / r64["wall"]
        err = float((r32["V"] - r64["V"]).abs().max().item())
        out["fp64"] = {"value": v64, "ms_per_step": 1e3 * r64["wall"] / k64,
                       "p50_ms": percentile(r64["lat"], 0.5), "p99_ms": percentile(r64["lat"], 0.99)}
        out["speedup_fp32_vs_fp64"] = out["value"] / v64
        out["max_abs_err_fp32_vs_fp64"] = err
        del s64
    if check:
        out["err_vs_oracle"] = oracle_check_sampled(p32, r32["V"].cpu().numpy(), user=user)
    del s32
    torch.cuda.synchronize()
    return out, p32


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="room5d", choices=sorted(WORKLOADS) + ["batch64", "serve"])
    ap.add_argument("--also", default="unicycle3d,robot2d,unicycle3d-intersect,traffic5d-text,room5d-beta",
                    help="comma-separated workloads timed after the headline one ('' for none)")
    ap.add_argument("--requests", type=int, default=200, help="serve: requests in the measured set")
    ap.add_argument("--slots", type=int, default=64, help="serve: requests on the device at once")
    ap.add_argument("--hbm-budget-gb", type=float, default=64.0, help="serve: device arena")
    ap.add_argument("--tune", action="store_true", help="run the autotuner before timing")
    ap.add_argument("--mode", default="otf", choices=["otf", "stored"])
    ap.add_argument("--variant", default="auto", choices=["auto", "lanes", "fixed", "group16", "group64", "factored"])
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="only run a plain device copy of this size 10 times (HBM counter calibration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-oracle-check", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (the solve is not sharded across GPUs); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.copy_calib_mib > 0:
        copy_calibration(args.copy_calib_mib)
        return
    if args.workload == "batch64":
        bench_batch(args)
        return
    if args.workload == "serve":
        bench_serve(args)
        return

    import torch
    torch.cuda.set_device(0)
    head, p32 = bench_solve(args.workload, args.mode, args.variant, args.steps, args.warmup,
                            fp64=not args.no_fp64, check=not args.no_oracle_check)
    print(f"[bench] {args.workload}: {head['value']:.4g} row-updates/s", file=sys.stderr, flush=True)
    out = {"metric": METRIC, "value": head.pop("value"), "unit": "row-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": head.pop("ms_per_step"),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic", "config": head.pop("config")}
    out.update(head)
    if "max_abs_err_fp32_vs_fp64" in out:
        out["err_tol"] = 1e-5
        out["err_ok"] = bool(out["max_abs_err_fp32_vs_fp64"] <= 1e-5 and
                             out.get("err_vs_oracle", {}).get("ok", True))
    also = {}
    for w in [x for x in args.also.split(",") if x and x != args.workload]:
        r, pw = bench_solve(w, "otf", "auto", args.steps, args.warmup, fp64=not args.no_fp64,
                            check=not args.no_oracle_check)
        r["config"]["features"] = {"disturbance_points": pw.n_w, "noise": pw.noise, "window": pw.window,
                                   "dynamics": pw.dyn}
        print(f"[bench] {w}: {r['value']:.4g} row-updates/s", file=sys.stderr, flush=True)
        also[w] = r
    if also:
        out["also"] = also
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p32.with_(precision="fp64"))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark: Deep Greedy Switching on one MI355X.

Default: one step = one full DGS solve (greedy start, layout, difference
evaluation of every agent, switching until no improving 2-exchange is
left) of the n = 16384 low-rank-plus-noise instance, with the benefit
matrix already resident in HBM.  Prints one JSON line; the line also
carries a short measurement of the batched workload (512 instances in one
graph replay of three launches, against a loop of single-instance solves).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Other workloads: lowrank4096, uniform256 (single instances), batched512
(the batched workload as the step) and serving (Poisson arrivals at
200/s for --serve-seconds, continuous batching against a plain
one-request-at-a-time loop).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "LSAP instances/sec and n=16384 solve ms (HBM % of peak); serving p50/p99 latency"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure

SINGLE = {
    "lowrank16384": dict(n=16384, generator="round((1000*u_i)*c_j)+noise, u,c~U(0.1,1), noise~U{0..99}"),
    "lowrank4096": dict(n=4096, generator="round((1000*u_i)*c_j)+noise, u,c~U(0.1,1), noise~U{0..99}"),
    "uniform256": dict(n=256, generator="iid uniform int32 in [0,1000)"),
    "geom4096": dict(n=4096, generator="GEOM: rounded Euclidean distances of random points in [0,1000]^2"),
    "geom16384": dict(n=16384, generator="GEOM: rounded Euclidean distances of random points in [0,1000]^2"),
}
WORKLOADS = sorted(SINGLE) + ["batched512", "serving"]

KERNELS = {"range": "k_range_check", "init": "k_greedy_pipe",
           "layout": "k_transpose+k_permuted+k_benefits", "scan": "k_scan_pairs+k_scan_reduce",
           "switch": "k_switch_v3"}
KERNEL_SOURCES = {"k_switch_v3": "dgs_switch3.hip", "k_scan_pairs+k_scan_reduce": "dgs_scan.hip",
                  "k_batch": "dgs_batch.hip"}


def algorithmic_bytes(phase: str, n: int, switches: int, rescans: int) -> int:
    """Bytes a phase must move at minimum (int32 entries), per solve."""
    nn = n * n
    if phase == "range":
        return 4 * nn  # read every entry once
    if phase == "init":
        return 4 * nn  # greedy reads every entry once
    if phase == "layout":
        return 16 * nn  # transpose and the permuted copy W (each read + write)
    if phase == "scan":
        return 4 * nn  # every exchange pair (i, k) needs a_i,tau(k) and a_k,tau(i) once
    if phase == "switch":
        # per switch: the two changed candidates of every agent need 4 entries
        # each (16n B)
        return 16 * n * switches
    raise KeyError(phase)


def reevaluation_bytes(n: int, rescans: int) -> int:
    """Bytes of the switching loop's own full re-evaluations of agents (two
    rows each, 8n B): a cost of this design's exact rule, reported beside the
    per-switch figure and not counted in it."""
    return 8 * n * rescans


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this kernel and workload, scaled by the copy-kernel calibration; None
    when there is none or the kernel's source changed since it was taken."""
    src = KERNEL_SOURCES.get(kernel)
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_hbm_counters.txt")
    if src is None or not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                fields[k.strip()] = v.strip()
    with open(os.path.join(ROOT, "paper_1106_5694_amd", "csrc", src), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != fields.get("source_sha256"):
            return None
    try:
        return int(float(fields["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _estimate(oracle, A, switches: int, budget_s: float, probe: int) -> tuple:
    """Seconds per solve of the oracle at its current thread count: greedy +
    first full evaluation timed, then a sample of switches sized to the
    budget, extrapolated linearly to all switches.  Returns (est, sampled)."""
    t0 = time.perf_counter()
    tau0 = oracle.greedy(A)
    t_greedy = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.dgs_incr(A, init=tau0, max_switches=0)
    t_scan = time.perf_counter() - t0
    k = min(switches, probe)
    t0 = time.perf_counter()
    oracle.dgs_incr(A, init=tau0, max_switches=k)
    per = max(time.perf_counter() - t0 - t_scan, 1e-9) / max(k, 1)
    k2 = int(min(switches, max(k, (budget_s - t_greedy - 2 * t_scan) / per)))
    if k2 > k:
        t0 = time.perf_counter()
        oracle.dgs_incr(A, init=tau0, max_switches=k2)
        per = max(time.perf_counter() - t0 - t_scan, 1e-9) / k2
        k = k2
    return t_greedy + t_scan + per * switches, k


def cpu_baseline(A, switches: int, seed: int, budget_s: float = 12.0) -> dict:
    """Time the CPU oracle on bounded samples: the headline instance on all
    host threads (the reported baseline) and on one thread, and complete
    solves of the n = 4096 instance of the same generator on both."""
    import oracle
    from workloads import gen

    threads = oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    est, k = _estimate(oracle, A, switches, budget_s, 200)
    oracle.set_threads(1)
    est1, k1 = _estimate(oracle, A, switches, budget_s / 2, 50)
    A4 = gen.lowrank_matrix(4096, seed)
    full4096 = {}
    for th in (1, threads):
        oracle.set_threads(th)
        t0 = time.perf_counter()
        r4 = oracle.dgs_incr(A4)
        full4096[f"threads_{th}"] = round(time.perf_counter() - t0, 3)
    # the definitional oracle (every agent re-evaluated from scratch after every
    # switch), one thread, on the n = 1024 instance of the same generator
    A1 = gen.lowrank_matrix(1024, seed)
    oracle.set_threads(1)
    t0 = time.perf_counter()
    r1 = oracle.dgs_full(A1)
    defin = {"n": 1024, "threads": 1, "seconds": round(time.perf_counter() - t0, 3), "switches": int(r1["S"])}
    oracle.set_threads(threads)
    return {
        "value": 1.0 / est,
        "unit": "instances/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"greedy + first full evaluation + first {k} of {switches} switches of the same "
                   f"instance (C oracle, incremental re-evaluation, {threads} OpenMP threads), "
                   f"extrapolated linearly to all switches: est. {est:.2f} s per solve"),
        "cpu_model": cpu_model(),
        "nproc": os.cpu_count(),
        "single_thread": {"est_s_per_solve": round(est1, 3), "switches_sampled": k1},
        "lowrank4096_full_solve_s": full4096,
        "lowrank4096_switches": int(r4["S"]),
        "definitional_full_rescan": defin,
    }


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def base_line(args, value: float, unit: str, ms_per_step: float, config: dict) -> dict:
    return {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": unit,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": config,
    }


def spec_n(workload: str) -> int:
    return SINGLE[workload]["n"]


def run_single(args, dgs, torch, gen, np) -> dict:
    spec = SINGLE[args.workload]
    n = spec["n"]
    t0 = time.perf_counter()
    A = gen.single_instance(args.workload, args.seed)
    log(f"generated {args.workload} seed {args.seed} in {time.perf_counter() - t0:.1f} s")
    Ad = torch.from_numpy(A).to(torch.device("cuda:0"))
    torch.cuda.synchronize()
    for w in range(args.warmup):
        _, res = dgs.solve(Ad, profile=True)
        log(f"warmup {w}: {res['device_ms']:.2f} ms device, S={res['switches']}")
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        tau, res = dgs.solve(Ad, profile=True)
        results.append(res)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    S = results[-1]["switches"]
    rescans = results[-1]["rescans"]
    phases = {}
    for p in dgs.PHASES:
        ms = float(np.mean([r["phase_ms"][p] for r in results]))
        byts = algorithmic_bytes(p, n, S, rescans)
        gbs = byts / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        phases[p] = {"ms": round(ms, 4), "algorithmic_bytes": byts, "GB/s": round(gbs, 1),
                     "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    dominant = max(phases, key=lambda p: phases[p]["ms"])
    d = phases[dominant]
    kernel = KERNELS[dominant]
    roofline = {"bound": "hbm", "achieved": d["GB/s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": d["hbm_frac"], "traffic": measured_traffic(kernel, args.workload),
                "kernel": kernel, "phase": dominant, "algorithmic_bytes_per_launch": d["algorithmic_bytes"],
                "avg_launch_ms": d["ms"]}
    if dominant == "switch":
        extra = reevaluation_bytes(n, rescans)
        gbs = (d["algorithmic_bytes"] + extra) / (d["ms"] * 1e-3) / 1e9
        roofline["bytes_basis"] = "16n B per switch (the two changed candidates of every agent)"
        roofline["incl_reevaluation"] = {"bytes": d["algorithmic_bytes"] + extra, "GB/s": round(gbs, 1),
                                         "frac": round(gbs / HBM_PEAK_GBS, 4),
                                         "basis": "plus 8n B per full re-evaluation of an agent"}
    config = {"workload": args.workload, "n": n, "seed": args.seed, "generator": spec["generator"],
              "start": "greedy", "switches": S, "rescans": rescans,
              "initial_benefit": results[-1]["initial_benefit"], "total_benefit": results[-1]["total_benefit"],
              "device_ms": round(float(np.mean([r["device_ms"] for r in results])), 3)}
    line = base_line(args, args.steps / wall, "instances/s", 1000.0 * wall / args.steps, config)
    line["roofline"] = roofline
    line["phases"] = phases
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        line["cpu_baseline"] = cpu_baseline(A, S, args.seed)
    del Ad, tau
    torch.cuda.synchronize()
    return line


def run_parallel(args, dgs, torch, gen, np, steps: int = 3) -> dict:
    """Parallel DGS (Algorithm 3 with Check Conflicts) on the same instance:
    every round applies all non-conflicting improving exchanges at once.
    A different trajectory from the steepest-ascent solve, so its own
    objective and switch count; reported beside the headline line."""
    A = gen.single_instance(args.workload, args.seed)
    Ad = torch.from_numpy(A).to(torch.device("cuda:0"))
    _, res = dgs.solve(Ad, profile=True, parallel=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for _ in range(steps):
        _, res = dgs.solve(Ad, profile=True, parallel=True)
        results.append(res)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    r = results[-1]
    out = {"ms_per_solve": round(1000.0 * wall / steps, 3), "instances_per_s": round(steps / wall, 3),
           "rounds": r["rounds"], "switches": r["switches"], "initial_benefit": r["initial_benefit"],
           "total_benefit": r["total_benefit"],
           "phase_ms": {p: round(float(np.mean([x["phase_ms"][p] for x in results])), 4) for p in dgs.PHASES}}
    del Ad
    return out


def run_lazy(args, dgs, torch, gen, np, steps: int = 2) -> dict:
    """Lazy DGS (Algorithm 1 with stale stored bests: stale agent and job bests, the
    paper's branch rule and improvement guard) on the same instance; its own
    trajectory, objective and switch count, reported beside the headline."""
    A = gen.single_instance(args.workload, args.seed)
    Ad = torch.from_numpy(A).to(torch.device("cuda:0"))
    _, res = dgs.solve(Ad, profile=True, lazy=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for _ in range(steps):
        _, res = dgs.solve(Ad, profile=True, lazy=True)
        results.append(res)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    r = results[-1]
    out = {"ms_per_solve": round(1000.0 * wall / steps, 3), "instances_per_s": round(steps / wall, 3),
           "passes": r["rounds"], "attempts": r["attempts"], "switches": r["switches"],
           "initial_benefit": r["initial_benefit"], "total_benefit": r["total_benefit"],
           "phase_ms": {p: round(float(np.mean([x["phase_ms"][p] for x in results])), 4) for p in dgs.PHASES}}
    del Ad
    return out


def run_rect(args, dgs, torch, gen, np, steps: int = 2) -> dict:
    """Rectangular DGS (dgs_solve_rect): the first 3n/4 rows of the workload
    as providers against all n columns as receivers, so a quarter of the jobs
    stay unassigned and moves to them are live.  Steepest ascent; reported
    beside the headline line."""
    A = gen.single_instance(args.workload, args.seed)
    n_rows = 3 * A.shape[0] // 4
    Ad = torch.from_numpy(np.ascontiguousarray(A[:n_rows])).to(torch.device("cuda:0"))
    del A
    _, res = dgs.solve_rect(Ad, profile=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, res = dgs.solve_rect(Ad, profile=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {"agents": n_rows, "jobs": int(Ad.shape[1]), "ms_per_solve": round(1000.0 * wall / steps, 3),
           "switches": res["switches"], "initial_benefit": res["initial_benefit"],
           "total_benefit": res["total_benefit"], "device_ms": round(res["device_ms"], 3),
           "memory": "n x m matrix and its transpose; unassigned jobs held by virtual agents (no m x m buffer)"}
    # the same instance from the global greedy start (largest remaining entry first)
    dgs.solve_rect(Ad, global_greedy=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, res = dgs.solve_rect(Ad, profile=True, global_greedy=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out["global_greedy_start"] = {"ms_per_solve": round(1000.0 * wall / steps, 3), "switches": res["switches"],
                                  "initial_benefit": res["initial_benefit"], "total_benefit": res["total_benefit"],
                                  "start_ms": round(res["phase_ms"]["init"], 3)}
    del Ad
    return out


def run_batched(args, dgs, torch, gen, np, steps: int, warmup: int, count: int = 512) -> dict:
    """The batched workload: `count` instances, n log-uniform in [64, 2048],
    iid uniform benefits in [0, 10000), solved by one replay per step of a
    captured graph of three launches (greedy starts with the transposes,
    evaluation, switching); against a loop of single-instance solves of the
    same device-resident instances."""
    t0 = time.perf_counter()
    ns = [int(n) for n in gen.loguniform_sizes(count, 64, 2048, args.seed)]
    As = gen.batch_instances(count, 64, 2048, args.seed)
    log(f"generated {count} batched instances in {time.perf_counter() - t0:.1f} s")
    plan = dgs.BatchPlan(ns, autotune=True)
    _, first = plan.run(As, outs=False)  # upload, tune, capture
    for _ in range(warmup):
        plan.run(None, outs=False)
    ms, walls = [], []
    for _ in range(max(steps, 10)):  # per-batch wall times; the median is reported
        t0 = time.perf_counter()
        _, res = plan.run(None, outs=False)
        walls.append(time.perf_counter() - t0)
        ms.append(res[0]["device_ms"])
    wall = float(np.median(walls))
    block, grid = plan.config()
    plan.close()

    # the plain per-instance solver on the same GPU, inputs resident in HBM
    Ads = [torch.from_numpy(A).to("cuda:0") for A in As]
    torch.cuda.synchronize()
    for A in Ads[:8]:
        dgs.solve(A)
    t1 = time.perf_counter()
    single = [dgs.solve(A)[1] for A in Ads]
    torch.cuda.synchronize()
    wall1 = time.perf_counter() - t1
    same = all(a["total_benefit"] == b["total_benefit"] and a["switches"] == b["switches"]
               for a, b in zip(first, single))
    del Ads
    torch.cuda.synchronize()
    entries = sum(n * n for n in ns)
    launch_ms = float(np.mean(ms))
    gbs = 4 * entries / (launch_ms * 1e-3) / 1e9
    return {
        "instances": count, "n_range": [64, 2048], "sum_n2": entries,
        "instances_per_s": round(count / wall, 2),
        "ms_per_batch": round(1000.0 * wall, 3),
        "batches_timed": len(walls),
        "device_ms_per_batch": round(float(np.median(ms)), 3),
        "per_instance_solver": {"instances_per_s": round(count / wall1, 2),
                                "ms_per_batch": round(1000.0 * wall1, 3)},
        "speedup_vs_per_instance": round((count / wall) / (count / wall1), 2),
        "results_identical": bool(same),
        "autotuned": {"block": block, "grid": grid},
        "roofline": {"bound": "hbm",
                     "kernel": "k_batch (k_batch_solve<., 0> with the transposes, k_batch_pairs, "
                               "k_batch_solve<., 1>: one graph replay)",
                     "achieved": round(gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "algorithmic_bytes_per_launch": 4 * entries,
                     "bytes_basis": "every benefit matrix read once", "avg_launch_ms": round(launch_ms, 3),
                     "traffic": measured_traffic("k_batch", "batched512")},
    }


def serving_pool(args, gen, size: int = 64):
    """Distinct low-rank instances with sizes log-uniform in [128, 16384]
    (pool instance p is seeded by (seed, p)); requests cycle through them."""
    _, pool_ns = gen.serving_trace(1.0, 200.0, 128, 16384, args.seed, size)
    t0 = time.perf_counter()
    pool = [gen.lowrank_matrix(int(n), args.seed * 1_000_003 + p) for p, n in enumerate(pool_ns)]
    log(f"generated the request pool ({len(pool)} instances, {sum(A.nbytes for A in pool) / 1e9:.2f} GB) "
        f"in {time.perf_counter() - t0:.1f} s")
    return pool


def _serve_continuous(dgs, pool, reqs) -> dict:
    """The continuous-batching server (dgs_server_*) on an arrival trace."""
    with dgs.Server() as srv:
        start = time.perf_counter()
        tickets = []
        for t, p in reqs:
            now = time.perf_counter() - start
            if t > now:
                time.sleep(t - now)
            tickets.append(srv.submit(pool[p]))
        for k, tk in enumerate(tickets):
            assert srv.wait(tk) is not None
            if (k + 1) % 500 == 0:
                log(f"serving: {k + 1} of {len(tickets)} requests done")
        st = srv.stats()
    return {"requests": int(st["completed"]), "completed_per_s": round(st["inst_per_s"], 2),
            "p50_us": round(st["p50_us"], 1), "p99_us": round(st["p99_us"], 1),
            "wall_s": round(time.perf_counter() - start, 2)}


def _serve_plain(dgs, np, pool, reqs) -> dict:
    """A plain loop that solves one request at a time (dgs_solve), in arrival
    order, on the same arrival trace; latency = arrival to result."""
    lat, queue, finished = [], [], []
    cv = threading.Condition()

    def worker():
        while True:
            with cv:
                while not queue:
                    cv.wait()
                item = queue.pop(0)
            if item is None:
                return
            t_arr, p = item
            dgs.solve(pool[p])
            finished.append(time.perf_counter())
            lat.append(finished[-1] - t_arr)
            if len(lat) % 500 == 0:
                log(f"serving: plain loop, {len(lat)} requests done")

    th = threading.Thread(target=worker)
    th.start()
    start = time.perf_counter()
    first_arrival = None
    for t, p in reqs:
        now = time.perf_counter() - start
        if t > now:
            time.sleep(t - now)
        with cv:
            t_arr = time.perf_counter()
            if first_arrival is None:
                first_arrival = t_arr
            queue.append((t_arr, p))
            cv.notify()
    with cv:
        queue.append(None)
        cv.notify()
    th.join()
    lat_us = np.asarray(lat) * 1e6
    return {"requests": len(lat),
            "completed_per_s": round(len(lat) / max(finished[-1] - first_arrival, 1e-9), 2),
            "p50_us": round(float(np.percentile(lat_us, 50)), 1),
            "p99_us": round(float(np.percentile(lat_us, 99)), 1),
            "wall_s": round(time.perf_counter() - start, 2)}


def run_serving(args, dgs, gen, np, pool, rate: float, seconds: float) -> dict:
    """Poisson arrivals at `rate` per second for `seconds`, n log-uniform in
    [128, 16384], low-rank-plus-noise benefits; the continuous-batching
    server against the plain one-request-at-a-time loop on the same trace."""
    arrivals = gen.poisson_arrivals(rate, seconds, args.seed)
    reqs = [(float(t), k % len(pool)) for k, t in enumerate(arrivals)]
    log(f"serving: {len(reqs)} requests over {seconds} s at {rate}/s; continuous batching")
    cb = _serve_continuous(dgs, pool, reqs)
    log(f"serving: continuous batching: {cb}; plain one-at-a-time loop")
    plain = _serve_plain(dgs, np, pool, reqs)
    log(f"serving: plain: {plain}")
    return {"offered_per_s": round(len(reqs) / seconds, 2), "seconds": seconds, "requests": len(reqs),
            "continuous_batching": cb, "plain_per_request": plain}


def serving_summary(args, dgs, gen, np) -> dict:
    """The serving workload at its own arrival rate (200/s, more than one GPU
    completes: the completed rate is then the saturation throughput and the
    latency is queueing) and at a rate the plain loop also sustains."""
    pool = serving_pool(args, gen)
    for A in sorted(pool, key=lambda A: -A.shape[0])[:2]:  # warm the library's caches
        dgs.solve(A)
    out = {"n_range": [128, 16384], "pool": len(pool),
           "note": "requests cycle through a pool of distinct instances"}
    out["overload_200_per_s"] = run_serving(args, dgs, gen, np, pool, 200.0, args.serve_summary_seconds)
    out[f"sustained_{int(args.sustained_rate)}_per_s"] = run_serving(args, dgs, gen, np, pool, args.sustained_rate,
                                                                     args.serve_summary_seconds)
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lowrank16384", choices=WORKLOADS)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="single-instance workloads: skip the batched summary")
    ap.add_argument("--no-parallel", action="store_true",
                    help="single-instance workloads: skip the Parallel DGS summary")
    ap.add_argument("--no-lazy", action="store_true",
                    help="single-instance workloads: skip the lazy DGS summary")
    ap.add_argument("--no-rect", action="store_true",
                    help="single-instance workloads: skip the rectangular DGS summary")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="--workload serving: seconds of Poisson arrivals at 200/s")
    ap.add_argument("--serve-summary-seconds", type=float, default=8.0,
                    help="single-instance workloads: seconds of arrivals per load of the serving summary")
    ap.add_argument("--sustained-rate", type=float, default=25.0,
                    help="single-instance workloads: the serving summary's lower arrival rate (per s)")
    ap.add_argument("--no-serving", action="store_true",
                    help="single-instance workloads: skip the serving summary")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 launches): the reference "
                         "kernel that scales the HBM byte counters of a profile")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only (every instance runs on a "
              "single device); --gpus must be 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1106_5694_amd as dgs
    from workloads import gen

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes, "launches": 5}))
        return 0
    dgs.lib()

    if args.workload in SINGLE:
        line = run_single(args, dgs, torch, gen, np)
        if not args.no_parallel:
            log("parallel DGS summary")
            line["parallel"] = run_parallel(args, dgs, torch, gen, np)
            log(f"parallel DGS: {line['parallel']}")
        if not args.no_lazy and spec_n(args.workload) <= 16384:
            log("lazy DGS summary")
            line["lazy"] = run_lazy(args, dgs, torch, gen, np)
            log(f"lazy DGS: {line['lazy']}")
        if not args.no_rect:
            log("rectangular DGS summary")
            line["rect"] = run_rect(args, dgs, torch, gen, np)
            log(f"rectangular DGS: {line['rect']}")
        if not args.no_batched:
            log("batched workload summary")
            line["batched"] = run_batched(args, dgs, torch, gen, np, steps=3, warmup=1)
        if not args.no_serving:
            log("serving summary")
            line["serving"] = serving_summary(args, dgs, gen, np)
    elif args.workload == "batched512":
        b = run_batched(args, dgs, torch, gen, np, steps=args.steps, warmup=args.warmup)
        config = {"workload": "batched512", "instances": 512, "n": "log-uniform [64, 2048]",
                  "generator": "iid uniform int32 in [0,10000)", "seed": args.seed}
        line = base_line(args, b["instances_per_s"], "instances/s", b["ms_per_batch"], config)
        line["roofline"] = b.pop("roofline")
        line["batched"] = b
    else:
        pool = serving_pool(args, gen)
        for A in sorted(pool, key=lambda A: -A.shape[0])[:2]:
            dgs.solve(A)
        s = run_serving(args, dgs, gen, np, pool, 200.0, args.serve_seconds)
        config = {"workload": "serving", "arrivals": "Poisson 200/s", "seconds": args.serve_seconds,
                  "n": "log-uniform [128, 16384]", "generator": "low-rank + noise", "seed": args.seed,
                  "pool": len(pool)}
        cb = s["continuous_batching"]
        # a step is one request: its share of the continuous-batching wall time
        line = base_line(args, cb["completed_per_s"], "instances/s",
                         1000.0 * cb["wall_s"] / max(cb["requests"], 1), config)
        line["serving"] = s
    print(json.dumps(line), flush=True)
    dgs.release_cached()
    return 0


if __name__ == "__main__":
    # success returns normally instead of raising SystemExit: under
    # rocprofv3 the SystemExit path ends the process before the profiler
    # has written its database
    rc = main()
    if rc:
        sys.exit(rc)

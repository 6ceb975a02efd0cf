#!/usr/bin/env python3
"""EMPC benchmark on one MI355X.

Headline workload: 512 independent MPC problems solved together (degrees of
freedom drawn from {2, 7, 14, 21, 36}, linear mass-spring-damper or
nonlinear pendulum chains, horizon 20..100, 5..10 knots, population 1024,
32 parents, one generation per tick, FP32), one HIP-graph replay per
control tick.  A step is one tick for all 512 problems: the graph replay
(population, rollout + cost of every class, selection) and the copy of the
packed u* to the host.  Printed as one JSON line:
  value        candidate rollouts per second over the timed ticks
               (problems x population x generations x ticks / wall time);
  latency_ms   per-tick latency (submit to u* on the host) p50 / p99;
  roofline     one tick on the GPU (the graph replay, timed with HIP events on
               its stream over further ticks): algorithmic FLOP of every
               problem's rollouts (linear: the knot-precompute count; chain:
               25 d FLOP per candidate-step, sines not counted) over the mean
               tick time, against the matrix-core FP32 peak for the linear
               problems' share and the plain-VALU FP32 peak for the chains'
               (their time-weighted blend);
  cpu_baseline the FP64 oracle (one thread) on a bounded sample of the same
               workload, scaled per rollout;
  workloads    every other configuration measured the same way, each with
               its own roofline and oracle baselines on one core and on all
               cores: the 14-DoF closed loop (C2), the 2-DoF FP64 chain (C1),
               the 36-link pendulum chain (C3), the gradient-refined form
               against plain EMPC at equal final cost (C4, 14-DoF linear and
               36-DoF chain), the batch in its persistent form and as 512
               single solves, the N-link robot relinearized every tick, the
               parameterized convex MPC, the 14-DoF loop's variants, and the
               non-smooth forms (full weights with a settling-band charge on
               a 7-DoF chain; joint limits with impacts and dry friction on
               the 36-link chain).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--only NAME]
"""
from __future__ import annotations

import argparse
import concurrent.futures
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("candidate rollouts/sec and EMPC solve latency p50/p99 (ms) at fixed DoF/horizon")
PEAK_FP32_MFMA = 157.3e12  # MI355X dense FP32 matrix peak, FLOP/s
PEAK_FP32_VALU = 78.6e12   # MI355X FP32 vector peak without packed math, FLOP/s
PEAK_FP64 = 78.6e12        # MI355X FP64 (vector and matrix), FLOP/s
CSRC = os.path.join(ROOT, "paper_2001_04931_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rollout_linear_c2_traffic.md")
ROLLOUT_SRCS = [os.path.join(CSRC, f) for f in ("rollout_linear.hpp", "internal.hpp")]
BATCH_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "batch_tick_c5_traffic.md")
BATCH_SRCS = [os.path.join(CSRC, f) for f in ("batched.hip", "rollout_linear.hpp",
                                               "rollout_chain.hpp", "evolve_body.hpp",
                                               "rollout_valu.hpp", "internal.hpp")]


# ---------------------------------------------------------------------------
# algorithmic work

def linear_flop_per_candidate(n, m, T, p):
    """Algorithmic FLOP of one linear rollout with the knot precompute
    (V_j = B_d U_j once per knot): per step A_d x (2n^2), the knot blend and
    the state cost (6n), the input blend and cost (6m); per candidate the p
    knot responses B_d U_j (2pnm)."""
    return T * (2 * n * n + 6 * n + 6 * m) + 2 * p * n * m


def chain_flop_per_candidate(d, T):
    """Per candidate-step 25 d FLOP (interpolation 3d, prefix d, gravity
    coefficient d, suffix d, acceleration 6d, two updates 4d, cost 9d); the
    d sines are counted separately, not as FLOP."""
    return 25 * d * T


def flop_per_candidate(prob):
    import workloads as W

    if prob.model == W.LINEAR:
        return linear_flop_per_candidate(prob.n, prob.m, prob.T, prob.p)
    return chain_flop_per_candidate(prob.m, prob.T)


def roofline(flop, seconds, peak, bound="mfma", **extra):
    achieved = flop / seconds
    d = {"bound": bound, "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
         "frac": achieved / peak}
    d.update(extra)
    return d


def _counted_bytes(summary, sources, hash_key, bytes_key):
    """HBM bytes from a committed counter summary, or None when it is absent
    or was taken on other kernel sources than the current ones."""
    if not os.path.exists(summary):
        return None
    t = {}
    with open(summary) as f:
        for line in f:
            key, sep, val = line.strip().strip("`").partition(": ")
            if sep and key in (hash_key, bytes_key):
                t[key] = val.strip()
    h = hashlib.sha256()
    for src in sources:
        with open(src, "rb") as f:
            h.update(f.read())
    if t.get(hash_key) != h.hexdigest() or bytes_key not in t:
        return None
    return float(t[bytes_key])


def traffic_entry():
    """HBM bytes per C2 rollout launch (FETCH_SIZE + WRITE_SIZE, scaled)."""
    return _counted_bytes(TRAFFIC_FILE, ROLLOUT_SRCS, "rollout_src_sha256", "bytes_per_launch")


def batch_traffic_entry():
    """HBM bytes per tick of the 512-problem batch (every kernel of a tick)."""
    return _counted_bytes(BATCH_TRAFFIC_FILE, BATCH_SRCS, "batch_src_sha256", "bytes_per_tick")


def copy_calibration(mib, reps):
    """A plain device-to-device copy of `mib` MiB, `reps` times: the known
    byte count against which the HBM traffic counters are scaled."""
    import torch

    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "reps": reps}),
          flush=True)


# ---------------------------------------------------------------------------
# the oracle as CPU baseline (one thread, and one oracle per core)

def host_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def oracle_baseline(jobs, sample, unit="rollouts/s"):
    """Runs the first job alone on one thread, then jobs[1:] at once, one
    thread each (the oracle's C calls release the interpreter lock).  Each
    job returns the rollouts it did.  Returns the one-core and all-core
    baseline objects."""
    import oracle

    oracle.build(force=False)
    t0 = time.perf_counter()
    n1 = jobs[0]()
    t1 = time.perf_counter() - t0
    one = {"value": n1 / t1, "unit": unit, "cores": 1, "kind": "oracle",
           "sample": "%s; one thread, %.1f s" % (sample, t1), "cpu": cpu_model()}
    rest = jobs[1:][:host_cores()]
    cores = len(rest)
    t0 = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(max_workers=cores) as ex:
        counts = list(ex.map(lambda f: f(), rest))
    ta = time.perf_counter() - t0
    allc = {"value": sum(counts) / ta, "unit": unit, "cores": cores, "kind": "oracle",
            "sample": "%s; %d independent copies on %d threads, %.1f s" % (sample, cores, cores,
                                                                            ta),
            "cpu": cpu_model()}
    return one, allc


def closed_loop_job(prob, ga, ticks, seed, noise_std=0.0, refine=False):
    """One oracle closed loop (its own solver and start state)."""
    def job():
        import oracle
        import workloads as W

        s = oracle.Solver(prob, ga, refine=refine)
        x = W.start_inside_limits(prob, W.draw_x0(prob.n, seed))
        noise = W.process_noise(prob.n, ticks, seed, noise_std) if noise_std > 0 else None
        for t in range(ticks):
            u, _, _ = s.solve(x, t)
            x = oracle.step(prob, x, u, None if noise is None else noise[t])
        return ga.pop * ga.generations * ticks
    return job


# ---------------------------------------------------------------------------
# GPU measurement helpers

def closed_loop(E, W, prob, ga, dtype, ticks, warmup, noise_std=0.0, refine_steps=0,
                profile=0, tune=False):
    """Closed-loop ticks on one problem: solve, u* and best cost to the host,
    plant step.  Returns (rollouts/s, per-tick latencies in ms, best costs,
    (launches, kernel ms) of `profile` further ticks with HIP events stamped
    by every rollout launch, or None)."""
    import torch

    dp = E.DeviceProblem(prob, dtype)
    if tune:
        E.empc_autotune(dp, E.make_ga(ga), reps=10, allow_valu=True)
    solver = E.Solver(dp, ga)
    total = warmup + ticks + profile
    x = torch.tensor(W.start_inside_limits(prob, W.draw_x0(prob.n, 0)), dtype=dtype,
                     device="cuda")
    x_next = torch.empty_like(x)
    noise = None
    if noise_std > 0:
        noise = torch.tensor(W.process_noise(prob.n, total, 0, noise_std), dtype=dtype,
                             device="cuda")
    u_host = torch.empty(prob.m, dtype=dtype).pin_memory()
    j_host = torch.empty(1, dtype=dtype).pin_memory()
    done = torch.cuda.Event()
    lats, costs = [], []
    t_start = wall = None
    prof = None
    for t in range(total):
        if t == warmup:
            torch.cuda.synchronize()
            t_start = time.perf_counter()
        if t == warmup + ticks:
            torch.cuda.synchronize()
            wall = time.perf_counter() - t_start
            if profile:
                E.empc_profile_begin(profile * ga.generations)
        t0 = time.perf_counter()
        u, J = solver.solve(x, t, refine_steps=refine_steps)
        u_host.copy_(u, non_blocking=True)
        j_host.copy_(J, non_blocking=True)
        done.record()
        done.synchronize()
        if warmup <= t < warmup + ticks:
            lats.append((time.perf_counter() - t0) * 1e3)
            costs.append(float(j_host.item()))
        E.empc_plant_step(dp, x, u, None if noise is None else noise[t], x_next)
        x, x_next = x_next, x
    torch.cuda.synchronize()
    if wall is None:
        wall = time.perf_counter() - t_start
    if profile:
        prof = E.empc_profile_end()
    return ga.pop * ga.generations * ticks / wall, np.array(lats), costs, prof


def lat_summary(lats):
    return {"p50": float(np.percentile(lats, 50)), "p99": float(np.percentile(lats, 99)),
            "mean": float(np.mean(lats)), "max": float(np.max(lats))}


def kernel_roofline(prof, flop_launch, peak, name, bound="mfma", **extra):
    launches, kernel_ms = prof
    mean_s = kernel_ms * 1e-3 / max(launches, 1)
    return roofline(flop_launch, mean_s, peak, bound, kernel=name, launches=int(launches),
                    mean_us=mean_s * 1e6, flop_per_launch=flop_launch, **extra)


# ---------------------------------------------------------------------------
# the batch (headline) and its other forms

def c5_problems(W):
    probs, ga = W.config_c5(512, 0)
    return [p.cast(np.float32) for p in probs], ga


def c5_flop(probs, ga):
    """(linear FLOP, chain FLOP) of one generation of every problem."""
    import workloads as W

    lin = sum(ga.pop * flop_per_candidate(p) for p in probs if p.model == W.LINEAR)
    ch = sum(ga.pop * flop_per_candidate(p) for p in probs if p.model != W.LINEAR)
    return lin, ch


def blended_roofline(lin, ch, seconds, **extra):
    """Linear FLOP against the matrix-core peak, chain FLOP against the
    plain-VALU peak: `peak` is the blended rate (total FLOP over the time
    both shares would take at their peaks), `frac` that time over the
    measured one."""
    t_peak = lin / PEAK_FP32_MFMA + ch / PEAK_FP32_VALU
    peak = (lin + ch) / t_peak
    return roofline(lin + ch, seconds, peak, "mfma+valu", linear_flop=lin, chain_flop=ch, **extra)


def batched_run(E, W, probs, ga, mode, ticks, warm, event_ticks=50, allow_valu=False):
    """One BatchSolver over `probs`, one graph replay per tick.  Returns a
    summary (throughput, host latency, GPU tick time by HIP events)."""
    import torch

    dps = [E.DeviceProblem(p, torch.float32) for p in probs]
    t_tune = time.perf_counter()
    bs = E.BatchSolver(dps, ga, autotune=mode == 0, allow_valu=allow_valu)
    bs.set_mode(mode)
    t_tune = time.perf_counter() - t_tune
    for i, p in enumerate(probs):
        bs.set_x0(i, W.draw_x0(p.n, i))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bs.solve()
    u_host = torch.empty(bs.u_star.numel(), dtype=torch.float32).pin_memory()
    done = torch.cuda.Event()
    lats = []
    for t in range(warm + ticks):
        if t == warm:
            torch.cuda.synchronize()
            t_start = time.perf_counter()
        t0 = time.perf_counter()
        g.replay()
        u_host.copy_(bs.u_star, non_blocking=True)
        done.record()
        done.synchronize()
        if t >= warm:
            lats.append((time.perf_counter() - t0) * 1e3)
    wall = time.perf_counter() - t_start
    # GPU time of a tick: events on the replay's stream around each replay
    st = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(event_ticks)]
    for a, b in ev:
        a.record(st)
        g.replay()
        b.record(st)
    torch.cuda.synchronize()
    gpu_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    classes = bs.classes() if mode == 0 else None
    bs.close()
    lats = np.array(lats)
    n = len(probs)
    return {"rollouts_per_s": n * ga.pop * ga.generations * ticks / wall,
            "latency_ms": lat_summary(lats), "ticks": ticks, "problems": n,
            "within_2ms": float(np.mean(lats <= 2.0)), "gpu_tick_ms": gpu_ms, "wall_s": wall,
            "plan_and_autotune_s": round(t_tune, 3),
            "mode": "persistent work queue" if mode else (
                "per-class launches, autotuned" + (", VALU form allowed" if allow_valu else "")),
            "classes": None if classes is None else [
                "%s%s x%d: shape %d of us %s, stream %d" % (
                    "lin" if c["model"] == "linear" else "chain", list(c["shape"]),
                    c["problems"], c["variant"], c["tuned_us"], c["stream"]) for c in classes]}


def c5_oracle_jobs(probs, ga, cores):
    """Oracle jobs on a 128-problem sample of the batch (every fourth
    problem), three ticks each (a cold start and two warm ticks, one
    generation of 1024 per tick): the first job does the whole sample, the
    others a share each."""
    import workloads as W

    sample = list(range(0, len(probs), 4))
    ticks = 3

    def job_for(idx):
        def job():
            import oracle

            for i in idx:
                s = oracle.Solver(probs[i], W.dataclasses.replace(ga, seed=ga.seed ^ (i << 32)))
                x = W.draw_x0(probs[i].n, i)
                for t in range(ticks):
                    s.solve(x, t)
            return len(idx) * ga.pop * ga.generations * ticks
        return job
    per = max(1, -(-len(sample) // cores))
    return [job_for(sample)] + [job_for(sample[i:i + per]) for i in range(0, len(sample), per)]


def c5_workload(E, W, ticks, warm, with_cpu=True):
    """The headline: 512 uneven problems, one graph replay per tick."""
    probs, ga = c5_problems(W)
    r = batched_run(E, W, probs, ga, 0, ticks, warm, allow_valu=True)
    lin, ch = c5_flop(probs, ga)
    r["roofline"] = blended_roofline(lin, ch, r["gpu_tick_ms"] * 1e-3,
                                     unit_of_work="one tick (graph replay), all 512 problems",
                                     traffic=batch_traffic_entry())
    r["flop_per_tick"] = lin + ch
    if with_cpu:
        r["cpu_baseline"], r["cpu_baseline_all_cores"] = oracle_baseline(
            c5_oracle_jobs(probs, ga, host_cores()),
            "3 ticks (cold start + 2 warm, 1 generation of 1024 each) of 128 of the 512 "
            "problems (every fourth), FP64")
    return r, probs, ga


def c5_extra(E, W, probs, ga, ticks, warm):
    """The batch in its persistent form, and the same 512 problems as
    single-problem solves one after another."""
    import torch

    out = {}
    r = batched_run(E, W, probs, ga, 1, ticks, warm)
    lin, ch = c5_flop(probs, ga)
    r["roofline"] = blended_roofline(lin, ch, r["gpu_tick_ms"] * 1e-3,
                                     unit_of_work="one tick (graph replay), all 512 problems")
    out["c5_persistent_form"] = r
    dps = [E.DeviceProblem(p, torch.float32) for p in probs]
    solvers = [E.Solver(dp, W.dataclasses.replace(ga, seed=ga.seed ^ (i << 32)))
               for i, dp in enumerate(dps)]
    xs = [torch.tensor(W.draw_x0(p.n, i), dtype=torch.float32, device="cuda")
          for i, p in enumerate(probs)]
    reps = 5
    for t in range(reps + 1):
        if t == 1:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        for s, x in zip(solvers, xs):
            s.solve(x, t)
    torch.cuda.synchronize()
    per_tick = (time.perf_counter() - t0) / reps
    out["c5_as_single_solves"] = {"tick_ms": per_tick * 1e3,
                                  "rollouts_per_s": len(probs) * ga.pop / per_tick,
                                  "ticks": reps, "launches_per_tick": 3 * len(probs)}
    return out


# ---------------------------------------------------------------------------
# single-problem workloads

def c2_workload(E, W, ticks, warm, with_cpu=True):
    """C2: 14-DoF linear chain, FP32, closed loop with process noise."""
    import torch

    prob, ga = W.config_c2(0)
    rate, lats, costs, prof = closed_loop(E, W, prob, ga, torch.float32, ticks, warm,
                                          noise_std=1e-3, profile=min(ticks, 20))
    flop = ga.pop * linear_flop_per_candidate(prob.n, prob.m, prob.T, prob.p)
    r = {"rollouts_per_s": rate, "latency_ms": lat_summary(lats), "ticks": ticks, "dtype": "f32",
         "final_best_cost": costs[-1],
         "roofline": kernel_roofline(prof, flop, PEAK_FP32_MFMA, "roll_linear_split<float,2,4>",
                                     traffic=traffic_entry())}
    if with_cpu:
        jobs = [closed_loop_job(prob, ga, 2, s, 1e-3) for s in range(1 + host_cores())]
        r["cpu_baseline"], r["cpu_baseline_all_cores"] = oracle_baseline(
            jobs, "2 closed-loop ticks (20 generations x 4096 candidates each), FP64")
    return r


def c1_workload(E, W, ticks=1000, with_cpu=True):
    """C1: 2-DoF linear chain, FP64, 1000 closed-loop solves, launch shapes
    picked by the single-problem autotuner."""
    import torch

    prob, ga = W.config_c1(0)
    dp = E.DeviceProblem(prob, torch.float64)
    tuned = E.empc_autotune(dp, E.make_ga(ga), reps=10, allow_valu=True)
    rate, lats, _, prof = closed_loop(E, W, prob, ga, torch.float64, ticks, 20, profile=20)
    flop = ga.pop * linear_flop_per_candidate(prob.n, prob.m, prob.T, prob.p)
    r = {"rollouts_per_s": rate, "latency_ms": lat_summary(lats), "ticks": ticks, "dtype": "f64",
         "autotuned": tuned,
         "roofline": kernel_roofline(prof, flop, PEAK_FP64, "tuned linear rollout (FP64)",
                                     bound="latency")}
    E.empc_autotune_reset()
    if with_cpu:
        jobs = [closed_loop_job(prob, ga, 1000, s) for s in range(1 + host_cores())]
        r["cpu_baseline"], r["cpu_baseline_all_cores"] = oracle_baseline(
            jobs, "1000 closed-loop ticks (10 generations x 256 candidates each), FP64")
    return r


def c3_workload(E, W, ticks=100, with_cpu=True):
    """C3: 36-link pendulum chain, FP32, pop 16384, 30 generations."""
    import torch

    prob, ga = W.config_c3(0)
    rate, lats, _, prof = closed_loop(E, W, prob, ga, torch.float32, ticks, 2, profile=5)
    flop = ga.pop * chain_flop_per_candidate(prob.m, prob.T)
    r = {"rollouts_per_s": rate, "latency_ms": lat_summary(lats), "ticks": ticks, "dtype": "f32",
         "roofline": kernel_roofline(prof, flop, PEAK_FP32_VALU, "roll_chain_rows<float,3>",
                                     bound="valu", sines_per_launch=ga.pop * prob.m * prob.T)}
    if with_cpu:
        one_gen = W.dataclasses.replace(ga, generations=1)
        jobs = [closed_loop_job(prob, one_gen, 1, s) for s in range(1 + host_cores())]
        r["cpu_baseline"], r["cpu_baseline_all_cores"] = oracle_baseline(
            jobs, "1 tick of 1 generation of 16384 candidates of the same chain, FP64")
    return r


def equal_cost(E, W, prob, ga, dtype, refine_steps, x0, max_gen=2560):
    """The refined solve's best cost after ga.generations at x0 (cold start),
    and plain EMPC's with the generations doubled until plain comes within
    1e-4 (relative) of the refined cost; solve times of both."""
    import torch

    dp = E.DeviceProblem(prob, dtype)
    x = torch.tensor(x0, dtype=dtype, device="cuda")

    def solve_once(g, steps):
        s = E.Solver(dp, W.dataclasses.replace(ga, generations=g))
        s.solve(x, 0, refine_steps=steps)  # first call: kernels loaded
        s.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, J = s.solve(x, 0, refine_steps=steps)
        torch.cuda.synchronize()
        return float(J.item()), (time.perf_counter() - t0) * 1e3

    J_ref, t_ref = solve_once(ga.generations, refine_steps)
    g = ga.generations
    J_plain, t_plain = solve_once(g, 0)
    trail = [(g, J_plain, t_plain)]
    while J_plain > J_ref * (1 + 1e-4) and g < max_gen:
        g *= 2
        J_plain, t_plain = solve_once(g, 0)
        trail.append((g, J_plain, t_plain))
    return {"refined": {"generations": ga.generations, "adam_steps": refine_steps,
                        "best_cost": J_ref, "solve_ms": t_ref},
            "plain_equal_cost": {"generations": g, "best_cost": J_plain, "solve_ms": t_plain,
                                 "reached": bool(J_plain <= J_ref * (1 + 1e-4))},
            "plain_trail": [{"generations": a, "best_cost": b, "solve_ms": c}
                            for a, b, c in trail]}


def c4_workload(E, W, ticks=100, with_cpu=True):
    """C4: gradient refinement (5 Adam steps on the 64 parents after every
    selection) on the 14-DoF linear loop and the 36-DoF pendulum chain,
    against plain EMPC at equal final cost."""
    import torch

    out = {}
    prob, ga = W.config_c2(0)
    rate_r, lats_r, _, _ = closed_loop(E, W, prob, ga, torch.float32, ticks, 2,
                                       noise_std=1e-3, refine_steps=5)
    rate_p, lats_p, _, _ = closed_loop(E, W, prob, ga, torch.float32, ticks, 2, noise_std=1e-3)
    r = {"rollouts_per_s": rate_r, "latency_ms": lat_summary(lats_r), "ticks": ticks,
         "dtype": "f32", "plain_rollouts_per_s": rate_p, "plain_latency_ms": lat_summary(lats_p),
         "equal_cost": equal_cost(E, W, prob.cast(np.float32), ga, torch.float32, 5,
                                  W.draw_x0(prob.n, 0))}
    if with_cpu:
        five_gen = W.dataclasses.replace(ga, generations=5)
        jobs = [closed_loop_job(prob, five_gen, 1, s, refine=True)
                for s in range(1 + host_cores())]
        r["cpu_baseline"], r["cpu_baseline_all_cores"] = oracle_baseline(
            jobs, "1 tick of 5 refined generations (4096 candidates, 5 Adam steps on 64 parents "
                  "each), FP64", unit="rollouts/s (refinement included)")
    out["c4_fp32_14dof_refined"] = r
    prob, ga = W.config_c3(0)
    out["c4_fp32_36dof_chain_refined"] = {
        "dtype": "f32", "equal_cost": equal_cost(E, W, prob.cast(np.float32), ga, torch.float32,
                                                 5, W.draw_x0(prob.n, 0), max_gen=480)}
    return out


def full_weight_flop_per_candidate(n, m, T):
    """Per step: dynamics 2n^2 + 2nm, the state quadratic form 2n^2 + 2n
    and its error n, the input quadratic form 2m^2 + 2m, the knot blend and
    input error 4m, the band indicator n; the terminal form once."""
    return T * (4 * n * n + 2 * n * m + 2 * m * m + 4 * n + 6 * m) + 2 * n * n + 3 * n


def nonsmooth_workload(E, W, ticks=100, with_cpu=True):
    """Sec. V-A's flexibility on the GPU: full Q, R, Qf with a settling-band
    charge on the 7-DoF linear chain (vector-ALU rollout), and joint limits
    with impacts plus a settling-band charge on the 36-joint pendulum chain
    with dry friction (C3's shape), each in a closed loop whose plant has
    the same effects."""
    import torch

    out = {}
    prob, ga = W.config_nonsmooth_linear(0)
    dp = E.DeviceProblem(prob, torch.float32)
    tuned = E.empc_autotune(dp, E.make_ga(ga), reps=10, allow_valu=True)
    rate, lats, costs, prof = closed_loop(E, W, prob, ga, torch.float32, ticks, 5,
                                          noise_std=1e-3, profile=10)
    E.empc_autotune_reset()
    flop = ga.pop * full_weight_flop_per_candidate(prob.n, prob.m, prob.T)
    r = {"rollouts_per_s": rate, "latency_ms": lat_summary(lats), "ticks": ticks,
         "dtype": "f32", "autotuned": tuned, "final_best_cost": costs[-1],
         "roofline": kernel_roofline(prof, flop, PEAK_FP32_VALU,
                                     "roll_linear_valu<full>"
                                     if tuned["rollout_form"] in (E.RF_VALU256, E.RF_VALU64)
                                     else "roll_linear_full_rows",
                                     bound="valu")}
    if with_cpu:
        jobs = [closed_loop_job(prob, W.dataclasses.replace(ga, generations=5), 1, s, 1e-3)
                for s in range(1 + host_cores())]
        r["cpu_baseline"], r["cpu_baseline_all_cores"] = oracle_baseline(
            jobs, "1 closed-loop tick of 5 generations x 4096 candidates, FP64")
    out["nonsmooth_7dof_full_weights_band"] = r
    prob, ga = W.config_nonsmooth_chain(0)
    rate, lats, costs, prof = closed_loop(E, W, prob, ga, torch.float32, ticks, 2, profile=5)
    flop = ga.pop * chain_flop_per_candidate(prob.m, prob.T)
    r = {"rollouts_per_s": rate, "latency_ms": lat_summary(lats), "ticks": ticks,
         "dtype": "f32", "final_best_cost": costs[-1],
         "roofline": kernel_roofline(prof, flop, PEAK_FP32_VALU, "roll_chain_rows<limits, friction, box>",
                                     bound="valu", sines_per_launch=ga.pop * prob.m * prob.T)}
    if with_cpu:
        one_gen = W.dataclasses.replace(ga, generations=1)
        jobs = [closed_loop_job(prob, one_gen, 1, s) for s in range(1 + host_cores())]
        r["cpu_baseline"], r["cpu_baseline_all_cores"] = oracle_baseline(
            jobs, "1 tick of 1 generation of 16384 candidates of the same chain, FP64")
    out["nonsmooth_36link_limits_friction_band"] = r
    return out


def variants_workload(E, W):
    """The 14-DoF closed loop with fewer generations per tick (the paper's one
    and three iterations per control step) and with the warm-start variants
    (carried parents moved one step later per tick, noise growing with the
    distance to the goal): throughput, latency and the mean best cost of
    the ticks (lower: the loop holds the chain nearer the goal)."""
    import torch

    prob, ga = W.config_c2(0)
    runs = {"G1": dict(generations=1), "G3": dict(generations=3), "G20": {},
            "G20_shift_noise_schedule": dict(shift=True, sigma_min=0.01, sigma_dist=1.0)}
    out = {}
    for name, kw in runs.items():
        g = W.dataclasses.replace(ga, **kw)
        rate, lats, costs, _ = closed_loop(E, W, prob, g, torch.float32, 30, 2, noise_std=1e-3)
        out[name] = {"rollouts_per_s": rate, "latency_ms": lat_summary(lats), "ticks": 30,
                     "generations": g.generations, "mean_best_cost": float(np.mean(costs)),
                     "last_best_cost": float(costs[-1])}
    return {"c2_variants": out}


def nlink_closed_loop(E, W, N, generations, ticks, dtype, seed=0):
    """The paper's N-link robot experiment on the GPU: every tick relinearize
    the robot at its state (and last torque), one EMPC solve on that model,
    u* to the host, RK4 step of the robot (4 substeps).  Returns (solve
    latencies ms, relinearization+solve latencies ms, rollouts/s, final
    distance to the goal)."""
    import torch

    robot, prob, x0, ga = W.config_nlink(N, seed, generations)
    R = E.NLinkRobot(robot.mass, robot.length, robot.damping, dtype)
    dp = E.DeviceProblem(prob, dtype, keep=("wd",))
    solver = E.Solver(dp, ga)
    x = torch.tensor(x0, dtype=dtype, device="cuda")
    u = torch.zeros(N, dtype=dtype, device="cuda")
    u_host = torch.empty(N, dtype=dtype).pin_memory()
    done = torch.cuda.Event()
    lin_ev = torch.cuda.Event()
    lats, tot = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for t in range(ticks):
        # the simulated robot's step (the plant, not the controller) has
        # finished before the controller's time starts
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E.empc_nlink_linearize(R, 0.01, x, u, dp.tensors["Ad"], dp.tensors["Bd"],
                               dp.tensors["wd"])
        lin_ev.record()
        lin_ev.synchronize()
        t1 = time.perf_counter()
        us, _ = solver.solve(x, t)
        u_host.copy_(us, non_blocking=True)
        done.record()
        done.synchronize()
        t2 = time.perf_counter()
        lats.append((t2 - t1) * 1e3)
        tot.append((t2 - t0) * 1e3)
        u.copy_(us)
        E.empc_nlink_step(R, 0.01, 4, x, u, x)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    dist = float(torch.linalg.vector_norm(x - torch.tensor(prob.x_goal, dtype=dtype,
                                                           device="cuda")).item())
    return np.array(lats), np.array(tot), ga.pop * generations * ticks / wall, dist


def nlink_workload(E, W, links=range(1, 14), ticks=1000, with_cpu=True):
    """The paper's EMPC experiment: N-link planar robots of 1..13 links, 1 kg
    and 0.25 m per link, |tau| <= 2 N m, horizon 100, 3 knots, control at
    100 Hz for 10 s (1000 ticks), 1 and 3 generations per tick; FP32 EMPC on
    the model relinearized (in FP64) every tick."""
    import torch

    out = {}
    for G in (1, 3):
        rows = {}
        for N in links:
            lats, tot, rate, dist = nlink_closed_loop(E, W, N, G, ticks, torch.float32)
            rows[str(N)] = {"solve_ms": {"p50": float(np.percentile(lats, 50)),
                                         "p99": float(np.percentile(lats, 99))},
                            "relinearize_and_solve_ms": {"p50": float(np.percentile(tot, 50)),
                                                         "p99": float(np.percentile(tot, 99))},
                            "rollouts_per_s": rate, "final_goal_distance": dist}
        out["G%d" % G] = rows
    r = {"ticks": ticks, "horizon": 100, "knots": 3, "pop": 1024, "dtype": "f32", "links": out}
    if with_cpu:
        def job_for(seed):
            def job():
                import dataclasses

                import oracle

                robot, prob, x0, ga = W.config_nlink(13, seed, 1)
                s = oracle.Solver(prob, ga)
                x, u = x0.copy(), np.zeros(13)
                for t in range(50):
                    Ad, Bd, wd = oracle.nlink_linearize(robot.mass, robot.length, robot.damping,
                                                        x, u, 0.01)
                    s.P = oracle.OracleProblem(dataclasses.replace(prob, Ad=Ad, Bd=Bd, wd=wd))
                    u, _, _ = s.solve(x, t)
                    x = oracle.nlink_rk4(robot.mass, robot.length, robot.damping, x, u, 0.01, 4)
                return ga.pop * 50
            return job
        r["cpu_baseline"], r["cpu_baseline_all_cores"] = oracle_baseline(
            [job_for(s) for s in range(1 + host_cores())],
            "50 relinearize-solve-step ticks of the 13-link robot (1 generation of 1024), FP64")
    return {"nlink_robot_relinearized": r}


def convex_workload(E, W, reps=50, with_cpu=True):
    """The paper's other method on the GPU: parameterized small-matrix convex
    MPC (form P, q, c, then the box QP) for the 2-DoF and 14-DoF linear
    chains and the 13-link robot linearized at its start (horizon 50 and
    100, 5 knots as in the paper's convex experiments), FP64; the solve
    time, the solver's iterations, and the gap of EMPC's best cost after the
    configuration's generations to the convex optimum."""
    import torch

    out = {}
    cases = {"c1_2dof": W.config_c1(0), "c2_14dof": W.config_c2(0)}
    for T in (50, 100):
        robot, prob, x0, ga = W.config_nlink(13, 0)
        prob = W.nlink_problem(13, T, 5, prob.x_goal)
        cases["nlink13_T%d" % T] = (prob, ga, robot, x0)
    for name, c in cases.items():
        prob, ga = c[0], c[1]
        dp = E.DeviceProblem(prob, torch.float64, keep=("wd",))
        if len(c) == 4:
            robot, x0 = c[2], c[3]
            R = E.NLinkRobot(robot.mass, robot.length, robot.damping, torch.float64)
            x = torch.tensor(x0, dtype=torch.float64, device="cuda")
            E.empc_nlink_linearize(R, 0.01, x, torch.zeros(prob.m, dtype=torch.float64,
                                                           device="cuda"),
                                   dp.tensors["Ad"], dp.tensors["Bd"], dp.tensors["wd"])
        else:
            x = torch.tensor(W.draw_x0(prob.n, 0), dtype=torch.float64, device="cuda")
        cs = E.ConvexSolver(dp)
        cs.solve(x)
        torch.cuda.synchronize()
        lats = []
        for _ in range(reps):
            t0 = time.perf_counter()
            cs.solve(x)
            torch.cuda.synchronize()
            lats.append((time.perf_counter() - t0) * 1e3)
        info = cs.info.cpu().numpy()
        Jstar = float(cs.cost.item())
        entry = {"pm": prob.p * prob.m, "T": prob.T, "n": prob.n,
                 "solve_ms": lat_summary(np.array(lats)),
                 "iterations": int(info[0]), "converged": bool(info[1]), "optimum": Jstar}
        if len(c) == 2:
            s = E.Solver(dp, ga)
            _, J = s.solve(x, 0)
            entry["empc_best_cost"] = float(J.item())
            entry["empc_gap"] = float(J.item()) / Jstar - 1.0
            if with_cpu and name == "c2_14dof":
                from oracle import convex

                x0 = W.draw_x0(prob.n, 0)
                t0 = time.perf_counter()
                P, q, cc = convex.qp_form(prob, x0)
                lo, hi = convex.knot_bounds(prob)
                convex.qp_solve(P, q, lo, hi)
                entry["cpu_baseline"] = {"value": (time.perf_counter() - t0) * 1e3, "unit": "ms",
                                         "cores": 1, "kind": "oracle",
                                         "sample": "one convex solve (form + bvls), FP64",
                                         "cpu": cpu_model()}
        out[name] = entry
    return {"convex_small_matrix_fp64": out}


WORKLOADS = ("c2", "c1", "c3", "c4", "c5x", "c2v", "nlink", "convex", "nonsmooth")


def other_workloads(E, W, names, with_cpu, c5_state=None):
    runs = {
        "c2": lambda: {"c2_fp32_14dof_closed_loop": c2_workload(E, W, 100, 5, with_cpu)},
        "c1": lambda: {"c1_fp64_2dof": c1_workload(E, W, 1000, with_cpu)},
        "c3": lambda: {"c3_fp32_36link_chain": c3_workload(E, W, 100, with_cpu)},
        "c4": lambda: c4_workload(E, W, 100, with_cpu),
        "c5x": lambda: c5_extra(E, W, *(c5_state or c5_problems(W)), 200, 10),
        "c2v": lambda: variants_workload(E, W),
        "nlink": lambda: nlink_workload(E, W, with_cpu=with_cpu),
        "convex": lambda: convex_workload(E, W, with_cpu=with_cpu),
        "nonsmooth": lambda: nonsmooth_workload(E, W, 100, with_cpu),
    }
    out = {}
    for name in WORKLOADS:
        if name in names:
            t0 = time.perf_counter()
            out.update(runs[name]())
            print("bench: workload %s done in %.1f s" % (name, time.perf_counter() - t0),
                  file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000, help="timed control ticks (headline)")
    ap.add_argument("--warmup", type=int, default=10, help="untimed control ticks")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the other configurations")
    ap.add_argument("--only", choices=WORKLOADS + ("c5",), default=None,
                    help="run only this configuration (for profiling) and print its summary "
                         "instead of the benchmark line")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain MIB-MiB device copy (traffic-counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the EMPC hot path here is a single-GPU "
              "build (multi-GPU sharding is described, not implemented); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        copy_calibration(args.copy_calibration, 5)
        return

    import paper_2001_04931_amd as E
    import workloads as W

    torch.cuda.set_device(0)
    with_cpu = not args.no_cpu_baseline
    if args.only == "c5":
        r, _, _ = c5_workload(E, W, args.steps, args.warmup, with_cpu)
        print(json.dumps(r), flush=True)
        return
    if args.only:
        print(json.dumps(other_workloads(E, W, (args.only,), with_cpu)), flush=True)
        return
    t0 = time.perf_counter()
    r, probs, ga = c5_workload(E, W, args.steps, args.warmup, with_cpu)
    print("bench: headline done in %.1f s" % (time.perf_counter() - t0), file=sys.stderr,
          flush=True)
    out = {
        "metric": METRIC,
        "value": r["rollouts_per_s"],
        "unit": "rollouts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["wall_s"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "EMPC batch: 512 independent problems, DoF ~ U{2,7,14,21,36}, "
                               "linear mass-spring-damper or nonlinear pendulum chain ~ "
                               "Bernoulli(1/2), horizon U{20..100}, knots U{5..10}, pop 1024, "
                               "32 parents, 1 generation/tick, sigma 0.1, seed 0, one HIP-graph "
                               "replay per tick",
                   "problems": len(probs), "pop": ga.pop, "n_elite": ga.n_elite,
                   "generations": ga.generations, "ticks": args.steps},
        "latency_ms": r["latency_ms"],
        "within_2ms": r["within_2ms"],
        "gpu_tick_ms": r["gpu_tick_ms"],
        "roofline": r["roofline"],
        "classes": r["classes"],
    }
    if with_cpu:
        out["cpu_baseline"] = r["cpu_baseline"]
        out["cpu_baseline_all_cores"] = r["cpu_baseline_all_cores"]
    if not args.no_workloads:
        out["workloads"] = other_workloads(E, W, WORKLOADS, with_cpu, (probs, ga))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

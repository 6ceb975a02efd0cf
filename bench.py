#!/usr/bin/env python3
"""EMPC benchmark on one MI355X: closed-loop control of the 14-DoF linear
mass-spring-damper chain (n = 28 states, m = 14 inputs), FP32, horizon 50,
10 knots per input, population 4096, 64 elites, 20 generations per control
tick, N(0, 1e-3^2) process noise on the simulated plant.

A step is one control tick: the EMPC solve (20 x {population, rollout +
cost, selection}), the copy of u* and the best cost to the host, then the
plant step.  Printed as one JSON line:
  value       candidate rollouts per second over the timed ticks
              (population x generations x ticks / wall time);
  latency_ms  per-tick solve latency (submit to u* on the host) p50 / p99;
  roofline    rollout kernel: algorithmic FLOP of the rollout and cost per
              launch over the mean launch time from HIP events recorded
              around every rollout launch of up to 20 further ticks of the
              same closed loop (the event markers slow the tick down, so the
              throughput ticks run without them), against the FP32
              matrix-core peak;
  cpu_baseline the FP64 oracle on a bounded sample of the same workload;
  workloads   the other configurations measured the same way: 2-DoF chain
              in FP64, 36-link pendulum chain, the gradient-refined form of
              the 14-DoF run beside plain EMPC, 512 uneven problems solved
              together, one HIP-graph replay per tick, and the 14-DoF loop
              with 1 / 3 / 20 generations per tick and the warm-start
              variants.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("candidate rollouts/sec and EMPC solve latency p50/p99 (ms) at fixed DoF/horizon")
PEAK_FP32_MFMA = 157.3e12  # MI355X dense FP32 matrix peak, FLOP/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rollout_linear_c2_traffic.md")
ROLLOUT_SRC = os.path.join(ROOT, "paper_2001_04931_amd", "csrc", "rollout_linear.hpp")


def linear_flop_per_candidate(n, m, T, p):
    """Algorithmic FLOP of one linear rollout with the knot precompute
    (V_j = B_d U_j once per knot): per step A_d x (2n^2), the knot blend and
    the state cost (6n), the input blend and cost (6m); per candidate the p
    knot responses B_d U_j (2pnm)."""
    return T * (2 * n * n + 6 * n + 6 * m) + 2 * p * n * m


def traffic_entry():
    """HBM bytes per rollout launch from the committed counter summary, or
    None when absent or taken on a different rollout kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    t = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            key, sep, val = line.strip().strip("`").partition(": ")
            if sep and key in ("rollout_src_sha256", "bytes_per_launch"):
                t[key] = val.strip()
    with open(ROLLOUT_SRC, "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()
    if t.get("rollout_src_sha256") != h or "bytes_per_launch" not in t:
        return None
    return float(t["bytes_per_launch"])


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


def cpu_baseline(prob, ga, ticks):
    """The FP64 oracle as it stands, single-threaded, on `ticks` closed-loop
    ticks of the same workload."""
    import oracle
    import workloads as W

    oracle.build(force=False)
    s = oracle.Solver(prob, ga)
    x = W.draw_x0(prob.n, 0)
    noise = W.process_noise(prob.n, ticks, 0)
    t0 = time.perf_counter()
    for t in range(ticks):
        u, _, _ = s.solve(x, t)
        x = oracle.step(prob, x, u, noise[t])
    dt = time.perf_counter() - t0
    return {"value": ga.pop * ga.generations * ticks / dt, "unit": "rollouts/s", "cores": 1,
            "kind": "oracle",
            "sample": "%d closed-loop ticks of the same workload (%d generations x %d candidates "
                      "each), FP64, one thread, %.1f s" % (ticks, ga.generations, ga.pop, dt)}


def closed_loop(E, W, prob, ga, dtype, ticks, warmup, noise_std=0.0, refine_steps=0):
    """Closed-loop ticks on one problem: solve, u* and best cost to the host,
    plant step.  Returns (rollouts/s, per-tick latencies in ms, best costs)."""
    import torch

    dp = E.DeviceProblem(prob, dtype)
    solver = E.Solver(dp, ga)
    total = warmup + ticks
    x = torch.tensor(W.draw_x0(prob.n, 0), dtype=dtype, device="cuda")
    x_next = torch.empty_like(x)
    noise = None
    if noise_std > 0:
        noise = torch.tensor(W.process_noise(prob.n, total, 0, noise_std), dtype=dtype,
                             device="cuda")
    u_host = torch.empty(prob.m, dtype=dtype).pin_memory()
    j_host = torch.empty(1, dtype=dtype).pin_memory()
    done = torch.cuda.Event()
    lats, costs = [], []
    t_start = None
    for t in range(total):
        if t == warmup:
            torch.cuda.synchronize()
            t_start = time.perf_counter()
        t0 = time.perf_counter()
        u, J = solver.solve(x, t, refine_steps=refine_steps)
        u_host.copy_(u, non_blocking=True)
        j_host.copy_(J, non_blocking=True)
        done.record()
        done.synchronize()
        if t >= warmup:
            lats.append((time.perf_counter() - t0) * 1e3)
            costs.append(float(j_host.item()))
        E.empc_plant_step(dp, x, u, None if noise is None else noise[t], x_next)
        x, x_next = x_next, x
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    return ga.pop * ga.generations * ticks / wall, np.array(lats), costs


def summary(rate, lats, **extra):
    d = {"rollouts_per_s": rate, "latency_ms": {"p50": float(np.percentile(lats, 50)),
                                                "p99": float(np.percentile(lats, 99))}}
    d.update(extra)
    return d


WORKLOADS = ("c1", "c3", "c4", "c5", "c2v", "nlink", "convex")


def other_workloads(E, W, names=WORKLOADS):
    """The remaining benchmark configurations, measured the same way."""
    import torch

    out = {}
    if "c1" in names:
        prob, ga = W.config_c1(0)
        rate, lats, _ = closed_loop(E, W, prob, ga, torch.float64, 100, 5)
        out["c1_fp64_2dof"] = summary(rate, lats, ticks=100, dtype="f64")

    if "c3" in names:
        prob, ga = W.config_c3(0)
        rate, lats, _ = closed_loop(E, W, prob, ga, torch.float32, 10, 2)
        out["c3_fp32_36link_chain"] = summary(rate, lats, ticks=10, dtype="f32")
    if "c4" in names:
        out.update(refined_workload(E, W))
    if "c5" in names:
        out.update(batched_workload(E, W))
        out.update(batched_workload(E, W, mode=1))
    if "c2v" in names:
        out.update(variants_workload(E, W))
    if "nlink" in names:
        out.update(nlink_workload(E, W))
    if "convex" in names:
        out.update(convex_workload(E, W))
    return out


def convex_workload(E, W, reps=50):
    """The paper's other method on the GPU: parameterized small-matrix convex
    MPC (form P, q, c, then the box QP) for the 2-DoF and 14-DoF linear
    chains and the 13-link robot linearized at rest-to-goal start (horizon
    50 and 100, 5 knots as in the paper's convex experiments), FP64; the
    solve time, active-set iterations, and the gap of EMPC's best cost after
    the configuration's generations to the convex optimum."""
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
                 "solve_ms": {"p50": float(np.percentile(lats, 50)),
                              "p99": float(np.percentile(lats, 99))},
                 "active_set_iterations": int(info[0]), "converged": bool(info[1]),
                 "optimum": Jstar}
        if len(c) == 2:
            s = E.Solver(dp, ga)
            _, J = s.solve(x, 0)
            entry["empc_best_cost"] = float(J.item())
            entry["empc_gap"] = float(J.item()) / Jstar - 1.0
        out[name] = entry
    return {"convex_small_matrix_fp64": out}


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


def nlink_workload(E, W, links=range(1, 14), ticks=1000):
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
    return {"nlink_robot_relinearized": {"ticks": ticks, "horizon": 100, "knots": 3,
                                         "pop": 1024, "dtype": "f32", "links": out}}


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
        rate, lats, costs = closed_loop(E, W, prob, g, torch.float32, 30, 2, noise_std=1e-3)
        out[name] = summary(rate, lats, ticks=30, dtype="f32", generations=g.generations,
                            mean_best_cost=float(np.mean(costs)),
                            last_best_cost=float(costs[-1]))
    return {"c2_variants": out}


def refined_workload(E, W):
    """C4: the gradient-refined form beside plain EMPC on the same ticks."""
    import torch

    out = {}
    prob, ga = W.config_c2(0)
    rate_p, lats_p, costs_p = closed_loop(E, W, prob, ga, torch.float32, 10, 1, noise_std=1e-3)
    rate_r, lats_r, costs_r = closed_loop(E, W, prob, ga, torch.float32, 10, 1, noise_std=1e-3,
                                          refine_steps=5)
    out["c4_fp32_14dof_refined"] = summary(
        rate_r, lats_r, ticks=10, dtype="f32", adam_steps_per_generation=5, elites_refined=64,
        plain_rollouts_per_s=rate_p,
        first_tick_best_cost={"plain": costs_p[0], "refined": costs_r[0]})
    return out


def batched_workload(E, W, mode=0, ticks=200):
    """C5: 512 uneven problems, one tick per HIP-graph replay; mode 0 the
    per-class launches (autotuned), 1 the persistent work-queue form."""
    import torch

    out = {}
    probs, ga = W.config_c5(512, 0)
    dps = [E.DeviceProblem(p.cast(np.float32), torch.float32) for p in probs]
    t_tune = time.perf_counter()
    bs = E.BatchSolver(dps, ga, autotune=mode == 0)  # autotunes the launch shapes
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
    warm = 10
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
    lats = np.array(lats)
    out["c5_fp32_512_problems" + ("_persistent" if mode else "")] = summary(
        len(probs) * ga.pop * ga.generations * ticks / wall, lats, ticks=ticks, dtype="f32",
        problems=len(probs), within_2ms=float(np.mean(lats <= 2.0)),
        plan_and_autotune_s=round(t_tune, 3),
        shapes=["%s%s x%d: shape %d of us %s, stream %d" % (
            "lin" if c["model"] == "linear" else "chain", list(c["shape"]), c["problems"],
            c["variant"], c["tuned_us"], c["stream"]) for c in bs.classes()])
    bs.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed control ticks")
    ap.add_argument("--warmup", type=int, default=5, help="untimed control ticks")
    ap.add_argument("--cpu-ticks", type=int, default=8, help="oracle ticks for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the other configurations (C1, C3, C4, C5, C2 variants)")
    ap.add_argument("--only", choices=WORKLOADS, default=None,
                    help="run only this other configuration (for profiling) and print "
                         "its summary instead of the benchmark line")
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
    if args.only:
        print(json.dumps(other_workloads(E, W, (args.only,))), flush=True)
        return
    prob, ga = W.config_c2(0)
    dtype = torch.float32
    dp = E.DeviceProblem(prob, dtype)
    solver = E.Solver(dp, ga)
    prof_ticks = min(args.steps, 20)
    total = args.warmup + args.steps
    x = torch.tensor(W.draw_x0(prob.n, 0), dtype=dtype, device="cuda")
    x_next = torch.empty_like(x)
    noise = torch.tensor(W.process_noise(prob.n, total + prof_ticks, 0), dtype=dtype,
                         device="cuda")
    u_host = torch.empty(prob.m, dtype=dtype).pin_memory()
    j_host = torch.empty(1, dtype=dtype).pin_memory()
    done = torch.cuda.Event()

    def tick(t):
        nonlocal x, x_next
        t0 = time.perf_counter()
        u, J = solver.solve(x, t)
        u_host.copy_(u, non_blocking=True)
        j_host.copy_(J, non_blocking=True)
        done.record()
        done.synchronize()
        lat = time.perf_counter() - t0
        E.empc_plant_step(dp, x, u, noise[t], x_next)
        x, x_next = x_next, x
        return lat

    for t in range(args.warmup):
        tick(t)
    # timed ticks: no timing markers in the stream
    lats = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for t in range(args.warmup, total):
        lats.append(tick(t))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    final_cost = float(j_host.item())
    # the same closed loop continued with HIP events around every rollout
    # launch (the start / stop markers add dispatch latency to the tick, so
    # they stay out of the throughput figure)
    E.empc_profile_begin(prof_ticks * ga.generations)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    for t in range(total, total + prof_ticks):
        tick(t)
    torch.cuda.synchronize()
    prof_wall = time.perf_counter() - tp
    launches, kernel_ms = E.empc_profile_end()

    rollouts = ga.pop * ga.generations * args.steps
    lat_ms = np.array(lats) * 1e3
    flop_launch = ga.pop * linear_flop_per_candidate(prob.n, prob.m, prob.T, prob.p)
    avg_launch_s = kernel_ms * 1e-3 / max(launches, 1)
    achieved = flop_launch / avg_launch_s
    traffic = traffic_entry()
    out = {
        "metric": METRIC,
        "value": rollouts / wall,
        "unit": "rollouts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "EMPC closed loop, 14-DoF linear mass-spring-damper chain "
                               "(n=28, m=14), ZOH dt=0.01, horizon 50, 10 knots, pop 4096, "
                               "64 elites, 20 generations/tick, sigma 0.1, seed 0",
                   "n": prob.n, "m": prob.m, "T": prob.T, "p": prob.p, "pop": ga.pop,
                   "n_elite": ga.n_elite, "generations": ga.generations,
                   "ticks": args.steps},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)),
                       "p99": float(np.percentile(lat_ms, 99)),
                       "mean": float(lat_ms.mean()), "max": float(lat_ms.max())},
        "kernel": {"name": "roll_linear_split", "launches": launches,
                   "timed_ticks": prof_ticks,
                   "ms_per_step_with_events": prof_wall * 1e3 / prof_ticks,
                   "mean_us": avg_launch_s * 1e6,
                   "rollouts_per_s": ga.pop / avg_launch_s,
                   "flop_per_launch": flop_launch},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP32_MFMA / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA, "traffic": traffic},
        "final_best_cost": final_cost,
    }
    if not args.no_workloads:
        out["workloads"] = other_workloads(E, W)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, ga, args.cpu_ticks)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

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
  roofline    rollout kernel: algorithmic FLOP per launch over the mean
              launch time from HIP events recorded around every rollout
              launch of the timed ticks, against the FP32 matrix-core peak;
  cpu_baseline the FP64 oracle on a bounded sample of the same workload.

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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rollout_linear_c2_traffic.json")
ROLLOUT_SRC = os.path.join(ROOT, "paper_2001_04931_amd", "csrc", "rollout.hip")


def linear_flop_per_step(n, m):
    # knot interpolation 3m, A_d x 2n^2, B_d u 2nm, stage cost 3n + 3m
    return 2 * n * n + 2 * n * m + 3 * n + 6 * m


def traffic_entry():
    """HBM bytes per rollout launch from the committed counter summary, or
    None when absent or taken on a different rollout kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    with open(ROLLOUT_SRC, "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()
    if t.get("rollout_src_sha256") != h:
        return None
    return t.get("bytes_per_launch")


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


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed control ticks")
    ap.add_argument("--warmup", type=int, default=5, help="untimed control ticks")
    ap.add_argument("--cpu-ticks", type=int, default=4, help="oracle ticks for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the EMPC hot path here is a single-GPU "
              "build (multi-GPU sharding is described, not implemented); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2001_04931_amd as E
    import workloads as W

    torch.cuda.set_device(0)
    prob, ga = W.config_c2(0)
    dtype = torch.float32
    dp = E.DeviceProblem(prob, dtype)
    solver = E.Solver(dp, ga)
    total = args.warmup + args.steps
    x = torch.tensor(W.draw_x0(prob.n, 0), dtype=dtype, device="cuda")
    x_next = torch.empty_like(x)
    noise = torch.tensor(W.process_noise(prob.n, total, 0), dtype=dtype, device="cuda")
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
    torch.cuda.synchronize()
    E.empc_profile_begin(args.steps * ga.generations)
    lats = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for t in range(args.warmup, total):
        lats.append(tick(t))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    launches, kernel_ms = E.empc_profile_end()
    final_cost = float(j_host.item())

    rollouts = ga.pop * ga.generations * args.steps
    lat_ms = np.array(lats) * 1e3
    flop_launch = ga.pop * prob.T * linear_flop_per_step(prob.n, prob.m)
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
        "kernel": {"name": "roll_linear_mfma", "launches": launches,
                   "mean_us": avg_launch_s * 1e6,
                   "rollouts_per_s": ga.pop / avg_launch_s,
                   "flop_per_launch": flop_launch},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP32_MFMA / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA, "traffic": traffic},
        "final_best_cost": final_cost,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, ga, args.cpu_ticks)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

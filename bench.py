"""Benchmark: RVE solves/s to residual 1e-6 on held-out 256x256 random-fibre
RVEs with the adapted 5% pattern (M = 3277), one MI355X.

A step is one batched solve (mor_solve_multi) of the whole batch of RVEs,
each RVE with its own microstructure and macro strain, from its start to
residual < 1e-6 (every RVE), including the final stress evaluation.  Inputs
(plans, macro strains) are resident on the device before the timed region.

Prints one JSON line (rank 0).  Beside the headline value it reports the
per-kernel roofline of the dominant kernel (HIP events around its launches
inside the timed region, algorithmic bytes counted by the kernels), the plain
single-RVE rate, the plan-construction cost, and the FP64 CPU oracle on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "RVE solves/s at residual 1e-6, 256² 2D 5% freqs: learned/batched vs plain"
GRID = 256
M_FREQ = int(math.ceil(0.05 * GRID * GRID))
TOL = 1e-6


def _gen(i):
    return synth.metric_rve(i, n=GRID)


def workload(count, workers=8):
    with ProcessPoolExecutor(max_workers=workers) as ex:
        items = list(ex.map(_gen, range(count), chunksize=8))
    gs = [g for g, _ in items]
    ebs = np.stack([e for _, e in items])
    return gs, ebs


def phases():
    import paper_2103_10203_amd as mor
    lm, mm = synth.phase_lame(synth.MATRIX_E, synth.MATRIX_NU)
    li, mi = synth.phase_lame(synth.FIBRE_E, synth.FIBRE_NU)
    return [mor.Phase(lm, mm), mor.Phase(li, mi)]


def cpu_baseline(gs, ebs, budget_s=15.0):
    """The FP64 oracle, as it stands, on the first RVEs of the same workload."""
    from oracle import material, pattern, solver
    lm, mm = synth.phase_lame(synth.MATRIX_E, synth.MATRIX_NU)
    li, mi = synth.phase_lame(synth.FIBRE_E, synth.FIBRE_NU)
    ph = (material.Phase(lm, mm), material.Phase(li, mi))
    done = 0
    t_solve = 0.0
    t_plan = 0.0
    its = []
    t0 = time.perf_counter()
    while done < len(gs) and time.perf_counter() - t0 < budget_s:
        tp = time.perf_counter()
        p = pattern.build_pattern(gs[done], M_FREQ)
        t_plan += time.perf_counter() - tp
        ts = time.perf_counter()
        r = solver.solve(gs[done], ph, solver.macro_tensor(ebs[done], 2), mask=p.mask(), tol=TOL)
        t_solve += time.perf_counter() - ts
        its.append(r.iterations)
        done += 1
    return {
        "value": done / t_solve,
        "unit": "RVE solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{done} held-out 256x256 RVEs (M={M_FREQ}, residual {TOL:g}), FP64 NumPy oracle, "
                  f"single thread, pattern construction excluded (with it: {done / (t_solve + t_plan):.3f}/s)",
        "mean_iterations": float(np.mean(its)),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--single", type=int, default=32, help="RVEs timed one launch each (plain path)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the batched RVE solves would shard across GPUs without per-iteration "
              "communication; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    import paper_2103_10203_amd as mor

    B = args.batch
    t = time.perf_counter()
    gs, ebs = workload(B)
    t_gen = time.perf_counter() - t
    ph = phases()

    torch.cuda.synchronize()
    t = time.perf_counter()
    plans = [mor.Plan(g, M_FREQ) for g in gs]
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t) * 1e3 / B
    plan_of = np.arange(B)

    # warmup (untimed)
    for _ in range(args.warmup):
        mor.solve_multi(plans, plan_of, ebs, ph, TOL)

    # timed region, with per-kernel HIP events inside the library
    mor.profile_reset()
    mor.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = None
    for _ in range(args.steps):
        out = mor.solve_multi(plans, plan_of, ebs, ph, TOL)
        iters = out.iterations
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    mor.profile_enable(False)
    assert out.status == mor.MOR_OK, out.status
    kern = {k: mor.profile_query(k) for k in ("row", "col", "final", "init")}
    dom = max(kern, key=lambda k: kern[k]["ms"])
    kd = kern[dom]
    achieved = kd["bytes"] / (kd["ms"] * 1e-3) / 1e9 if kd["ms"] > 0 else 0.0

    value = B * args.steps / elapsed
    ms_per_step = elapsed * 1e3 / args.steps

    # plain path: one RVE per launch
    ns = min(args.single, B)
    single = None
    if ns > 0:
        for i in range(2):
            mor.solve(plans[i], ebs[i:i + 1], ph, TOL)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(ns):
            mor.solve(plans[i], ebs[i:i + 1], ph, TOL)
        torch.cuda.synchronize()
        single = ns / (time.perf_counter() - t)

    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "RVE solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"held-out random-fibre RVEs {GRID}x{GRID} (vf~U[0.2,0.5], r~U[8,16] px), "
                        f"adapted pattern M={M_FREQ} (5%), batch {B} in one mor_solve_multi call, "
                        f"residual {TOL:g}, cold start",
            "grid": [GRID, GRID],
            "M": M_FREQ,
            "batch": B,
            "tol": TOL,
            "start": "cold",
            "fields": "FP32, FP64 residual and stress sums",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "avg_launch_us": kd["ms"] * 1e3 / max(kd["launches"], 1),
            "launches": kd["launches"],
        },
        "kernels": {k: {"ms": v["ms"], "launches": v["launches"],
                        "GBps": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 else 0.0}
                    for k, v in kern.items()},
        "iterations": {"mean": float(np.mean(iters)), "p50": float(np.percentile(iters, 50)),
                       "p95": float(np.percentile(iters, 95)), "max": int(np.max(iters))},
        "plain_single_rve_solves_per_s": single,
        "plan_ms_per_rve": plan_ms,
        "end_to_end_solves_per_s": 1.0 / (1.0 / value + plan_ms * 1e-3),
        "workload_gen_s": t_gen,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(gs, ebs, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

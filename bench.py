"""Benchmark of the solver-free componentwise ADMM on one MI355X.

A step is one complete solve (Algorithm 1 from the default start point until
the relative residual test holds at eps_rel = 1e-4, rho = 100) of the seeded
synthetic 8500-bus feeder, with the problem already resident in HBM (set-up is
done and timed separately).  `value` is ADMM iterations per second over the
timed steps; `ms_per_step` is the time to tolerance.

    python bench.py [--steps K] [--warmup W] [--workload 8500bus] [--precision mixed|fp64]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "8500-bus ADMM iters/s & time-to-1e-4 residual; served solves/s + p99 latency"


def algorithmic_bytes_per_iteration(sum_ns2, L, n, elem):
    """Minimum bytes one iteration must move without re-use tricks: the
    factors (elem * sum n_s^2), per slot bbar, index, lambda and z read+write
    and the consensus gathers ((7 elem + 8) L), per variable the x gather and
    write, bounds and row pointer ((4 elem + 4) n)."""
    return elem * sum_ns2 + (7 * elem + 8) * L + (4 * elem + 4) * n


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="8500bus")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--check-every", type=int, default=1024)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--kernel", default="auto", choices=["auto", "step", "persistent"])
    ap.add_argument("--block-waves", type=int, default=0)
    ap.add_argument("--fixed-iters", type=int, default=0,
                    help="time this many iterations per step instead of solving to tolerance")
    return ap.parse_args()


def cpu_baseline(inst, eps, budget_s):
    """The FP64 oracle timed on the host on a bounded sample of the same
    workload: as many iterations of Algorithm 1 as fit in about budget_s."""
    import numpy as np
    from oracle import admm
    P = admm.setup(inst)
    t0 = time.perf_counter()
    admm.solve(P, rho=100.0, eps_rel=eps, fixed_iters=20, record=False)
    per = (time.perf_counter() - t0) / 20
    iters = max(20, int(budget_s / max(per, 1e-6)))
    t0 = time.perf_counter()
    admm.solve(P, rho=100.0, eps_rel=eps, fixed_iters=iters, record=False)
    dt = time.perf_counter() - t0
    try:
        aff = len(os.sched_getaffinity(0))
    except Exception:
        aff = os.cpu_count()
    return {"value": iters / dt, "unit": "iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} FP64 iterations of the same {inst.name} instance from the default start "
                      f"({dt:.1f} s, NumPy single thread; host affinity {aff} cores)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch
    from opfgen import build_instance, by_name
    from paper_2501_08293_amd import OPF_PREC_FP64, OPF_PREC_MIXED, Solver

    dev = torch.device("cuda:0")
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    inst = build_instance(by_name(args.workload, args.seed))
    gen_s = time.perf_counter() - t0
    stream = torch.cuda.Stream()
    prec = OPF_PREC_MIXED if args.precision == "mixed" else OPF_PREC_FP64
    flat = (inst.n, inst.c, inst.lb, inst.ub, inst.var_kind) + tuple(inst.flat())
    kern = {"auto": 0, "step": 1, "persistent": 2}[args.kernel]
    solver = Solver(*flat, rho=100.0, eps_rel=args.eps, precision=prec, check_every=args.check_every,
                    kernel=kern, block_waves=args.block_waves, stream=stream.cuda_stream)
    info = solver.info()
    x = torch.zeros(inst.n, dtype=torch.float64, device=dev)
    fixed = args.fixed_iters or None
    for _ in range(args.warmup):
        solver.solve(x=x, fixed_iters=fixed)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    results = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        r = solver.solve(x=x, fixed_iters=fixed)
        ev[k][1].record(stream)
        results.append(r)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    dev_ms = sum(a.elapsed_time(b) for a, b in ev)
    iters = sum(r["iterations"] for r in results)
    it32 = sum(r["iterations_fp32"] for r in results)
    it64 = iters - it32
    value = iters / wall
    # dominant kernel: the fused iteration (FP32 bulk in mixed mode)
    elem = 4 if prec == OPF_PREC_MIXED else 8
    bpi32 = algorithmic_bytes_per_iteration(info.sum_ns2, inst.L, inst.n, 4)
    bpi64 = algorithmic_bytes_per_iteration(info.sum_ns2, inst.L, inst.n, 8)
    alg_bytes = bpi32 * it32 + bpi64 * it64
    achieved = alg_bytes / (dev_ms * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == OPF_PREC_MIXED else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{inst.name} seed {args.seed}: synthetic radial feeder, S={inst.S} components, "
                        f"n={inst.n} variables, L={inst.L} local slots; rho=100, eps_rel={args.eps:g}",
            "precision": args.precision,
            "iterations_per_solve": results[-1]["iterations"],
            "iterations_fp32_per_solve": results[-1]["iterations_fp32"],
            "time_to_tolerance_ms": round(1e3 * wall / args.steps, 3),
            "objective": results[-1]["objective"],
            "setup_ms": round(info.setup_ms, 1),
            "generator_s": round(gen_s, 2),
            "waves": info.waves,
            "lanes": info.lanes,
            "kernel": {1: "step", 2: "persistent"}.get(info.kernel, "?"),
            "block_waves": info.block_waves,
            "workgroups": info.grid_blocks,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "kernel": "admm_step_kernel (fused global+local+dual+residual iteration)",
            "bytes_per_iteration_fp32": bpi32,
            "bytes_per_iteration_fp64": bpi64,
            "avg_iteration_us": round(1e3 * dev_ms / iters, 3),
        },
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(inst, args.eps, args.cpu_seconds)
    solver.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

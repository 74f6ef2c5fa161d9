"""Benchmark of the solver-free componentwise ADMM on one MI355X.

Headline (`value`): the synthetic 8500-bus feeder, solved from the default
start point until the paper's relative residual test holds at eps_rel = 1e-4
(rho = 100), with the problem resident in HBM (set-up done and timed
separately).  A step is one complete solve; `value` is ADMM iterations per
second over the timed steps and `ms_per_step` is the time to tolerance.

Also reported on the same JSON line:
  * roofline of the dominant kernel (the FP32 persistent iteration kernel),
  * the FP64 CPU oracle on a bounded sample of the same workload,
  * batch: 256 load scenarios of a 2500-bus feeder on the MFMA path,
  * serving: a Poisson stream of mixed-size, reconfigured feeders through the
    serving runtime, against the same stream served one solve at a time.

    python bench.py [--steps K] [--warmup W] [--skip-batch] [--skip-serve]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# residual balancing of the penalty measured beside the fixed-penalty headline
BALANCE = dict(rho_every=10)
BF16_DENSE_PEAK_TFLOPS = 2500.0
METRIC = "8500-bus ADMM iters/s & time-to-1e-4 residual; served solves/s + p99 latency"
KERNEL_SOURCES = ["paper_2501_08293_amd/csrc/admm_persistent.hip", "paper_2501_08293_amd/csrc/admm_kernels.h",
                  "paper_2501_08293_amd/csrc/admm_sync.h"]


def algorithmic_bytes_per_iteration(sum_ns2, L, n, elem):
    """Minimum bytes one iteration must move without re-using data across
    iterations: the factors (elem * sum n_s^2), per slot bbar, index, lambda
    and z read+write and the consensus gathers ((7 elem + 8) L), per variable
    the x gather and write, bounds and row pointer ((4 elem + 4) n)."""
    return elem * sum_ns2 + (7 * elem + 8) * L + (4 * elem + 4) * n


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="8500bus")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--kernel", default="auto", choices=["auto", "step", "persistent", "tiled"])
    ap.add_argument("--block-waves", type=int, default=0)
    ap.add_argument("--autotune", type=int, default=1, choices=[0, 1],
                    help="schedule, workgroup shape and batch workgroup order chosen by the library's autotuner")
    ap.add_argument("--workgroup-order", type=int, default=0, choices=[0, 1],
                    help="persistent kernel: 0 = hardware workgroup order, 1 = XCD-contiguous packing ranges")
    ap.add_argument("--check-every", type=int, default=1024)
    ap.add_argument("--max-iter", type=int, default=1_000_000, help="iteration cap of the single-instance solve")
    ap.add_argument("--fixed-iters", type=int, default=0,
                    help="time this many iterations per step instead of solving to tolerance")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--skip-more", action="store_true", help="skip the other single-instance legs")
    ap.add_argument("--skip-batch", action="store_true")
    ap.add_argument("--batch-workload", default="2500bus")
    ap.add_argument("--batch-k", type=int, default=256)
    ap.add_argument("--batch-fixed", type=int, default=0,
                    help="run this many batch iterations instead of solving to tolerance (counter passes)")
    ap.add_argument("--skip-serve", action="store_true")
    ap.add_argument("--serve-families", type=int, default=16)
    ap.add_argument("--serve-requests", type=int, default=120)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--serve-eps", type=float, default=1e-3)
    ap.add_argument("--serve-chunk", type=int, default=512,
                    help="iterations each resident solve runs per shared launch")
    ap.add_argument("--only", choices=["batch", "serve"], default=None,
                    help="run only this leg and print its record (for profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device copy of known size (counter calibration for profiles)")
    return ap.parse_args()


def cpu_baseline(inst, eps, budget_s, workload):
    """The FP64 oracle timed on the host on a bounded sample of the same
    workload: as many iterations of Algorithm 1 as fit in about budget_s, in
    one process and with the components split over worker processes (the
    paper's CPU runs); time to tolerance extrapolated from the oracle's
    stored iteration count at this tolerance."""
    from threadpoolctl import threadpool_limits
    from oracle import admm
    from oracle.parallel import solve_parallel
    with threadpool_limits(limits=1):
        return _cpu_baseline(admm, solve_parallel, inst, eps, budget_s, workload)


def _cpu_baseline(admm, solve_parallel, inst, eps, budget_s, workload):
    P = admm.setup(inst)
    t0 = time.perf_counter()
    admm.solve(P, rho=100.0, eps_rel=eps, fixed_iters=20, record=False)
    per = (time.perf_counter() - t0) / 20
    iters = max(20, int(budget_s / 2 / max(per, 1e-6)))
    t0 = time.perf_counter()
    admm.solve(P, rho=100.0, eps_rel=eps, fixed_iters=iters, record=False)
    dt1 = time.perf_counter() - t0
    rate1 = iters / dt1
    try:
        aff = len(os.sched_getaffinity(0))
    except Exception:
        aff = os.cpu_count()
    procs = max(1, min(16, aff) - 1)
    itp = max(20, int(budget_s / 2 * rate1))
    t0 = time.perf_counter()
    solve_parallel(P, procs, rho=100.0, eps_rel=eps, fixed_iters=itp)
    dtp = time.perf_counter() - t0
    ratep = itp / dtp
    ref = stored_reference(workload, eps)
    out = {"value": round(ratep, 2), "unit": "iters/s", "cores": procs + 1, "kind": "oracle",
           "sample": f"{itp} FP64 iterations of Algorithm 1 on the same {inst.name} instance from the default start "
                     f"({dtp:.1f} s; components split over {procs} worker processes, global update and "
                     f"termination test in the master; NumPy, one BLAS thread each; host affinity {aff} cores)",
           "one_process": {"value": round(rate1, 2), "unit": "iters/s", "cores": 1,
                           "sample": f"{iters} iterations in {dt1:.1f} s"}}
    if "oracle_iterations" in ref:
        out["time_to_tolerance_s_extrapolated"] = round(ref["oracle_iterations"] / ratep, 1)
        out["one_process"]["time_to_tolerance_s_extrapolated"] = round(ref["oracle_iterations"] / rate1, 1)
        out["oracle_iterations_to_tolerance"] = ref["oracle_iterations"]
    return out


def copy_calibration():
    """A plain device copy of 256 MiB (reads 256 MiB, writes 256 MiB): the
    reference for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = 256 * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}), flush=True)


def stored_reference(workload, eps):
    """Objective of the FP64 oracle's solve to eps and of the LP optimum
    (HiGHS on the centralised LP), as stored under tests/golden (None when
    not stored)."""
    g = os.path.join(ROOT, "tests", "golden")
    adm = os.path.join(g, f"admm_{workload}_s0_eps{eps:g}.json")
    lp = os.path.join(g, f"lp_{workload}_s0.json")
    out = {}
    if os.path.exists(adm):
        d = json.load(open(adm))
        out["oracle_objective"] = d["objective"]
        out["oracle_iterations"] = d["iterations"]
        out["oracle_seconds_one_core"] = d.get("oracle_seconds")
    if os.path.exists(lp):
        out["lp_objective"] = json.load(open(lp))["objective"]
    return out


def accuracy(obj, ref):
    """Relative objective error against the oracle's solve at the same
    tolerance, and the gap to the LP optimum."""
    acc = {}
    if "oracle_objective" in ref:
        acc["objective_rel_err_vs_oracle"] = abs(obj - ref["oracle_objective"]) / abs(ref["oracle_objective"])
    if "lp_objective" in ref:
        acc["lp_gap"] = (obj - ref["lp_objective"]) / abs(ref["lp_objective"])
    return acc


def traffic_from_profiles(workload, precision):
    """HBM bytes per iteration from the committed counter summary (the json
    block of profiles/traffic_admm_persistent_<workload>_<precision>.md), if it
    was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_admm_persistent_{workload}_{precision}.md")
    if not os.path.exists(path):
        return None
    try:
        text = open(path).read()
        block = text.split("```json", 1)[1].split("```", 1)[0]
        d = json.loads(block)
    except Exception:
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d


def single_instance(args, torch):
    from opfgen import build_instance, by_name
    from paper_2501_08293_amd import OPF_PREC_FP64, OPF_PREC_MIXED, Solver
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    inst = build_instance(by_name(args.workload, args.seed))
    gen_s = time.perf_counter() - t0
    stream = torch.cuda.Stream()
    prec = OPF_PREC_MIXED if args.precision == "mixed" else OPF_PREC_FP64
    kern = {"auto": 0, "step": 1, "persistent": 2, "tiled": 3}[args.kernel]
    flat = (inst.n, inst.c, inst.lb, inst.ub, inst.var_kind) + tuple(inst.flat())
    solver = Solver(*flat, rho=100.0, eps_rel=args.eps, precision=prec, check_every=args.check_every,
                    max_iter=args.max_iter,
                    kernel=kern, block_waves=args.block_waves, workgroup_order=args.workgroup_order,
                    autotune=args.autotune, stream=stream.cuda_stream)
    info = solver.info()
    x = torch.zeros(inst.n, dtype=torch.float64, device=dev)
    fixed = args.fixed_iters or None
    for _ in range(args.warmup):
        solver.solve(x=x, fixed_iters=fixed)
    torch.cuda.synchronize()
    results = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        results.append(solver.solve(x=x, fixed_iters=fixed))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    solver.close()
    # the same set-up with the component factors computed on the device
    dev_setup = Solver(*flat, rho=100.0, eps_rel=args.eps, precision=prec, kernel=kern,
                       block_waves=args.block_waves, setup_on_device=True, stream=stream.cuda_stream)
    setup_ms_device = dev_setup.info().setup_ms
    dev_setup.close()
    iters = sum(r["iterations"] for r in results)
    it32 = sum(r["iterations_fp32"] for r in results)
    it64 = iters - it32
    k32 = sum(r["kernel_ms_fp32"] for r in results)
    k64 = sum(r["kernel_ms"] for r in results) - k32
    bpi32 = algorithmic_bytes_per_iteration(info.sum_ns2, inst.L, inst.n, 4)
    bpi64 = algorithmic_bytes_per_iteration(info.sum_ns2, inst.L, inst.n, 8)
    # dominant kernel: the FP32 bulk in mixed mode, FP64 otherwise
    bw = info.block_waves
    if prec == OPF_PREC_MIXED and it32 > 0:
        dom_name, dom_bytes, dom_ms, dom_iters = f"admm_persistent_kernel<float, {bw}>", bpi32, k32, it32
    else:
        dom_name, dom_bytes, dom_ms, dom_iters = f"admm_persistent_kernel<double, {bw}>", bpi64, k64, it64
    dom_launches = args.steps
    if info.kernel == 1:
        dom_name = dom_name.replace("persistent", "step")
        dom_launches = dom_iters
    elif info.kernel == 3:
        dom_name = dom_name.replace("persistent", "tiled_pair" if info.tiled_pair else "tiled")
    achieved = dom_bytes * dom_iters / (dom_ms * 1e-3) / 1e9 if dom_ms > 0 else 0.0
    tr = traffic_from_profiles(args.workload, args.precision)
    traffic = None
    if tr is not None and tr.get("kernel", "").replace(", false", "") == dom_name:
        traffic = round(tr["bytes_per_iteration"] * dom_iters / max(dom_launches, 1))
    line = {
        "metric": METRIC,
        "value": round(iters / wall, 1),
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
            "status": results[-1]["status"],
            "objective": results[-1]["objective"],
            "setup_ms": round(info.setup_ms, 1),
            "setup_ms_device_factors": round(setup_ms_device, 1),
            "generator_s": round(gen_s, 2),
            "waves": info.waves,
            "lanes": info.lanes,
            "kernel": {1: "step", 2: "persistent", 3: "tiled"}.get(info.kernel, "?"),
            "block_waves": info.block_waves,
            "workgroups": info.grid_blocks,
            "factors_in_lds": info.factors_in_lds,
            "fp64_lds_workgroups": info.fp64_lds_workgroups,
            "kernel_ms_per_solve": round(sum(r["kernel_ms"] for r in results) / args.steps, 3),
            **accuracy(results[-1]["objective"], stored_reference(args.workload, args.eps)),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            # achieved counts the algorithmic bytes (factors once per iteration although they stay in LDS);
            # the HBM rate the counters measure for the same launch:
            "traffic_gbs": round(traffic / (dom_ms / max(dom_launches, 1) * 1e-3) / 1e9, 1) if traffic else None,
            "kernel": dom_name,
            "bytes_per_iteration": dom_bytes,
            "avg_launch_ms": round(dom_ms / max(dom_launches, 1), 4),
            "avg_iteration_us": round(1e3 * dom_ms / max(dom_iters, 1), 3),
            "kernel_source_hash": kernel_source_hash(),
        },
    }
    return line, inst


def solve_leg(workload, precision, eps, torch, steps=1, fixed=None, warm=True, **kw):
    """One workload solved `steps` times (or `fixed` iterations timed), with
    the problem resident on the device: iterations, time, rate, accuracy and
    the algorithmic-bytes rate of its iteration kernel."""
    from opfgen import build_instance, by_name
    from paper_2501_08293_amd import OPF_PREC_FP64, OPF_PREC_MIXED, Solver
    inst = build_instance(by_name(workload, 0))
    prec = OPF_PREC_MIXED if precision == "mixed" else OPF_PREC_FP64
    stream = torch.cuda.Stream()
    s = Solver(inst.n, inst.c, inst.lb, inst.ub, inst.var_kind, *inst.flat(), rho=100.0, eps_rel=eps,
               precision=prec, check_every=1024, stream=stream.cuda_stream, max_iter=3_000_000, **kw)
    info = s.info()
    x = torch.zeros(inst.n, dtype=torch.float64, device="cuda")
    if warm:
        s.solve(x=x, fixed_iters=fixed)                  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [s.solve(x=x, fixed_iters=fixed) for _ in range(steps)]
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    s.close()
    r = outs[-1]
    it = int(r["iterations"])
    elem = 4 if prec == OPF_PREC_MIXED else 8
    bpi = algorithmic_bytes_per_iteration(info.sum_ns2, inst.L, inst.n, elem)
    kms = r["kernel_ms_fp32"] if prec == OPF_PREC_MIXED else r["kernel_ms"]
    kit = int(r["iterations_fp32"]) if prec == OPF_PREC_MIXED else it
    gbs = bpi * kit / (kms * 1e-3) / 1e9 if kms > 0 else 0.0
    out = {"workload": f"{inst.name}: S={inst.S}, n={inst.n}, L={inst.L}", "precision": precision,
           "eps_rel": eps, "status": int(r["status"]), "iterations": it, "iterations_fp32": int(r["iterations_fp32"]),
           "ms": round(1e3 * wall, 3), "iters_per_s": round(it / wall, 1),
           "kernel": {1: "step", 2: "persistent", 3: "tiled"}.get(info.kernel, "?"), "workgroups": info.grid_blocks,
           "us_per_iteration": round(1e3 * kms / max(kit, 1), 3),
           "algorithmic_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
           "objective": r["objective"]}
    if info.kernel == 3:
        out["tiles_per_workgroup"] = "two in flight" if info.tiled_pair else "in turn"
    if kw:
        out["options"] = kw
        out["rho_final"] = r["rho_final"]
    if fixed is None:
        acc = accuracy(r["objective"], stored_reference(workload, eps))
        if kw.get("rho_every") or kw.get("local_updates", 1) > 1:
            acc.pop("objective_rel_err_vs_oracle", None)    # the stored solve is Algorithm 1 with fixed rho
        out.update(acc)
    return out


def more_legs(args, torch):
    """The other single-instance workloads of the measurement plan: the
    headline feeder in FP64 (every step FP64), the 13- and 123-bus feeders
    in both precisions, the 21000-bus (~30k component) feeder at a fixed
    iteration count, and the headline with residual balancing of the penalty."""
    legs = {}
    legs["8500bus_fp64"] = solve_leg("8500bus", "fp64", args.eps, torch)
    for w in ("13bus", "123bus"):
        for p in ("fp64", "mixed"):
            legs[f"{w}_{p}"] = solve_leg(w, p, args.eps, torch, steps=5)
    legs["21000bus_mixed_fixed4096"] = solve_leg("21000bus", "mixed", args.eps, torch, fixed=4096)
    legs["21000bus_fp64_fixed4096"] = solve_leg("21000bus", "fp64", args.eps, torch, fixed=4096)
    legs["21000bus_mixed_step_fixed4096"] = solve_leg("21000bus", "mixed", args.eps, torch, fixed=4096, kernel=1)
    legs["21000bus_mixed"] = solve_leg("21000bus", "mixed", args.eps, torch, warm=False)
    legs["8500bus_mixed_balanced"] = solve_leg("8500bus", "mixed", args.eps, torch, **BALANCE)
    return legs


def batch_leg(args, torch):
    import numpy as np
    from opfgen import build_instance, by_name, scenario_load_factors, scenario_rhs
    from paper_2501_08293_amd import BatchSolver
    f = by_name(args.batch_workload, args.seed)
    inst = build_instance(f)
    K = args.batch_k
    B = scenario_rhs(inst, scenario_load_factors(f, K, seed=1000))
    st = torch.cuda.Stream()
    fixed = args.batch_fixed > 0
    t_setup = time.perf_counter()
    s = BatchSolver(inst.n, inst.c, inst.lb, inst.ub, inst.var_kind, *inst.flat(), b_scen=B, rho=100.0,
                    eps_rel=1e-12 if fixed else args.eps, max_iter=args.batch_fixed if fixed else 1_000_000,
                    check_every=256, stream=st.cuda_stream, autotune=bool(args.autotune))
    setup_s = time.perf_counter() - t_setup
    info = s.info()
    t0 = time.perf_counter()
    out = s.solve()
    wall = time.perf_counter() - t0
    s.close()
    it = out["iterations"]
    T = int(out["total_iterations"])
    # MFMA work issued per batch iteration: per packed wavefront and 64-scenario
    # chunk, 4 tiles x 4 k-steps x 6 products of 32x32x16
    chunks = (K + 63) // 64
    mfma_flops = info.waves * chunks * 4 * 4 * 6 * (2 * 32 * 32 * 16) * T
    useful_flops = 2 * info.sum_ns2 * int(it.sum())
    tf = mfma_flops / wall / 1e12
    # algorithmic bytes of one batch iteration: the shared FP64 factors once
    # (8 sum n_s^2) and, per slot and scenario with FP32 state, lambda and z
    # read and written, the x gather and bbar (24 B)
    bytes_iter = 8 * info.sum_ns2 + K * inst.L * 24
    gbs = bytes_iter * T / wall / 1e9
    # what this design moves: z and lambda read+write and bbar per slot (20 L),
    # the consensus reads of z and lambda of every copy of each slot's variable
    # (8 sum_i N_i^2), the x write (4 n) per padded scenario column, and the
    # three bf16 factor planes (3 * 2 * 64 * 64 per wave)
    cnt = np.bincount(np.concatenate([c.idx for c in inst.comps]), minlength=inst.n).astype(np.int64)
    per_col = 20 * inst.L + 8 * int((cnt * cnt).sum()) + 4 * inst.n
    design_bytes = 64 * chunks * per_col + 3 * 2 * 64 * 64 * info.waves
    return {
        "workload": f"{inst.name}: {K} load scenarios (lognormal(0, 0.3) per bus), shared A_s; eps_rel={args.eps:g}",
        "scenarios": K, "converged": int(out["converged"]), "status": int(out["status"]),
        "time_to_all_ms": round(1e3 * wall, 1), "batch_iterations": T,
        "scenario_iterations_min_med_max": [int(it.min()), int(np.median(it)), int(it.max())],
        "scenario_solves_per_s": round(K / wall, 2),
        "scenario_iterations_per_s": round(float(it.sum()) / wall, 1),
        "us_per_batch_iteration": round(1e6 * wall / max(T, 1), 2),
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_iteration": int(bytes_iter),
                     "design_bytes_per_iteration": int(design_bytes),
                     "design_gbs": round(design_bytes * T / wall / 1e9, 1)},
        "mfma": {"issued_tflops": round(tf, 2), "peak_tflops_bf16_dense": BF16_DENSE_PEAK_TFLOPS,
                 "frac": round(tf / BF16_DENSE_PEAK_TFLOPS, 5),
                 "useful_fraction_of_issued": round(useful_flops * 6 / max(mfma_flops, 1), 4)},
        "precision": "bf16 three-term split products on MFMA, fp32 accumulate, fp32 state, fp64 residual sums",
        "workgroup_order": {0: "hardware, wavefront-major", 1: "XCD-contiguous, wavefront-major",
                            2: "hardware, chunk-major", 3: "XCD-contiguous, chunk-major"}.get(info.batch_order),
        "scenario_groups": info.batch_groups,
        "setup_s_with_autotune": round(setup_s, 2),
        "zip_loads": zip_batch_timing(args, torch, K) if not fixed else None,
    }


def zip_batch_timing(args, torch, K):
    """The same batch with voltage-dependent (ZIP) loads: components whose
    A_s change with the scenario run on per-scenario factors.  A fixed number
    of iterations is timed (per-iteration cost against the shared path)."""
    import numpy as np
    from opfgen import build_instance, by_name, scenario_load_factors, scenario_zip
    from paper_2501_08293_amd import BatchSolver
    f = by_name(args.batch_workload + "-zip", args.seed)
    inst = build_instance(f)
    b_scen, a_pos, a_scen = scenario_zip(inst, scenario_load_factors(f, K, seed=1000))
    st = torch.cuda.Stream()
    t0 = time.perf_counter()
    s = BatchSolver(inst.n, inst.c, inst.lb, inst.ub, inst.var_kind, *inst.flat(), b_scen=b_scen, rho=100.0,
                    eps_rel=1e-12, max_iter=2048, check_every=256, stream=st.cuda_stream, a_pos=a_pos,
                    a_scen=a_scen, autotune=bool(args.autotune))
    setup_s = time.perf_counter() - t0
    info = s.info()
    s.solve()
    t0 = time.perf_counter()
    out = s.solve()
    wall = time.perf_counter() - t0
    s.close()
    cm = inst.flat()[0]
    cn = inst.flat()[1]
    comp_of = np.searchsorted(np.cumsum(cm.astype(np.int64) * cn), a_pos, side="right")
    return {"workload": f"{inst.name}: {K} scenarios, {len(a_pos)} scenario-varying A entries in "
                        f"{len(np.unique(comp_of))} of {inst.S} components; 2048 iterations timed",
            "setup_s": round(setup_s, 2), "workgroup_order": info.batch_order, "scenario_groups": info.batch_groups,
            "us_per_batch_iteration": round(1e6 * wall / max(int(out["total_iterations"]), 1), 2)}


def serve_leg(args, torch, rate=None, baseline=True):
    import numpy as np
    from opfgen import build_instance, scenario_rhs
    from opfgen.serving import component_keys, make_family, poisson_arrivals, reconfigure
    from paper_2501_08293_amd import OPF_PREC_FP64, OPF_PREC_MIXED, Server, Solver
    prec = OPF_PREC_MIXED if args.serve_precision == "mixed" else OPF_PREC_FP64
    t0 = time.perf_counter()
    pool = []          # (family id, instance, component keys)
    for fid in range(args.serve_families):
        fam = make_family(fid, args.seed)
        rng = np.random.default_rng([args.seed, fid, 5])
        variants = [fam.base] + [reconfigure(fam, k, rng) for k in range(min(2, len(fam.ties)))]
        for g in variants:
            inst = build_instance(g)
            pool.append((fid, inst, component_keys(inst)))
    gen_s = time.perf_counter() - t0
    N = args.serve_requests
    rng = np.random.default_rng([args.seed, 808])
    rate = args.serve_rate if rate is None else rate
    arrivals = poisson_arrivals(N, rate, args.seed)
    reqs = []
    for k in range(N):
        fid, inst, keys = pool[int(rng.integers(len(pool)))]
        fac = np.clip(rng.lognormal(0.0, 0.3, size=(1, inst.feeder.n_bus)), 0.5, 1.0)
        b = scenario_rhs(inst, fac)[0]
        cm, cn, A, _, idx = inst.flat()
        reqs.append((fid, inst, keys, (inst.n, inst.c, inst.lb, inst.ub, inst.var_kind, cm, cn, A, b, idx)))
    # continuous batching through the serving runtime
    st = torch.cuda.Stream()
    srv = Server(rho=100.0, eps_rel=args.serve_eps, iters_per_poll=args.serve_chunk, arena_bytes=8 << 30,
                 max_workgroups=16384, setup_threads=6, precision=prec, stream=st.cuda_stream)
    done = {}
    ids = {}
    t_start = time.perf_counter()
    k = 0
    while len(done) < N:
        now = time.perf_counter() - t_start
        while k < N and arrivals[k] <= now:
            fid, inst, keys, arrs = reqs[k]
            ids[srv.submit(*arrs, family=fid, comp_keys=keys)] = k
            k += 1
        for r in srv.poll(max_out=256, wait_ms=1):
            done[ids[r["request_id"]]] = r
    span = time.perf_counter() - t_start
    sstats = srv.stats()
    srv.close()
    lat = np.array([done[i]["latency_ms"] for i in range(N)])
    ok = sum(1 for i in range(N) if done[i]["status"] == 0)
    # algorithmic bytes of every served iteration (FP32 bulk and FP64 ones at
    # their element sizes) over the served span
    served_bytes = 0.0
    for i in range(N):
        inst_i, r_i = reqs[i][1], done[i]
        s2 = sum(len(c.idx) ** 2 for c in inst_i.comps)
        it32 = int(r_i["iterations_fp32"])
        it64 = int(r_i["iterations"]) - it32
        served_bytes += (algorithmic_bytes_per_iteration(s2, inst_i.L, inst_i.n, 4) * it32 +
                         algorithmic_bytes_per_iteration(s2, inst_i.L, inst_i.n, 8) * it64)
    served_gbs = served_bytes / span / 1e9
    warm = sum(1 for i in range(N) if done[i]["warm_components"] > 0)
    print(f"[bench] served {N} requests at {rate:g}/s in {span:.1f} s", file=sys.stderr, flush=True)
    roof = {"bound": "hbm", "achieved": round(served_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(served_gbs / HBM_PEAK_GBS, 4),
            "basis": "algorithmic bytes of every served iteration over the served span"}
    if not baseline:
        return {"workload": f"{N} requests, Poisson {rate:g}/s, {args.serve_families} feeder families, "
                            f"eps_rel={args.serve_eps:g}",
                "solves_per_s": round(ok / span, 2), "span_s": round(span, 2),
                "p50_latency_ms": round(float(np.percentile(lat, 50)), 1),
                "p99_latency_ms": round(float(np.percentile(lat, 99)), 1),
                "max_latency_ms": round(float(lat.max()), 1), "converged": ok, "warm_started": warm,
                "launches": int(sstats["launches"]), "roofline": roof}
    # baseline: the same trace served one solve at a time, FIFO, cold start,
    # with the single-instance solver (set-up included, as in the runtime)
    base_lat = []
    base_ok = 0
    free_at = 0.0
    base_obj_err = []
    base_obj = []
    t_b = time.perf_counter()
    for i in range(N):
        start = max(arrivals[i], free_at)
        wait = start - (time.perf_counter() - t_b)
        if wait > 0:
            time.sleep(wait)
        fid, inst, keys, arrs = reqs[i]
        s = Solver(*arrs, rho=100.0, eps_rel=args.serve_eps, check_every=256, precision=prec, stream=st.cuda_stream)
        r = s.solve()
        s.close()
        base_ok += int(r["status"] == 0)
        free_at = time.perf_counter() - t_b
        base_lat.append(1e3 * (free_at - arrivals[i]))
        base_obj_err.append(abs(r["objective"] - done[i]["objective"]) / max(1e-12, abs(r["objective"])))
        base_obj.append(r["objective"])
    base_lat = np.array(base_lat)
    # accuracy at equal termination test: a sample stratified by feeder size
    # (per band the first warm-started and the first cold request, the
    # largest families included), each against a tight reference solve
    # (eps_rel 1e-5) of the same request
    bands = [(0, 300), (300, 1500), (1500, 4000), (4000, 10 ** 6)]
    samp = []
    for lo, hi in bands:
        inb = [i for i in range(N) if lo <= reqs[i][1].feeder.n_bus < hi]
        samp += [i for i in inb if done[i]["warm_components"] > 0][:1]
        samp += [i for i in inb if done[i]["warm_components"] == 0][:1]
    err_srv, err_base, rows = [], [], []
    for i in samp:
        s = Solver(*reqs[i][3], rho=100.0, eps_rel=1e-5, check_every=1024, precision=OPF_PREC_MIXED,
                   max_iter=4_000_000, stream=st.cuda_stream)
        ref = s.solve()["objective"]
        s.close()
        es = abs(done[i]["objective"] - ref) / max(1e-12, abs(ref))
        eb = abs(base_obj[i] - ref) / max(1e-12, abs(ref))
        err_srv.append(es)
        err_base.append(eb)
        rows.append({"buses": int(reqs[i][1].feeder.n_bus), "warm": int(done[i]["warm_components"] > 0),
                     "served": round(es, 6), "one_at_a_time": round(eb, 6)})
    return {
        "workload": f"{N} requests, Poisson {args.serve_rate:g}/s, {args.serve_families} feeder families "
                    f"(13-8500 buses log-uniform, tie-switch reconfigurations, fresh loads), eps_rel={args.serve_eps:g}",
        "precision": "FP32 bulk + FP64 polish (both served and one at a time)" if prec == OPF_PREC_MIXED else "FP64",
        "solves_per_s": round(ok / span, 2),
        "p50_latency_ms": round(float(np.percentile(lat, 50)), 1),
        "p99_latency_ms": round(float(np.percentile(lat, 99)), 1),
        "converged": ok, "warm_started": warm,
        "baseline_one_at_a_time": {"solves_per_s": round(base_ok / free_at, 2),
                                   "p50_latency_ms": round(float(np.percentile(base_lat, 50)), 1),
                                   "p99_latency_ms": round(float(np.percentile(base_lat, 99)), 1),
                                   "converged": base_ok},
        "speedup_solves_per_s": round((ok / span) / max(base_ok / free_at, 1e-9), 2),
        "max_objective_rel_diff_vs_baseline": float(max(base_obj_err)),
        "objective_rel_err_vs_eps1e-5_stratified": {
            "requests": len(samp),
            "served_max": float(max(err_srv)) if samp else None,
            "served_median": float(np.median(err_srv)) if samp else None,
            "one_at_a_time_max": float(max(err_base)) if samp else None,
            "one_at_a_time_median": float(np.median(err_base)) if samp else None,
            "per_request": rows},
        "launches": int(sstats["launches"]), "generator_s": round(gen_s, 1),
        "roofline": roof,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU only; --gpus must be 1"}), flush=True)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.only:
        leg = batch_leg(args, torch) if args.only == "batch" else serve_leg(args, torch)
        print(json.dumps({args.only: leg}), flush=True)
        return
    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    progress("single instance")
    line, inst = single_instance(args, torch)
    progress(f"single instance done: {line['ms_per_step']} ms per solve")
    if not args.skip_more:
        line["more"] = more_legs(args, torch)
        progress("more single-instance legs done")
    if not args.skip_batch:
        line["batch"] = batch_leg(args, torch)
        progress(f"batch done: {line['batch']['time_to_all_ms']} ms")
    if not args.skip_serve:
        line["serving"] = serve_leg(args, torch)
        # the same families and request mix arriving ten times slower: admission
        # while solves run (no one-at-a-time baseline)
        line["serving"]["paced"] = serve_leg(args, torch, rate=args.serve_rate / 10, baseline=False)
        progress(f"serving done: {line['serving']['solves_per_s']} solves/s")
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(inst, args.eps, args.cpu_seconds, args.workload)
        progress("cpu baseline done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Writes the stored expected values under tests/golden/ by running the FP64
oracle (oracle/) on the seeded synthetic feeders (opfgen/).  Nothing here
touches the HIP library.

    python tests/golden/make_golden.py 13bus 123bus     # seconds
    python tests/golden/make_golden.py 8500bus:1e-4     # tens of minutes
    python tests/golden/make_golden.py lp:8500bus       # LP optimum by HiGHS
    python tests/golden/make_golden.py 2500bus@scen3:1e-4   # scenario 3 of the batch benchmark
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from opfgen import build_instance, by_name, scenario_load_factors, scenario_rhs, with_rhs  # noqa: E402
from oracle import admm  # noqa: E402
from oracle.central import CentralLP  # noqa: E402

RHO = 100.0


def golden(name, seed=0, eps_rel=1e-4, n_sample=256, scenario=None):
    f = by_name(name, seed)
    inst = build_instance(f)
    tag = name
    if scenario is not None:
        # scenario k of the benchmark's batch: every bus's load scaled by the
        # k-th draw of lognormal(0, 0.3) (stream seed 1000, 256 scenarios)
        k = int(scenario)
        inst = with_rhs(inst, scenario_rhs(inst, scenario_load_factors(f, 256, seed=1000))[k])
        tag = f"{name}-scen{k}"
    P = admm.setup(inst)
    t0 = time.time()
    r = admm.solve(P, rho=RHO, eps_rel=eps_rel, max_iter=2_000_000, record=True, progress=5000)
    dt = time.time() - t0
    vidx = np.nonzero(inst.var_kind == 2)[0]
    rng = np.random.default_rng(12345)
    samp = np.sort(rng.choice(vidx, size=min(n_sample, len(vidx)), replace=False))
    xs = np.sort(rng.choice(inst.n, size=min(n_sample, inst.n), replace=False))
    hist = r.history
    m = hist[:, 0] ** 2 + (hist[:, 1] / RHO) ** 2
    out = dict(
        workload=tag, seed=seed, rho=RHO, eps_rel=eps_rel, stats=inst.stats(),
        iterations=int(r.iterations), converged=bool(r.converged), objective=r.objective,
        pres=r.pres, dres=r.dres, eps_prim=r.eps_prim, eps_dual=r.eps_dual,
        w_index=[int(i) for i in samp], w_value=[float(r.x[i]) for i in samp],
        w_min=float(r.x[vidx].min()), w_max=float(r.x[vidx].max()), w_sum=float(r.x[vidx].sum()),
        x_sum=float(r.x.sum()),
        x_index=[int(i) for i in xs], x_value=[float(r.x[i]) for i in xs],
        z_norm=float(np.linalg.norm(r.z)), lam_norm=float(np.linalg.norm(r.lam)),
        history_every=max(1, r.iterations // 200),
        merit_history=[float(v) for v in m[::max(1, r.iterations // 200)]],
        oracle_seconds=dt,
        source="oracle/admm.py solve() on opfgen.by_name(workload, seed); written by tests/golden/make_golden.py",
    )
    path = os.path.join(HERE, f"admm_{tag}_s{seed}_eps{eps_rel:g}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"wrote {path}: {r.iterations} iterations, objective {r.objective:.12g}, {dt:.1f}s", flush=True)


def lp_golden(name, seed=0):
    """Optimum of the centralised LP (assembled from the feeder, not from the
    components) by HiGHS: the point the ADMM approaches."""
    f = by_name(name, seed)
    t0 = time.time()
    lp = CentralLP(f)
    t1 = time.time()
    res = lp.solve()
    t2 = time.time()
    inst = build_instance(f)
    pos = [lp.pos[k] for k in inst.var_keys]
    x = np.asarray(res.x)[pos]
    vidx = np.nonzero(inst.var_kind == 2)[0]
    out = dict(
        workload=name, seed=seed, objective=float(res.fun), rows=int(lp.A.shape[0]), cols=int(lp.A.shape[1]),
        w_min=float(x[vidx].min()), w_max=float(x[vidx].max()),
        assemble_seconds=t1 - t0, highs_seconds=t2 - t1,
        source="oracle/central.py CentralLP(opfgen.by_name(workload, seed)).solve() (HiGHS); "
               "written by tests/golden/make_golden.py",
    )
    path = os.path.join(HERE, f"lp_{name}_s{seed}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"wrote {path}: objective {res.fun:.12g} (assembly {t1 - t0:.1f}s, HiGHS {t2 - t1:.1f}s)", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or ["13bus", "123bus"]
    for nm in names:
        if nm.startswith("lp:"):
            lp_golden(nm[3:])
            continue
        eps = 1e-4
        if ":" in nm:
            nm, e = nm.split(":")
            eps = float(e)
        scen = None
        if "@scen" in nm:
            nm, scen = nm.split("@scen")
        golden(nm, eps_rel=eps, scenario=scen)

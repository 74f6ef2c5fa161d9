"""Seed sweep: the synthetic feeders of seeds 1-20 (13-bus, 13-bus with ZIP
and delta loads, 123-bus) through the C ABI against the FP64 oracle.

Checks: at a fixed iteration count (30) x, z and lambda agree to 1e-9
relative on both schedules (step and persistent); solved to eps_rel = 1e-3 the
stop iteration agrees within one and the objective within 1e-6 relative on
seeds 1-8 of the 13-bus and 1-4 of the 123-bus feeder."""
import sys

import numpy as np
import pytest

from opfgen import build_instance, by_name
from oracle import admm

pytestmark = pytest.mark.gpu
RHO = 100.0


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _args(inst):
    return (inst.n, inst.c, inst.lb, inst.ub, inst.var_kind) + tuple(inst.flat())


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


@pytest.mark.parametrize("name", ["13bus", "13bus-zip", "123bus"])
def test_seed_sweep_fixed_iterations(name):
    from paper_2501_08293_amd import Solver
    for seed in range(1, 21):
        _say(f"[gpu] seed sweep {name} seed {seed}, t=30")
        inst = build_instance(by_name(name, seed))
        ref = admm.solve(admm.setup(inst), rho=RHO, eps_rel=1e-4, fixed_iters=30, record=False)
        for kernel in (1, 2):
            s = Solver(*_args(inst), rho=RHO, eps_rel=1e-4, kernel=kernel)
            out = s.solve(fixed_iters=30)
            s.close()
            for key, r in (("x", ref.x), ("z", ref.z), ("lam", ref.lam)):
                assert _rel(out[key], r) <= 1e-9, (seed, kernel, key)


@pytest.mark.parametrize("name,seeds", [("13bus", 8), ("123bus", 4)])
def test_seed_sweep_solve_to_tolerance(name, seeds):
    from paper_2501_08293_amd import Solver
    for seed in range(1, seeds + 1):
        _say(f"[gpu] seed sweep {name} seed {seed}, solve to 1e-3")
        inst = build_instance(by_name(name, seed))
        ref = admm.solve(admm.setup(inst), rho=RHO, eps_rel=1e-3, record=False)
        s = Solver(*_args(inst), rho=RHO, eps_rel=1e-3)
        out = s.solve()
        s.close()
        assert out["status"] == 0 and ref.converged
        assert abs(out["iterations"] - ref.iterations) <= 1, seed
        assert abs(out["objective"] - ref.objective) <= 1e-6 * abs(ref.objective), seed

"""Residual balancing of the penalty on the GPU (through the C ABI) against
the FP64 oracle's schedule with the same lag (OPF_RHO_LAG).

Bars as for the fixed penalty: FP64 iterates within 1e-9 relative at fixed t
and the penalty reached equal (the penalties are rho times powers of tau);
at termination the iteration count within +-1 and the objective within 1e-6;
the step and persistent schedules bit for bit; mixed precision within 1e-4
of the FP64 oracle at the same tolerance."""
import sys

import numpy as np
import pytest

from opfgen import build_instance, by_name
from oracle import admm

pytestmark = pytest.mark.gpu
RHO = 100.0
STEP, PERSIST = 1, 2
KERNELS = [pytest.param(STEP, id="step"), pytest.param(PERSIST, id="persistent")]
_cache = {}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _inst(name):
    if name not in _cache:
        _cache[name] = build_instance(by_name(name, 0))
    return _cache[name]


def _P(name):
    key = ("P", name)
    if key not in _cache:
        _cache[key] = admm.setup(_inst(name))
    return _cache[key]


def _solver(inst, **kw):
    from paper_2501_08293_amd import Solver
    return Solver(inst.n, inst.c, inst.lb, inst.ub, inst.var_kind, *inst.flat(), **kw)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


def _rule(every, relative=True, mu=10.0, tau=2.0, lo=10.0, hi=1000.0):
    from paper_2501_08293_amd import OPF_RHO_LAG
    gpu = dict(rho_every=every, rho_mode=0 if relative else 1, rho_mu=mu, rho_tau=tau, rho_min=lo, rho_max=hi)
    return gpu, (every, mu, tau, OPF_RHO_LAG, lo, hi, relative)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("name,every,relative", [("13bus", 1, True), ("13bus", 7, False), ("123bus", 1, True),
                                                 ("123bus", 10, True)])
@pytest.mark.parametrize("t", [3, 4, 5, 12, 60, 400])
def test_balanced_iterates_match_oracle_fp64(name, every, relative, t, kernel):
    _say(f"[gpu] balanced penalty {name} every={every} relative={relative} t={t} kernel={kernel} (FP64, run_fixed)")
    gpu, bal = _rule(every, relative)
    ref = admm.solve(_P(name), rho=RHO, eps_rel=1e-4, fixed_iters=t, balance=bal)
    s = _solver(_inst(name), rho=RHO, eps_rel=1e-4, kernel=kernel, block_waves=2, **gpu)
    out = s.solve(fixed_iters=t)
    s.close()
    assert out["iterations"] == t
    assert out["rho_final"] == ref.rho_final
    assert _rel(out["x"], ref.x) < 1e-9
    assert _rel(out["z"], ref.z) < 1e-9
    assert _rel(out["lam"], ref.lam) < 1e-9


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("name", ["13bus", "123bus"])
def test_balanced_solve_matches_oracle_fp64(name, kernel):
    _say(f"[gpu] balanced penalty solve {name} eps=1e-4 kernel={kernel} (FP64)")
    gpu, bal = _rule(10)
    ref = admm.solve(_P(name), rho=RHO, eps_rel=1e-4, balance=bal)
    assert ref.converged
    s = _solver(_inst(name), rho=RHO, eps_rel=1e-4, kernel=kernel, check_every=64, **gpu)
    out = s.solve()
    s.close()
    assert out["status"] == 0
    assert abs(out["iterations"] - ref.iterations) <= 1
    assert abs(out["objective"] - ref.objective) <= 1e-6 * abs(ref.objective)
    assert _rel(out["x"], ref.x) < 1e-6


def test_balanced_step_equals_persistent_bitwise():
    _say("[gpu] balanced penalty: step schedule = persistent schedule bit for bit (123bus, 700 iterations)")
    gpu, _ = _rule(1)
    outs = []
    for kernel in (STEP, PERSIST):
        s = _solver(_inst("123bus"), rho=RHO, eps_rel=1e-4, kernel=kernel, block_waves=4, **gpu)
        outs.append(s.solve(fixed_iters=700))
        s.close()
    a, b = outs
    assert a["rho_final"] == b["rho_final"]
    for k in ("x", "z", "lam"):
        assert np.array_equal(a[k], b[k]), k


def test_balanced_mixed_precision_matches_oracle():
    from paper_2501_08293_amd import OPF_PREC_MIXED
    _say("[gpu] balanced penalty, mixed precision 123bus eps=1e-4 vs the FP64 oracle")
    gpu, bal = _rule(10)
    ref = admm.solve(_P("123bus"), rho=RHO, eps_rel=1e-4, balance=bal)
    s = _solver(_inst("123bus"), rho=RHO, eps_rel=1e-4, precision=OPF_PREC_MIXED, **gpu)
    out = s.solve()
    s.close()
    assert out["status"] == 0
    assert abs(out["objective"] - ref.objective) <= 1e-4 * abs(ref.objective)
    vidx = np.nonzero(_inst("123bus").var_kind == 2)[0]
    assert np.max(np.abs(out["x"][vidx] - ref.x[vidx])) <= 1e-4

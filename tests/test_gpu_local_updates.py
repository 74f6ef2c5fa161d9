"""Several local updates per global update (Section III-D's second
acceleration) on the GPU: the kernels run one projection and a dual step of
k rho; the oracle repeats the local and dual updates k times literally with x
fixed.  The two agree to the FP64 bar (1e-9 relative at fixed t), which
checks the reduction on the product path."""
import sys

import numpy as np
import pytest

from opfgen import build_instance, by_name
from oracle import admm

pytestmark = pytest.mark.gpu
RHO = 100.0
_cache = {}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _inst(name):
    if name not in _cache:
        _cache[name] = build_instance(by_name(name, 0))
        _cache["P" + name] = admm.setup(_cache[name])
    return _cache[name], _cache["P" + name]


def _solver(inst, **kw):
    from paper_2501_08293_amd import Solver
    return Solver(inst.n, inst.c, inst.lb, inst.ub, inst.var_kind, *inst.flat(), **kw)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


@pytest.mark.parametrize("kernel", [1, 2], ids=["step", "persistent"])
@pytest.mark.parametrize("name", ["13bus", "123bus"])
@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("t", [1, 5, 40])
def test_local_updates_match_literal_oracle(name, k, t, kernel):
    _say(f"[gpu] {k} local updates per global update {name} t={t} kernel={kernel} (FP64)")
    inst, P = _inst(name)
    ref = admm.solve(P, rho=RHO, eps_rel=1e-4, fixed_iters=t, local_updates=k)
    s = _solver(inst, rho=RHO, eps_rel=1e-4, kernel=kernel, block_waves=2, local_updates=k)
    out = s.solve(fixed_iters=t)
    s.close()
    assert _rel(out["x"], ref.x) < 1e-9
    assert _rel(out["z"], ref.z) < 1e-9
    assert _rel(out["lam"], ref.lam) < 1e-9
    assert abs(out["dres"] - ref.dres) <= 1e-9 * max(ref.dres, 1e-300) + 1e-14


def test_local_updates_with_balanced_penalty_match_oracle():
    from paper_2501_08293_amd import OPF_RHO_LAG
    _say("[gpu] 2 local updates with residual balancing, 13bus t=60, persistent (FP64)")
    inst, P = _inst("13bus")
    ref = admm.solve(P, rho=RHO, eps_rel=1e-4, fixed_iters=60, local_updates=2,
                     balance=(1, 10.0, 2.0, OPF_RHO_LAG, 10.0, 1000.0))
    s = _solver(inst, rho=RHO, eps_rel=1e-4, kernel=2, local_updates=2, rho_every=1)
    out = s.solve(fixed_iters=60)
    s.close()
    assert out["rho_final"] == ref.rho_final
    assert _rel(out["x"], ref.x) < 1e-9 and _rel(out["lam"], ref.lam) < 1e-9

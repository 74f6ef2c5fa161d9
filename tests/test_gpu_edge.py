"""Edge-case shapes through the C ABI against the FP64 oracle: a component as
wide as a wavefront (64 slots), components without equations, a repeated
equation, a variable with ten copies (beyond the copies a slot keeps in
registers), infinite and one-sided bounds (random LP, `opfgen.random_lp`);
every schedule, two workgroup shapes, FP64 (1e-9) and mixed (1e-5) bars,
device set-up, and the serving runtime (same bits as the step schedule)."""
import sys
import time

import numpy as np
import pytest

from opfgen.random_lp import random_instance
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


@pytest.fixture(scope="module")
def lp():
    inst = random_instance(0)
    assert max(c.A.shape[1] for c in inst.comps) == 64
    assert min(c.A.shape[0] for c in inst.comps) == 0
    return inst, admm.setup(inst)


@pytest.mark.parametrize("kernel", [1, 2], ids=["step", "persistent"])
@pytest.mark.parametrize("bw", [1, 4])
def test_edge_shapes_match_oracle_fp64(lp, kernel, bw):
    from paper_2501_08293_amd import Solver
    inst, P = lp
    _say(f"[gpu] random LP edge shapes kernel={kernel} block_waves={bw}")
    s = Solver(*_args(inst), rho=RHO, eps_rel=1e-4, kernel=kernel, block_waves=bw)
    for t in (1, 7, 50):
        ref = admm.solve(P, rho=RHO, eps_rel=1e-4, fixed_iters=t, record=False)
        out = s.solve(fixed_iters=t)
        for key, r in (("x", ref.x), ("z", ref.z), ("lam", ref.lam)):
            assert _rel(out[key], r) <= 1e-9, (t, key)
    s.close()


def test_edge_shapes_mixed_and_device_setup(lp):
    from paper_2501_08293_amd import OPF_PREC_MIXED, Solver
    inst, P = lp
    _say("[gpu] random LP edge shapes: mixed precision, device set-up")
    ref = admm.solve(P, rho=RHO, eps_rel=1e-4, fixed_iters=50, record=False)
    s = Solver(*_args(inst), rho=RHO, eps_rel=1e-4, precision=OPF_PREC_MIXED)
    out = s.solve(fixed_iters=50)
    s.close()
    assert _rel(out["x"], ref.x) <= 1e-5
    s = Solver(*_args(inst), rho=RHO, eps_rel=1e-4, setup_on_device=True)
    out = s.solve(fixed_iters=50)
    s.close()
    assert _rel(out["x"], ref.x) <= 1e-9 and _rel(out["lam"], ref.lam) <= 1e-9


def test_edge_shapes_served_like_step_schedule(lp):
    from paper_2501_08293_amd import Server, Solver
    inst, _ = lp
    _say("[gpu] random LP edge shapes: served alone vs step schedule")
    srv = Server(rho=RHO, eps_rel=1e-4, warm_start=False, iters_per_poll=64, arena_bytes=64 << 20,
                 max_iter=3000)
    rid = srv.submit(*_args(inst))
    t0 = time.time()
    res = None
    while res is None:
        for r in srv.poll(max_out=4, wait_ms=50):
            res = r
        assert time.time() - t0 < 120
    srv.close()
    s = Solver(*_args(inst), rho=RHO, eps_rel=1e-4, kernel=1, block_waves=4, max_iter=3000)
    one = s.solve(raise_on_error=False)
    s.close()
    assert res["iterations"] == one["iterations"]
    assert np.array_equal(res["x"], one["x"])

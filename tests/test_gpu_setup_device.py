"""Device-side set-up (row reduction and projection factors on the GPU).

Checks, through the C ABI: with the factors computed by the device set-up, the
iterates at fixed t match the FP64 oracle to the same 1e-9 relative bar as the
host set-up (the factors agree to rounding), and match the host-set-up solver
to 1e-12; a solve to tolerance stops within one iteration of the host-set-up
solve; the mixed-precision path uses the narrowed device factors; a component
with contradictory equations is rejected with OPF_EINFEASIBLE_COMPONENT by the
device as by the host."""
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


@pytest.mark.parametrize("name", ["13bus", "13bus-zip", "123bus", "2500bus"])
def test_device_factors_match_oracle_and_host_setup(name):
    from paper_2501_08293_amd import Solver
    _say(f"[gpu] device set-up vs host set-up vs oracle, {name}, t=50")
    inst = build_instance(by_name(name, 0))
    t = 50
    dev = Solver(*_args(inst), rho=RHO, eps_rel=1e-4, setup_on_device=True, kernel=2)
    host = Solver(*_args(inst), rho=RHO, eps_rel=1e-4, setup_on_device=False, kernel=2)
    a = dev.solve(fixed_iters=t)
    b = host.solve(fixed_iters=t)
    _say(f"  set-up ms: device factors {dev.info().setup_ms:.1f}, host factors {host.info().setup_ms:.1f}")
    dev.close()
    host.close()
    ref = admm.solve(admm.setup(inst), rho=RHO, eps_rel=1e-4, fixed_iters=t, record=False)
    for key, r in (("x", ref.x), ("z", ref.z), ("lam", ref.lam)):
        assert _rel(a[key], r) <= 1e-9, key
        assert _rel(a[key], b[key]) <= 1e-12, key


def test_device_setup_solve_to_tolerance_and_mixed():
    from paper_2501_08293_amd import OPF_PREC_MIXED, Solver
    _say("[gpu] device set-up: 123bus to 1e-4, FP64 and mixed")
    inst = build_instance(by_name("123bus", 0))
    outs = []
    for dev in (True, False):
        s = Solver(*_args(inst), rho=RHO, eps_rel=1e-4, setup_on_device=dev)
        outs.append(s.solve())
        s.close()
    assert outs[0]["status"] == 0
    assert abs(outs[0]["iterations"] - outs[1]["iterations"]) <= 1
    assert abs(outs[0]["objective"] - outs[1]["objective"]) <= 1e-9 * abs(outs[1]["objective"])
    s = Solver(*_args(inst), rho=RHO, eps_rel=1e-4, setup_on_device=True, precision=OPF_PREC_MIXED)
    m = s.solve()
    s.close()
    assert m["status"] == 0 and m["iterations_fp32"] > 0
    assert abs(m["objective"] - outs[1]["objective"]) <= 1e-4 * abs(outs[1]["objective"])


def _two_component_problem(b_second):
    """x0 + x1 = 1 (component 0); x0 + x1 = 1 and 2 x0 + 2 x1 = b (component 1).
    b = 2 is consistent (a redundant row), b = 3 contradicts the first row."""
    n = 2
    c = np.array([1.0, 0.0])
    lb = np.array([0.0, 0.0])
    ub = np.array([1.0, 1.0])
    kind = np.zeros(n, np.uint8)
    comp_m = np.array([1, 2], np.int32)
    comp_n = np.array([2, 2], np.int32)
    A = np.array([1.0, 1.0, 1.0, 1.0, 2.0, 2.0])
    b = np.array([1.0, 1.0, b_second])
    idx = np.array([0, 1, 0, 1], np.int32)
    return n, c, lb, ub, kind, comp_m, comp_n, A, b, idx


@pytest.mark.parametrize("dev", [True, False], ids=["device", "host"])
def test_contradictory_component_rejected(dev):
    from paper_2501_08293_amd import OpfError, Solver
    _say(f"[gpu] contradictory component, set-up on device={dev}")
    with pytest.raises(OpfError) as e:
        Solver(*_two_component_problem(3.0), rho=RHO, eps_rel=1e-4, setup_on_device=dev)
    assert e.value.code == -4
    s = Solver(*_two_component_problem(2.0), rho=RHO, eps_rel=1e-6, setup_on_device=dev)
    out = s.solve()
    s.close()
    assert out["status"] == 0
    assert abs(out["x"][0] + out["x"][1] - 1.0) <= 1e-5
    assert abs(out["objective"]) <= 1e-5          # min x0 s.t. x0 + x1 = 1, 0 <= x <= 1

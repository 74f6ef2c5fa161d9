"""The allocation-free solve (opf_admm_solve_noalloc, kernel scratch in the
library's static device array) returns what opf_admm_solve returns, bit for
bit, on consecutive calls that share the array, the second with a smaller
problem; problems whose scratch exceeds the array are rejected."""
import sys

import numpy as np
import pytest

from opfgen import build_instance, by_name

pytestmark = pytest.mark.gpu
RHO = 100.0


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _solver(inst, **kw):
    from paper_2501_08293_amd import Solver
    return Solver(inst.n, inst.c, inst.lb, inst.ub, inst.var_kind, *inst.flat(), rho=RHO, **kw)


def _same(a, b):
    assert a["status"] == b["status"]
    assert a["iterations"] == b["iterations"] and a["iterations_fp32"] == b["iterations_fp32"]
    assert a["objective"] == b["objective"]
    for k in ("x", "z", "lam"):
        assert np.array_equal(a[k], b[k]), k
    for k in ("pres", "dres", "eps_prim", "eps_dual"):
        assert a[k] == b[k], k


@pytest.mark.parametrize("kernel,precision,bw", [(2, 0, 0), (2, 1, 0), (1, 0, 0), (3, 1, 1), (3, 0, 1)],
                         ids=["persistent-fp64", "persistent-mixed", "step-fp64", "tiled-mixed", "tiled-fp64"])
def test_noalloc_equals_solve_on_two_calls_second_smaller(kernel, precision, bw):
    for name in ("123bus", "13bus"):
        _say(f"[gpu] allocation-free solve {name} kernel={kernel} precision={precision} block_waves={bw}")
        inst = build_instance(by_name(name, 0))
        s = _solver(inst, eps_rel=1e-4, kernel=kernel, precision=precision, check_every=128, block_waves=bw)
        ref = s.solve()
        got = s.solve(noalloc=True)
        s.close()
        assert ref["status"] == 0
        _same(got, ref)


def test_noalloc_rejects_scratch_beyond_the_array():
    from paper_2501_08293_amd import Solver, binding
    _say("[gpu] allocation-free solve: a problem whose scratch exceeds the static array is rejected")
    n = 600_000                       # one single-slot component per variable: 600k packed lanes
    s = Solver(n, np.zeros(n), -np.ones(n), np.ones(n), np.ones(n, np.uint8), np.zeros(n, np.int32),
               np.ones(n, np.int32), np.zeros(0), np.zeros(0), np.arange(n, dtype=np.int32), rho=RHO,
               eps_rel=1e-3, kernel=1)
    with pytest.raises(binding.OpfError) as e:
        s.solve(noalloc=True)
    s.close()
    assert e.value.code == binding.OPF_EINVAL
    assert "static array" in str(e.value)

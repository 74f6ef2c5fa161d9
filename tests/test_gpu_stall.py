"""The stall watch of the FP64 iterations (opf_admm_options.stall_window).

On an infeasible LP (a random feasible one plus two one-slot components fixing
variable 0 to +0.5 and -0.5) the solve stops with OPF_STALLED after the
merit pres^2 + (dres / rho)^2 has fallen by less than stall_delta over
stall_checks windows, with the oracle's iterate at the same iteration
(FP64, 1e-9) and the merit on its closed-form floor 0.5; without the watch it
runs to max_iter.  On a feasible problem the watch changes nothing: the same
stop iteration and the same bits."""
import sys

import numpy as np
import pytest

from opfgen import build_instance, by_name
from opfgen.random_lp import inconsistent_instance
from oracle import admm

pytestmark = pytest.mark.gpu
RHO = 100.0


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _solver(inst, **kw):
    from paper_2501_08293_amd import Solver
    return Solver(inst.n, inst.c, inst.lb, inst.ub, inst.var_kind, *inst.flat(), rho=RHO, **kw)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


@pytest.mark.parametrize("kernel", [1, 2])
def test_infeasible_lp_stops_with_stalled(kernel):
    from paper_2501_08293_amd.binding import OPF_NOT_CONVERGED, OPF_STALLED
    inst = inconsistent_instance(0, 120)
    _say(f"[gpu] stall watch: inconsistent LP, kernel={kernel}, window 256")
    s = _solver(inst, eps_rel=1e-4, kernel=kernel, max_iter=200_000, stall_window=256, check_every=128)
    out = s.solve(raise_on_error=False)
    s.close()
    assert out["status"] == OPF_STALLED
    t = int(out["iterations"])
    assert t % 256 == 0 and 3 * 256 <= t <= 20_000
    merit = out["pres"] ** 2 + (out["dres"] / RHO) ** 2
    assert 0.5 <= merit < 0.501
    ref = admm.solve(admm.setup(inst), rho=RHO, eps_rel=1e-4, fixed_iters=t, record=False)
    assert _rel(out["x"], ref.x) < 1e-9
    assert _rel(out["z"], ref.z) < 1e-9
    _say(f"  stalled at {t} iterations, merit {merit:.6f}")
    s = _solver(inst, eps_rel=1e-4, kernel=kernel, max_iter=3000, check_every=128)
    out = s.solve(raise_on_error=False)
    s.close()
    assert out["status"] == OPF_NOT_CONVERGED and out["iterations"] == 3000


def test_mixed_precision_polish_stalls():
    from paper_2501_08293_amd import OPF_PREC_MIXED
    from paper_2501_08293_amd.binding import OPF_STALLED
    inst = inconsistent_instance(1, 120)
    _say("[gpu] stall watch: inconsistent LP, mixed precision (bulk to max_iter, then the FP64 polish stalls)")
    s = _solver(inst, eps_rel=1e-4, precision=OPF_PREC_MIXED, max_iter=2000, stall_window=256)
    out = s.solve(raise_on_error=False)
    s.close()
    assert out["status"] == OPF_STALLED
    assert out["iterations_fp32"] == 2000 and out["iterations"] > 2000


@pytest.mark.parametrize("precision", [0, 1])
def test_feasible_solve_is_unchanged_by_the_watch(precision):
    inst = build_instance(by_name("123bus", 0))
    _say(f"[gpu] stall watch on a feasible solve: 123bus precision={precision}")
    outs = []
    for win in (0, 1024):
        s = _solver(inst, eps_rel=1e-4, precision=precision, stall_window=win)
        outs.append(s.solve())
        s.close()
    a, b = outs
    assert a["status"] == 0 and b["status"] == 0
    assert a["iterations"] == b["iterations"]
    for f in ("x", "z", "lam"):
        assert np.array_equal(a[f], b[f]), f

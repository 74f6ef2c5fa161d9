"""The plateau the stall watch looks for, on the oracle (CPU).

On an infeasible componentwise LP (every component's equations solvable,
their consensus not) the merit pres^2 + (dres / rho)^2 of the termination
test's residuals (Section III-C) still never increases, but it cannot fall
below the squared distance the consensus leaves between inconsistent copies:
two one-slot components that fix variable 0 to +0.5 and -0.5 keep
pres^2 >= min_x (x - 0.5)^2 + (x + 0.5)^2 = 0.5.  On the feasible LP without
them the merit keeps falling."""
import numpy as np

from opfgen.random_lp import inconsistent_instance, random_instance
from oracle import admm

RHO = 100.0


def _merit(inst, t):
    r = admm.solve(admm.setup(inst), rho=RHO, eps_rel=1e-4, fixed_iters=t, record=True)
    h = r.history
    return h[:, 0] ** 2 + (h[:, 1] / RHO) ** 2


def test_infeasible_lp_merit_settles_on_its_lower_bound():
    m = _merit(inconsistent_instance(0, 120), 3000)
    assert np.all(np.diff(m) <= 1e-9 * m[:-1])          # non-increasing
    assert m[-1] >= 0.5                                  # the closed-form floor
    assert m[-1] - 0.5 < 1e-3                            # and it gets there
    assert (m[-1001] - m[-1]) / m[-1] < 1e-4             # a plateau: <0.01 % over the last 1000 iterations


def test_feasible_lp_merit_keeps_falling():
    m = _merit(random_instance(0, 120), 3000)
    assert np.all(np.diff(m) <= 1e-9 * m[:-1])
    assert (m[-1001] - m[-1]) / m[-1] > 0.01             # still > 1 % per 1000 iterations

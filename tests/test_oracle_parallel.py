"""The oracle's multi-process mode (components split over worker processes,
as in the paper's CPU runs) performs the same arithmetic as the
single-process oracle: equal iterates at fixed t and the same stop."""
import numpy as np
import pytest

from opfgen import build_instance, by_name
from oracle import admm
from oracle.parallel import solve_parallel, split_components


@pytest.mark.parametrize("name,procs", [("13bus", 2), ("123bus", 3)])
def test_parallel_oracle_equals_serial(name, procs):
    P = admm.setup(build_instance(by_name(name, 0)))
    ref = admm.solve(P, rho=100.0, eps_rel=1e-3, fixed_iters=40)
    x, z, lam, t, conv, r = solve_parallel(P, procs, rho=100.0, eps_rel=1e-3, fixed_iters=40)
    assert t == 40
    assert np.array_equal(x, ref.x) and np.array_equal(z, ref.z) and np.array_equal(lam, ref.lam)
    assert r == (ref.pres, ref.dres, ref.eps_prim, ref.eps_dual)


def test_parallel_oracle_stops_where_serial_does():
    P = admm.setup(build_instance(by_name("13bus", 0)))
    ref = admm.solve(P, rho=100.0, eps_rel=1e-3)
    x, z, lam, t, conv, r = solve_parallel(P, 2, rho=100.0, eps_rel=1e-3)
    assert conv and t == ref.iterations
    assert np.array_equal(x, ref.x)


def test_split_is_contiguous_and_balanced():
    P = admm.setup(build_instance(by_name("123bus", 0)))
    parts = split_components(P, 4)
    assert parts[0][0] == 0 and parts[-1][1] == len(P.idx)
    assert all(a[1] == b[0] for a, b in zip(parts, parts[1:]))
    w = [sum(len(P.idx[s]) ** 2 for s in range(lo, hi)) for lo, hi in parts]
    assert max(w) <= 1.5 * (sum(w) / 4) + max(len(i) ** 2 for i in P.idx)

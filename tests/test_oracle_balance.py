"""Pins of the oracle's residual-balancing schedule (the acceleration Section
III-D points to, Wohlberg's rule), on the CPU.

The schedule is pinned by what must hold for any correct implementation, not
by re-running its own code:
  * a schedule that changes the penalty once equals two plain runs joined by
    a warm start (the duals are unscaled, so nothing is carried over but
    (z, lambda)), which fixes the lag, the penalty each update uses and the
    dual residual's penalty;
  * a rule that can never fire equals the fixed-penalty run bit for bit;
  * the relative form is homogeneous: scaling c, rho and the bounds on rho by
    a power of two scales lambda and every penalty exactly and leaves x and z
    unchanged (the plain form is not, which the same test shows);
  * every recorded change is a factor tau or 1/tau in the direction the rule
    defines, and the penalty stays in its bounds."""
import dataclasses
import math

import numpy as np
import pytest

from opfgen import build_instance, make_13bus
from oracle import admm

RHO = 100.0


@pytest.fixture(scope="module")
def P13():
    return admm.setup(build_instance(make_13bus(0)))


@pytest.mark.parametrize("lag", [1, 4])
def test_one_change_equals_a_restart(P13, lag):
    every, rho2, T = 10, 50.0, 60
    # bounds pinned at rho2: the first decision (after iteration `every`)
    # moves the penalty there whatever the residuals say
    r = admm.solve(P13, rho=RHO, eps_rel=1e-3, fixed_iters=T, balance=(every, 10.0, 2.0, lag, rho2, rho2))
    k = every + lag - 1                # iterations run with the start penalty
    a = admm.solve(P13, rho=RHO, eps_rel=1e-3, fixed_iters=k)
    b = admm.solve(P13, rho=rho2, eps_rel=1e-3, fixed_iters=T - k, z0=a.z, lam0=a.lam)
    assert np.array_equal(r.x, b.x)
    assert np.array_equal(r.z, b.z)
    assert np.array_equal(r.lam, b.lam)
    assert np.array_equal(r.rho_history, np.array([RHO] * k + [rho2] * (T - k)))
    assert np.array_equal(r.history[:k], a.history)
    assert np.array_equal(r.history[k:], b.history)


def test_rule_that_never_fires_equals_fixed_penalty(P13):
    r = admm.solve(P13, rho=RHO, eps_rel=1e-3, fixed_iters=200, balance=(1, math.inf, 2.0, 4, 1.0, 1e4))
    f = admm.solve(P13, rho=RHO, eps_rel=1e-3, fixed_iters=200)
    assert np.array_equal(r.x, f.x) and np.array_equal(r.lam, f.lam)
    assert np.all(r.rho_history == RHO)


def _scaled(P, kappa):
    return dataclasses.replace(P, c=P.c * kappa)


@pytest.mark.parametrize("relative", [True, False])
def test_relative_rule_is_homogeneous_in_cost_and_penalty(P13, relative):
    kappa = 2.0 ** -10        # exact in binary floating point
    bal = (5, 10.0, 2.0, 4, 10.0, 1000.0, relative)
    balk = (5, 10.0, 2.0, 4, 10.0 * kappa, 1000.0 * kappa, relative)
    r = admm.solve(P13, rho=RHO, eps_rel=1e-3, fixed_iters=300, balance=bal)
    s = admm.solve(_scaled(P13, kappa), rho=RHO * kappa, eps_rel=1e-3, fixed_iters=300, balance=balk)
    assert len(set(r.rho_history.tolist())) > 1, "the schedule must change for the test to mean anything"
    same = (np.array_equal(s.rho_history, kappa * r.rho_history) and np.array_equal(s.x, r.x)
            and np.array_equal(s.z, r.z) and np.array_equal(s.lam, kappa * r.lam))
    # pres and the tolerances are invariant or scale with kappa together; the
    # plain form compares pres with dres, which scales with kappa alone
    assert same == relative


@pytest.mark.parametrize("relative", [True, False])
def test_changes_follow_the_rule_and_bounds(P13, relative):
    every, mu, tau, lag, lo, hi = 3, 5.0, 2.0, 4, 12.5, 800.0
    r = admm.solve(P13, rho=RHO, eps_rel=1e-3, fixed_iters=400, balance=(every, mu, tau, lag, lo, hi, relative))
    rh = r.rho_history
    H = r.history
    assert np.all((rh >= lo) & (rh <= hi))
    moved = 0
    for u in range(every, len(rh) - lag + 1, every):
        pres, dres, ep, ed = H[u - 1]
        a, b = (pres / ep, dres / ed) if relative else (pres, dres)
        prev, new = rh[u + lag - 2], rh[u + lag - 1]
        if a > mu * b:
            want = min(prev * tau, hi)
        elif b > mu * a:
            want = max(prev / tau, lo)
        else:
            want = prev
        assert new == want, (u, prev, new, want)
        moved += new != prev
        # between decisions the penalty does not move
        for t in range(u + lag, min(u + lag + every - 1, len(rh))):
            assert rh[t] == new
    assert moved > 0


# ---- planted mistakes in the rule (CPU only): each must make a pin above fail

def _mut_direction_swapped(pres, dres, eps_prim, eps_dual, mu, tau, relative=True):
    rp, rd = (pres / eps_prim, dres / eps_dual) if relative else (pres, dres)
    if rp > mu * rd:
        return 1.0 / tau
    if rd > mu * rp:
        return tau
    return 1.0


def _mut_one_tolerance(pres, dres, eps_prim, eps_dual, mu, tau, relative=True):
    # both residuals divided by the primal tolerance
    rp, rd = (pres / eps_prim, dres / eps_prim) if relative else (pres, dres)
    if rp > mu * rd:
        return tau
    if rd > mu * rp:
        return 1.0 / tau
    return 1.0


@pytest.mark.parametrize("mut,pin", [(_mut_direction_swapped, "rule"), (_mut_one_tolerance, "homogeneous")])
def test_planted_rule_mistake_is_caught(P13, monkeypatch, mut, pin):
    monkeypatch.setattr(admm, "balance_factor", mut)
    with pytest.raises(AssertionError):
        if pin == "rule":
            test_changes_follow_the_rule_and_bounds(P13, True)
        else:
            test_relative_rule_is_homogeneous_in_cost_and_penalty(P13, True)

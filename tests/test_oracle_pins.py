"""Pins of the FP64 oracle (Algorithm 1) against what the paper and the
mathematics fix: library routines, brute force, closed forms, invariants and
an independently assembled centralised LP solved by HiGHS.  CPU only."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

from opfgen import build_instance, by_name, make_13bus
from oracle import admm
from oracle.central import CentralLP
from pin_helpers import _trajectory, termination_is_homogeneous, termination_matches_literal

RHO = 100.0


@pytest.fixture(scope="module")
def P13(inst13):
    return admm.setup(inst13)


@pytest.fixture(scope="module")
def P13zip(inst13zip):
    return admm.setup(inst13zip)


# --------------------------------------------------------------------------
# precomputation (closed_2) and row reduction
# --------------------------------------------------------------------------

def test_factors_are_the_pinv_projector(P13, P13zip):
    """Abar_s = -(I - pinv(A_s) A_s), bbar_s = pinv(A_s) b_s; I - P is a
    symmetric idempotent with eigenvalues in {0, 1}; A_s bbar_s = b_s."""
    for P in (P13, P13zip):
        for A, b, Ab, bb in zip(P.A, P.b, P.Abar, P.bbar):
            n = A.shape[1]
            F = -Ab
            pinv = np.linalg.pinv(A)
            np.testing.assert_allclose(F, np.eye(n) - pinv @ A, atol=1e-12)
            np.testing.assert_allclose(bb, pinv @ b, atol=1e-12)
            np.testing.assert_allclose(F, F.T, atol=1e-12)
            np.testing.assert_allclose(F @ F, F, atol=1e-12)
            ev = np.linalg.eigvalsh(0.5 * (F + F.T))
            assert np.all(np.minimum(np.abs(ev), np.abs(ev - 1)) < 1e-10)
            np.testing.assert_allclose(A @ bb, b, atol=1e-12)


def test_rref_drops_redundant_rows_and_flags_contradictions():
    rng = np.random.default_rng(0)
    A = rng.normal(size=(4, 9))
    b = rng.normal(size=4)
    A2 = np.vstack([A, A[1] + 2 * A[3]])
    b2 = np.concatenate([b, [b[1] + 2 * b[3]]])
    R, rb, piv = admm.rref(A2, b2)
    assert R.shape == (4, 9) and len(piv) == 4
    Ab1, bb1 = admm.local_factors(A, b)
    Ab2, bb2 = admm.local_factors(A2, b2)
    np.testing.assert_allclose(Ab1, Ab2, atol=1e-12)
    np.testing.assert_allclose(bb1, bb2, atol=1e-12)
    # reduced rows have unit pivots and zeros elsewhere in the pivot columns
    np.testing.assert_allclose(R[:, piv], np.eye(4), atol=1e-12)
    b3 = b2.copy()
    b3[-1] += 1.0
    with pytest.raises(admm.InfeasibleComponent):
        admm.rref(A2, b3)


# --------------------------------------------------------------------------
# one iteration: each update against brute force
# --------------------------------------------------------------------------

def _some_state(P, seed=0):
    rng = np.random.default_rng(seed)
    z = rng.normal(size=P.L)
    lam = rng.normal(size=P.L)
    return z, lam


def test_global_update_is_the_bounded_scalar_minimiser(P13):
    """Each x_i minimises (c + sum_s B_s^T lambda_s)_i x_i
    + rho/2 sum_s sum_j (x_i - (x_s)_j)^2 over [lb_i, ub_i] (Section III-B)."""
    z, lam = _some_state(P13, 1)
    x = admm.global_update(P13, z, lam, RHO)
    for i in range(P13.n):
        slots = np.nonzero(P13.gidx == i)[0]
        g = P13.c[i] + lam[slots].sum()

        def obj(v, g=g, slots=slots):
            return g * v + 0.5 * RHO * np.sum((v - z[slots]) ** 2)
        lo = P13.lb[i] if np.isfinite(P13.lb[i]) else -1e3
        hi = P13.ub[i] if np.isfinite(P13.ub[i]) else 1e3
        if lo == hi:
            assert x[i] == lo
            continue
        res = minimize_scalar(obj, bounds=(lo, hi), method="bounded", options=dict(xatol=1e-12))
        assert abs(res.x - x[i]) < 1e-7, (i, res.x, x[i])


def test_local_update_solves_the_kkt_system(P13zip):
    """x_s minimises -<lambda_s, x_s> + rho/2 ||B_s x - x_s||^2 s.t. A_s x_s = b_s:
    the KKT system [[rho I, A^T], [A, 0]] [x_s; mu] = [rho B_s x + lambda_s; b_s]."""
    P = P13zip
    z, lam = _some_state(P, 2)
    x = admm.global_update(P, z, lam, RHO)
    zs = admm.local_update(P, x, lam, RHO)
    for s, (A, b) in enumerate(zip(P.A, P.b)):
        Ah, bh, _ = admm.rref(A, b)
        m, n = Ah.shape
        K = np.block([[RHO * np.eye(n), Ah.T], [Ah, np.zeros((m, m))]])
        o = P.offs[s]
        rhs = np.concatenate([RHO * x[P.idx[s]] + lam[o:o + n], bh])
        sol = np.linalg.solve(K, rhs)
        np.testing.assert_allclose(zs[o:o + n], sol[:n], rtol=1e-10, atol=1e-10)


def test_grouped_local_update_equals_per_component_loop(P13zip):
    z, lam = _some_state(P13zip, 3)
    x = admm.global_update(P13zip, z, lam, RHO)
    np.testing.assert_allclose(admm.local_update(P13zip, x, lam, RHO),
                               admm.local_update_loop(P13zip, x, lam, RHO), rtol=1e-13, atol=1e-13)


def test_initial_point_rule(P13):
    z, lam = admm.initial_point(P13)
    assert np.all(lam == 0)
    for j, i in enumerate(P13.gidx):
        if P13.var_kind[i] == 2:
            assert z[j] == 1.0
        elif np.isfinite(P13.lb[i]) and np.isfinite(P13.ub[i]):
            assert z[j] == 0.5 * (P13.lb[i] + P13.ub[i])
        else:
            assert z[j] == 0.0


# --------------------------------------------------------------------------
# invariants along the trajectory
# --------------------------------------------------------------------------

def test_equality_blocks_hold_after_every_local_update(P13zip):
    """P1: ||A_s x_s - b_s||_inf <= 1e-12 max(1, ||b_s||_inf), original A_s."""
    for x, z, _, lam in _trajectory(P13zip, 50):
        for s, (A, b) in enumerate(zip(P13zip.A, P13zip.b)):
            o = P13zip.offs[s]
            zs = z[o:o + A.shape[1]]
            assert np.max(np.abs(A @ zs - b)) <= 1e-12 * max(1.0, np.max(np.abs(b))) * 10


def test_duals_stay_in_row_space_and_x_in_box(P13zip):
    """P5: lambda_s in range(A_s^T), i.e. (I - P_s) lambda_s = 0, for t >= 1;
    x stays in [lb, ub] exactly."""
    P = P13zip
    for x, z, _, lam in _trajectory(P, 30):
        assert np.all(x >= P.lb) and np.all(x <= P.ub)
        for s in range(len(P.idx)):
            o = P.offs[s]
            k = len(P.idx[s])
            F = -P.Abar[s]
            assert np.max(np.abs(F @ lam[o:o + k])) <= 1e-9 * max(1.0, np.max(np.abs(lam[o:o + k])))


@pytest.mark.parametrize("name", ["13bus", "13bus-zip", "123bus"])
def test_merit_is_monotone(name):
    """P6: rho ||z^t - z^{t-1}||^2 + ||lambda^t - lambda^{t-1}||^2 / rho, i.e.
    rho (pres^2 + (dres/rho)^2), never increases from t = 2 on (two-block
    ADMM contraction)."""
    P = admm.setup(build_instance(by_name(name, 0)))
    r = admm.solve(P, rho=RHO, eps_rel=1e-4, fixed_iters=3000)
    m = r.history[:, 0] ** 2 + (r.history[:, 1] / RHO) ** 2
    d = np.diff(m[1:])
    assert np.all(d <= 1e-10 * m[1:-1])


# --------------------------------------------------------------------------
# end to end against closed forms and a brute-force LP solve
# --------------------------------------------------------------------------

def _sweep(f):
    """Closed-form solution of the lossless linearised model for constant-power
    wye loads with the substation as the only source: backward sweep of the
    per-phase loads, then a forward sweep w_child = w_parent + Mp p + Mq q with
    Mp = -2Re(Gamma o conj Z), Mq = 2Im(Gamma o conj Z)."""
    from oracle.central import mp_mq_complex
    n = f.n_bus
    P = np.zeros((n, 3))
    Q = np.zeros((n, 3))
    for ld in f.loads:
        P[ld.bus] += ld.a
        Q[ld.bus] += ld.b
    children = [[] for _ in range(n)]
    pl = {}
    for ln in f.lines:
        children[ln.parent].append(ln)
    order = []
    stack = [0]
    while stack:
        u = stack.pop()
        order.append(u)
        for ln in children[u]:
            stack.append(ln.child)
    for u in reversed(order):
        for ln in children[u]:
            P[u] += P[ln.child]
            Q[u] += Q[ln.child]
    w = np.ones((n, 3))
    for u in order:
        for ln in children[u]:
            mp, mq = mp_mq_complex(ln.r, ln.x)
            ph = list(ln.phases)
            w[ln.child, ph] = w[u, ph] + mp[np.ix_(ph, ph)] @ P[ln.child, ph] + mq[np.ix_(ph, ph)] @ Q[ln.child, ph]
    return w, sum(ld.a.sum() for ld in f.loads)


def test_converged_admm_matches_closed_form_sweep():
    """P8: 13-bus, constant power, no DERs: the optimum is the sweep solution
    and the objective is the total real load."""
    f = make_13bus(0)
    inst = build_instance(f)
    P = admm.setup(inst)
    r = admm.solve(P, rho=RHO, eps_rel=1e-9)
    assert r.converged
    w, total = _sweep(f)
    assert abs(r.objective - total) <= 1e-6 * total
    for k, key in enumerate(inst.var_keys):
        if key[0] == "w":
            assert abs(r.x[k] - w[key[1], key[2]]) < 1e-6


@pytest.mark.parametrize("name,eps", [("13bus", 1e-9), ("13bus-zip", 1e-9), ("123bus", 1e-8)])
def test_converged_admm_matches_highs_on_central_lp(name, eps):
    """P12: the oracle run to a tight tolerance reaches the optimum of the
    centralised LP (assembled independently from the feeder) found by HiGHS:
    objective within 1e-6 relative; w within 1e-6 where the optimum is unique."""
    f = by_name(name, 0)
    inst = build_instance(f)
    P = admm.setup(inst)
    r = admm.solve(P, rho=RHO, eps_rel=eps)
    assert r.converged
    lp = CentralLP(f)
    res = lp.solve()
    assert abs(r.objective - res.fun) <= 1e-6 * max(1.0, abs(res.fun))
    # w is unique at this optimum: check a few with the optimal-face range
    wkeys = [k for k in inst.var_keys if k[0] == "w"]
    for key in wkeys[:: max(1, len(wkeys) // 6)]:
        lo, hi = lp.value_range(key, res.fun)
        if hi - lo < 1e-7:
            assert abs(r.x[inst.var_keys.index(key)] - 0.5 * (lo + hi)) < 1e-6


def test_kkt_certificate_at_termination():
    """P7: with g = c + B^T lambda: g_i = 0 where lb < x < ub, g_i >= 0 at lb,
    g_i <= 0 at ub (to tolerance); A_s x[idx_s] = b_s nearly."""
    f = by_name("13bus-zip", 0)
    inst = build_instance(f)
    P = admm.setup(inst)
    r = admm.solve(P, rho=RHO, eps_rel=1e-9)
    g = P.c + admm.B_T(P, r.lam)
    tol = 1e-5
    free = (r.x > P.lb + 1e-9) & (r.x < P.ub - 1e-9)
    fixed = P.lb == P.ub            # e.g. the substation voltage: any sign
    assert np.max(np.abs(g[free])) < tol
    assert np.all(g[(r.x <= P.lb + 1e-9) & ~free & ~fixed] >= -tol)
    assert np.all(g[(r.x >= P.ub - 1e-9) & ~free & ~fixed] <= tol)
    for s, (A, b) in enumerate(zip(P.A, P.b)):
        assert np.max(np.abs(A @ r.x[P.idx[s]] - b)) < 1e-6


def test_termination_test_literal_reading():
    """The stop rule uses the stacked norms; stopping at t means the test
    failed at every earlier t."""
    P = admm.setup(build_instance(make_13bus(0)))
    r = admm.solve(P, rho=RHO, eps_rel=1e-3)
    h = r.history
    ok = (h[:, 0] <= h[:, 2]) & (h[:, 1] <= h[:, 3])
    assert ok[-1] and not ok[:-1].any()
    assert r.iterations == len(h)


def test_termination_quantities_equal_the_printed_sums():
    """Section III-C's pres, dres, eps_prim and eps_dual, evaluated literally with
    dense B_s per component (B_s^T maps a component's vector into R^n), equal the
    oracle's norms of the stacked slot vectors, at every one of the first
    iterations on the 13-bus feeder and the edge-case random LP (a ten-copy
    variable, equation-free components, infinite bounds)."""
    from opfgen.random_lp import random_instance
    for inst in (build_instance(make_13bus(0)), random_instance(0, n=160)):
        assert termination_matches_literal(admm.setup(inst))


@pytest.mark.parametrize("which", ["13bus", "random"])
def test_termination_is_scale_invariant(which):
    """Homogeneity: the residual history of the LP scaled by 8 is 8 times the
    original one, and the stop iteration is the same (an absolute tolerance, a
    squared or unsquared norm in the wrong place would break it)."""
    from opfgen.random_lp import random_instance
    inst = build_instance(make_13bus(0)) if which == "13bus" else random_instance(0, n=160)
    assert termination_is_homogeneous(inst)


def test_multiple_local_updates_collapse_to_a_scaled_dual_step():
    """Several local updates per global update (Section III-D's second
    acceleration): with x fixed, the closed-form local update followed by the
    dual update, repeated k times, returns the same local copies as the first
    update and the duals of one dual step of length k rho.  The reason: after a
    dual update lambda_s lies in range(A_s^T), so (I - P_s) lambda_s = 0 and the
    projection of x + lambda_s / rho equals that of x."""
    P = admm.setup(build_instance(make_13bus(0)))
    traj = _trajectory(P, 5)
    x, z1, _, lam_prev = traj[-1]
    lam0 = traj[-2][3]                    # lambda of iteration t-1: in range(A^T) already
    for k in (2, 3, 5):
        z = admm.local_update(P, x, lam0, RHO)
        lam = admm.dual_update(P, x, z, lam0, RHO)
        for _ in range(k - 1):
            zk = admm.local_update(P, x, lam, RHO)
            np.testing.assert_allclose(zk, z, rtol=0, atol=1e-12 * max(1.0, np.max(np.abs(z))))
            lam = admm.dual_update(P, x, zk, lam, RHO)
        np.testing.assert_allclose(lam, lam0 + k * RHO * (x[P.gidx] - z), rtol=0,
                                   atol=1e-9 * max(1.0, np.max(np.abs(lam))))


# --------------------------------------------------------------------------
# the same invariants on the edge-case shapes of the random LP (64-slot and
# equation-free components, a repeated row, a ten-copy variable, infinite bounds)
# --------------------------------------------------------------------------

def test_invariants_hold_on_edge_case_shapes():
    from opfgen.random_lp import random_instance
    P = admm.setup(random_instance(0))
    for A, b, Ab, bb in zip(P.A, P.b, P.Abar, P.bbar):
        n = A.shape[1]
        if A.shape[0] == 0:                 # no equations: the projection is the identity
            np.testing.assert_allclose(-Ab, np.eye(n), atol=0)
            assert np.all(bb == 0)
            continue
        pinv = np.linalg.pinv(A)
        np.testing.assert_allclose(-Ab, np.eye(n) - pinv @ A, atol=1e-10)
        np.testing.assert_allclose(bb, pinv @ b, atol=1e-10)
    traj = _trajectory(P, 40)
    for x, z, _, lam in traj:
        assert np.all(x >= P.lb) and np.all(x <= P.ub)
        for s, (A, b) in enumerate(zip(P.A, P.b)):
            o = P.offs[s]
            k = A.shape[1]
            if A.shape[0]:
                assert np.max(np.abs(A @ z[o:o + k] - b)) <= 1e-10 * max(1.0, np.max(np.abs(b)))
            F = -P.Abar[s]
            assert np.max(np.abs(F @ lam[o:o + k])) <= 1e-9 * max(1.0, np.max(np.abs(lam[o:o + k])))
    r = admm.solve(P, rho=RHO, eps_rel=1e-6, fixed_iters=400)
    m = r.history[:, 0] ** 2 + (r.history[:, 1] / RHO) ** 2
    assert np.all(np.diff(m[1:]) <= 1e-10 * m[1:-1])

"""Planted mistakes in the oracle (on the CPU only): each plausible slip in
one step of Algorithm 1 must make at least one pin fail.  This checks that the
pins constrain every step, not that the oracle is right."""
import math

import numpy as np
import pytest

from opfgen import build_instance, make_13bus
from opfgen.random_lp import random_instance
from oracle import admm
from pin_helpers import termination_is_homogeneous, termination_matches_literal

RHO = 100.0


def _pins_hold(P, f):
    """A compact version of the pins: brute-force global update (P4), KKT local
    update (P3), dual row-space invariant (P5), monotone merit (P6) and the
    closed-form optimum (P8)."""
    rng = np.random.default_rng(0)
    z = rng.normal(size=P.L)
    lam = rng.normal(size=P.L)
    x = admm.global_update(P, z, lam, RHO)
    for i in range(0, P.n, 7):
        sl = np.nonzero(P.gidx == i)[0]
        g = P.c[i] + lam[sl].sum()
        xs = (z[sl].sum() - g / RHO) / len(sl)
        xs = min(max(xs, P.lb[i]), P.ub[i])
        if abs(xs - x[i]) > 1e-9:
            return False
    zs = admm.local_update(P, x, lam, RHO)
    for s in range(0, len(P.idx), 3):
        Ah, bh, _ = admm.rref(P.A[s], P.b[s])
        m, n = Ah.shape
        K = np.block([[RHO * np.eye(n), Ah.T], [Ah, np.zeros((m, m))]])
        o = P.offs[s]
        sol = np.linalg.solve(K, np.concatenate([RHO * x[P.idx[s]] + lam[o:o + n], bh]))
        if np.max(np.abs(sol[:n] - zs[o:o + n])) > 1e-9:
            return False
    r = admm.solve(P, rho=RHO, eps_rel=1e-9, max_iter=40000)
    if not r.converged:
        return False
    m = r.history[:, 0] ** 2 + (r.history[:, 1] / RHO) ** 2
    if np.any(np.diff(m[1:]) > 1e-10 * m[1:-1]):
        return False
    for s in range(len(P.idx)):
        o = P.offs[s]
        k = len(P.idx[s])
        if np.max(np.abs(-P.Abar[s] @ r.lam[o:o + k])) > 1e-7 * max(1.0, np.abs(r.lam[o:o + k]).max()):
            return False
    total = sum(ld.a.sum() for ld in f.loads)
    return abs(r.objective - total) <= 1e-6 * total


@pytest.fixture(scope="module")
def base():
    f = make_13bus(0)
    return f, build_instance(f)


def test_unmutated_oracle_passes(base):
    f, inst = base
    assert _pins_hold(admm.setup(inst), f)


def _mut_global_drop_c(P, z, lam, rho):
    xhat = admm.B_T(P, z - lam / rho) / P.N
    return np.minimum(np.maximum(xhat, P.lb), P.ub)


def _mut_global_closed1_typo(P, z, lam, rho):
    # the printed scalar form, which also divides the sum of copies by rho
    xhat = -(P.c + admm.B_T(P, lam) - admm.B_T(P, z)) / (rho * P.N)
    return np.minimum(np.maximum(xhat, P.lb), P.ub)


def _mut_global_no_clip(P, z, lam, rho):
    return -(1.0 / rho) * P.c / P.N + admm.B_T(P, z - lam / rho) / P.N


def _mut_global_lambda_sign(P, z, lam, rho):
    xhat = -(1.0 / rho) * P.c / P.N + admm.B_T(P, z + lam / rho) / P.N
    return np.minimum(np.maximum(xhat, P.lb), P.ub)


def _mut_local_transpose_sign(P, x, lam, rho):
    d = -rho * x[P.gidx] + lam
    z = np.empty(P.L)
    for s in range(len(P.idx)):
        o = P.offs[s]
        k = len(P.idx[s])
        z[o:o + k] = (P.Abar[s] @ d[o:o + k]) / rho + P.bbar[s]
    return z


def _mut_local_drop_bbar(P, x, lam, rho):
    return admm.local_update_loop(P, x, lam, rho) - P.bbar_stacked


def _mut_dual_sign(P, x, z, lam, rho):
    return lam - rho * (x[P.gidx] - z)


def _mut_dual_scale(P, x, z, lam, rho):
    return lam + (x[P.gidx] - z)


MUTANTS = [
    ("global_update", _mut_global_drop_c),
    ("global_update", _mut_global_closed1_typo),
    ("global_update", _mut_global_no_clip),
    ("global_update", _mut_global_lambda_sign),
    ("local_update", _mut_local_transpose_sign),
    ("local_update", _mut_local_drop_bbar),
    ("dual_update", _mut_dual_sign),
    ("dual_update", _mut_dual_scale),
]


@pytest.mark.parametrize("fname,mut", MUTANTS, ids=[m.__name__ for _, m in MUTANTS])
def test_planted_mistake_is_caught(base, monkeypatch, fname, mut):
    f, inst = base
    P = admm.setup(inst)
    monkeypatch.setattr(admm, fname, mut)
    try:
        ok = _pins_hold(P, f)
    except (FloatingPointError, np.linalg.LinAlgError, ValueError, OverflowError):
        ok = False
    assert not ok


def test_planted_factor_mistake_is_caught(base, monkeypatch):
    """A factor without the '- I' (the projector instead of Abar)."""
    f, inst = base
    orig = admm.local_factors

    def bad(A, b):
        Ab, bb = orig(A, b)
        return Ab + np.eye(A.shape[1]), bb
    monkeypatch.setattr(admm, "local_factors", bad)
    P = admm.setup(inst)
    assert not _pins_hold(P, f)


# ---- the termination quantities (Section III-C)

def _mut_res_min(P, x, z, z_prev, lam, rho, eps_rel):
    Bx = x[P.gidx]
    pres = math.sqrt(float(np.sum((Bx - z) ** 2)))
    dres = rho * math.sqrt(float(np.sum((z - z_prev) ** 2)))
    eps_prim = eps_rel * min(math.sqrt(float(np.sum(Bx ** 2))), math.sqrt(float(np.sum(z ** 2))))
    return pres, dres, eps_prim, eps_rel * math.sqrt(float(np.sum(lam ** 2)))


def _mut_res_boyd_dual(P, x, z, z_prev, lam, rho, eps_rel):
    # copies summed before the norm: ||B^T lambda|| instead of the stacked norm
    pres, dres, eps_prim, _ = admm.__dict__["_orig_residuals"](P, x, z, z_prev, lam, rho, eps_rel)
    return pres, dres, eps_prim, eps_rel * math.sqrt(float(np.sum(admm.B_T(P, lam) ** 2)))


def _mut_res_prim_over_variables(P, x, z, z_prev, lam, rho, eps_rel):
    # ||x|| over global variables instead of ||B x|| over slots
    pres, dres, _, eps_dual = admm.__dict__["_orig_residuals"](P, x, z, z_prev, lam, rho, eps_rel)
    eps_prim = eps_rel * max(math.sqrt(float(np.sum(x ** 2))), math.sqrt(float(np.sum(z ** 2))))
    return pres, dres, eps_prim, eps_dual


def _mut_res_dual_by_variables(P, x, z, z_prev, lam, rho, eps_rel):
    # B^T applied to the change of the local copies (sums over copies)
    pres, _, eps_prim, eps_dual = admm.__dict__["_orig_residuals"](P, x, z, z_prev, lam, rho, eps_rel)
    return pres, rho * math.sqrt(float(np.sum(admm.B_T(P, z - z_prev) ** 2))), eps_prim, eps_dual


def _mut_res_dres_no_rho(P, x, z, z_prev, lam, rho, eps_rel):
    pres, dres, eps_prim, eps_dual = admm.__dict__["_orig_residuals"](P, x, z, z_prev, lam, rho, eps_rel)
    return pres, dres / rho, eps_prim, eps_dual


def _mut_res_squared_dual_tol(P, x, z, z_prev, lam, rho, eps_rel):
    pres, dres, eps_prim, _ = admm.__dict__["_orig_residuals"](P, x, z, z_prev, lam, rho, eps_rel)
    return pres, dres, eps_prim, eps_rel * float(np.sum(lam ** 2))


def _mut_res_absolute_floor(P, x, z, z_prev, lam, rho, eps_rel):
    pres, dres, eps_prim, eps_dual = admm.__dict__["_orig_residuals"](P, x, z, z_prev, lam, rho, eps_rel)
    return pres, dres, eps_prim + eps_rel, eps_dual + eps_rel


RES_MUTANTS = [_mut_res_min, _mut_res_boyd_dual, _mut_res_prim_over_variables, _mut_res_dual_by_variables,
               _mut_res_dres_no_rho, _mut_res_squared_dual_tol, _mut_res_absolute_floor]


def _termination_pins_hold():
    """The termination pins: the printed sums with dense B_s (13-bus feeder and the
    edge-case random LP) and homogeneity under an exact scaling of the LP."""
    insts = (build_instance(make_13bus(0)), random_instance(0, n=160))
    return all(termination_matches_literal(admm.setup(i)) and termination_is_homogeneous(i) for i in insts)


def test_unmutated_termination_passes():
    assert _termination_pins_hold()


@pytest.mark.parametrize("mut", RES_MUTANTS, ids=[m.__name__ for m in RES_MUTANTS])
def test_planted_termination_mistake_is_caught(monkeypatch, mut):
    monkeypatch.setitem(admm.__dict__, "_orig_residuals", admm.residuals)
    monkeypatch.setattr(admm, "residuals", mut)
    assert not _termination_pins_hold()

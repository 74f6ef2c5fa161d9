"""Planted mistakes in the oracle (on the CPU only): each plausible slip in
one step of Algorithm 1 must make at least one pin fail.  This checks that the
pins constrain every step, not that the oracle is right."""
import numpy as np
import pytest

from opfgen import build_instance, make_13bus
from oracle import admm

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

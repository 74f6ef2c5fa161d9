"""Helpers shared by the oracle pins and the planted-mistake tests (CPU only)."""
import math

import numpy as np

from oracle import admm

RHO = 100.0


def _trajectory(P, iters):
    z, lam = admm.initial_point(P)
    out = []
    for t in range(iters):
        x = admm.global_update(P, z, lam, RHO)
        zn = admm.local_update(P, x, lam, RHO)
        lam = admm.dual_update(P, x, zn, lam, RHO)
        out.append((x, zn, z, lam))
        z = zn
    return out


def literal_termination(P, x, z, z_prev, lam, rho, eps_rel):
    """The termination quantities of Section III-C evaluated as printed, with an
    explicit dense 0/1 selection matrix B_s (n_s x n) per component: B_s x,
    B_s^T(x_s^t - x_s^{t-1}) and B_s^T lambda_s are vectors of length n, and
    every sum runs over components."""
    pres2 = dres2 = bx2 = zs2 = lam2 = 0.0
    for s in range(len(P.idx)):
        o = int(P.offs[s])
        k = len(P.idx[s])
        B = np.zeros((k, P.n))
        B[np.arange(k), P.idx[s]] = 1.0
        xs, xs_prev, ls = z[o:o + k], z_prev[o:o + k], lam[o:o + k]
        pres2 += float(np.sum((B @ x - xs) ** 2))
        dres2 += float(np.sum((B.T @ (xs - xs_prev)) ** 2))
        bx2 += float(np.sum((B @ x) ** 2))
        zs2 += float(np.sum(xs ** 2))
        lam2 += float(np.sum((B.T @ ls) ** 2))
    return (math.sqrt(pres2), rho * math.sqrt(dres2), eps_rel * max(math.sqrt(bx2), math.sqrt(zs2)),
            eps_rel * math.sqrt(lam2))


def termination_matches_literal(P, iters=12, eps_rel=1e-4, rtol=1e-12):
    for t, (x, z, z_prev, lam) in enumerate(_trajectory(P, iters)):
        got = admm.residuals(P, x, z, z_prev, lam, RHO, eps_rel)
        ref = literal_termination(P, x, z, z_prev, lam, RHO, eps_rel)
        for g, r in zip(got, ref):
            if not abs(g - r) <= rtol * max(abs(r), 1e-300):
                return False
    return True


def scaled_instance(inst, alpha):
    """The same LP with c, every b_s and the bounds multiplied by alpha."""
    import copy
    out = copy.deepcopy(inst)
    out.c = inst.c * alpha
    out.lb = inst.lb * alpha
    out.ub = inst.ub * alpha
    for comp in out.comps:
        comp.b = np.asarray(comp.b, dtype=np.float64) * alpha
    return out


def termination_is_homogeneous(inst, alpha=8.0, iters=400, eps_rel=1e-3):
    """Scaling c, b and the bounds by alpha scales x, z and lambda of every
    iterate by alpha (all three updates are positively homogeneous of degree
    one when the start point is scaled too), so pres, dres, eps_prim and
    eps_dual scale by alpha and the termination test stops at the same
    iteration.  alpha is a power of two, so the scaling is exact in binary
    floating point."""
    P = admm.setup(inst)
    Q = admm.setup(scaled_instance(inst, alpha))
    z0, l0 = admm.initial_point(P)
    r = admm.solve(P, rho=RHO, eps_rel=eps_rel, max_iter=iters, z0=z0, lam0=l0)
    q = admm.solve(Q, rho=RHO, eps_rel=eps_rel, max_iter=iters, z0=alpha * z0, lam0=alpha * l0)
    if r.iterations != q.iterations or r.converged != q.converged:
        return False
    return bool(np.allclose(q.history, alpha * r.history, rtol=1e-12, atol=0.0))

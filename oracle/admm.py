"""ORACLE -- test infrastructure only.

Plain FP64 CPU implementation of the solver-free componentwise ADMM
(Algorithm 1 of the paper).  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this module; the product path never
does.  It shares no code with the HIP library.

Notation follows the paper:
  * A_s, b_s        local equality data of component s (Section III-A, OurModel)
  * B_s             0/1 selection, stored as idx_s (local slot -> global index)
  * Abar_s, bbar_s  precomputed factors of the local update, eq. closed_2
  * x               global variables (clipped to [lb, ub])
  * x_s (stacked z) local copies; lambda_s (stacked lam) duals of B_s x = x_s
  * rho             penalty; eps_rel relative tolerance (termination test)

Readings of the paper used here (each also listed in the design notes):
  * global update: the sparse form of Section IV-C (global_sparse); the scalar
    form closed_1 divides the sum of local copies by rho as well, which does
    not follow from its own 1-D objective;
  * lambda_s has n_s entries (it multiplies B_s x - x_s);
  * residual norms are taken literally: sums over components of the squared
    norms of B_s^T(.), i.e. norms of the stacked vectors;
  * the termination test runs after each full iteration (do-while); z at t=0
    is the initial point, so dres at t = 1 is defined;
  * initial point: lambda = 0; x_s entry = 1 for a voltage variable, the
    midpoint of the bounds when both are finite, 0 otherwise.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

VOLTAGE = 2


# ----------------------------------------------------------------------------
# Row reduction (Section IV-B): [A_s | b_s] -> reduced row echelon form
# ----------------------------------------------------------------------------

class InfeasibleComponent(ValueError):
    pass


def rref(A: np.ndarray, b: np.ndarray):
    """Gauss-Jordan elimination with partial pivoting on the augmented matrix
    [A | b].  Returns the nonzero rows (full row rank) of the reduced form and
    the pivot columns.  Pivot tolerance max(m, n) * eps * max|A|.  A zero row
    of A whose right-hand side is nonzero means the equations contradict each
    other (InfeasibleComponent)."""
    M = np.hstack([np.asarray(A, dtype=np.float64), np.asarray(b, dtype=np.float64).reshape(-1, 1)])
    m, n = A.shape
    amax = float(np.max(np.abs(A))) if A.size else 0.0
    tol = max(m, n) * np.finfo(np.float64).eps * max(amax, 1e-300)
    row = 0
    pivots = []
    for col in range(n):
        if row >= m:
            break
        p = row + int(np.argmax(np.abs(M[row:, col])))
        if abs(M[p, col]) <= tol:
            M[row:, col] = 0.0
            continue
        if p != row:
            M[[row, p]] = M[[p, row]]
        M[row] = M[row] / M[row, col]
        for r in range(m):
            if r != row and M[r, col] != 0.0:
                M[r] = M[r] - M[r, col] * M[row]
        pivots.append(col)
        row += 1
    rest = M[row:, n]
    bscale = max(1.0, float(np.max(np.abs(b)))) if len(b) else 1.0
    if rest.size and np.max(np.abs(rest)) > tol * bscale:
        raise InfeasibleComponent("row reduction found 0 = nonzero")
    return M[:row, :n].copy(), M[:row, n].copy(), pivots


def local_factors(A: np.ndarray, b: np.ndarray):
    """Precomputation of Algorithm 1 (closed_2):
         Abar_s = A_s^T (A_s A_s^T)^{-1} A_s - I,   bbar_s = A_s^T (A_s A_s^T)^{-1} b_s
    on the row-reduced (full row rank) A_s."""
    Ah, bh, _ = rref(A, b)
    n = A.shape[1]
    if Ah.shape[0] == 0:
        return -np.eye(n), np.zeros(n)
    G = Ah @ Ah.T
    Abar = Ah.T @ np.linalg.solve(G, Ah) - np.eye(n)
    bbar = Ah.T @ np.linalg.solve(G, bh)
    return Abar, bbar


# ----------------------------------------------------------------------------
# Problem set-up
# ----------------------------------------------------------------------------

@dataclass
class Problem:
    n: int
    c: np.ndarray
    lb: np.ndarray
    ub: np.ndarray
    var_kind: np.ndarray
    idx: list                 # idx_s per component (int64 arrays)
    Abar: list                # Abar_s per component
    bbar: list                # bbar_s per component
    A: list                   # original A_s (for invariants)
    b: list
    gidx: np.ndarray = None   # stacked idx (B as a slot -> variable map)
    N: np.ndarray = None      # diag(B^T B): number of copies of each variable
    offs: np.ndarray = None   # slot offset of each component
    buckets: dict = field(default_factory=dict)   # n_s -> (component ids, stacked Abar, slots)
    bbar_stacked: np.ndarray = None               # [bbar_1; ...; bbar_S]

    @property
    def L(self) -> int:
        return int(self.offs[-1])


def setup(inst) -> Problem:
    """Validates the componentwise instance and precomputes the local factors."""
    idx = []
    Abar = []
    bbar = []
    As = []
    bs = []
    for comp in inst.comps:
        ix = np.asarray(comp.idx, dtype=np.int64)
        if len(set(ix.tolist())) != len(ix):
            raise ValueError("B_s must select each global variable at most once")
        Ab, bb = local_factors(comp.A, comp.b)
        idx.append(ix)
        Abar.append(Ab)
        bbar.append(bb)
        As.append(np.asarray(comp.A, dtype=np.float64))
        bs.append(np.asarray(comp.b, dtype=np.float64))
    gidx = np.concatenate(idx) if idx else np.zeros(0, np.int64)
    N = np.bincount(gidx, minlength=inst.n).astype(np.float64)
    if np.any(N == 0):
        raise ValueError("every global variable needs at least one local copy (B^T B invertible)")
    lb = np.asarray(inst.lb, np.float64)
    ub = np.asarray(inst.ub, np.float64)
    if np.any(lb > ub):
        raise ValueError("lb > ub")
    offs = np.zeros(len(idx) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(i) for i in idx])
    P = Problem(n=inst.n, c=np.asarray(inst.c, np.float64), lb=lb, ub=ub,
                var_kind=np.asarray(inst.var_kind, np.uint8), idx=idx, Abar=Abar, bbar=bbar, A=As, b=bs,
                gidx=gidx, N=N, offs=offs,
                bbar_stacked=np.concatenate(bbar) if bbar else np.zeros(0))
    # the per-component products of one size are evaluated together (the
    # "for s in [S] in parallel" loop of Algorithm 1); the arithmetic of each
    # component is unchanged
    by = {}
    for s, ix in enumerate(idx):
        by.setdefault(len(ix), []).append(s)
    for k, ss in by.items():
        ss = np.asarray(ss, dtype=np.int64)
        P.buckets[k] = (ss, np.stack([Abar[s] for s in ss]) if len(ss) else None,
                        np.stack([offs[s] + np.arange(k) for s in ss]))
    return P


def initial_point(P: Problem):
    """Initial lambda_s and x_s (Section V-A default setting)."""
    lam = np.zeros(P.L)
    z = np.empty(P.L)
    for j, i in enumerate(P.gidx):
        if P.var_kind[i] == VOLTAGE:
            z[j] = 1.0
        elif np.isfinite(P.lb[i]) and np.isfinite(P.ub[i]):
            z[j] = 0.5 * (P.lb[i] + P.ub[i])
        else:
            z[j] = 0.0
    return z, lam


# ----------------------------------------------------------------------------
# One iteration of Algorithm 1
# ----------------------------------------------------------------------------

def B_T(P: Problem, v: np.ndarray) -> np.ndarray:
    """B^T v: sum of the local entries that copy each global variable."""
    return np.bincount(P.gidx, weights=v, minlength=P.n)


def global_update(P: Problem, z: np.ndarray, lam: np.ndarray, rho: float) -> np.ndarray:
    """Global update, sparse form (global_sparse):
         xhat = -(1/rho)(B^T B)^{-1} c + (B^T B)^{-1} B^T (z - lam/rho)
         x    = min(max(xhat, lb), ub)."""
    xhat = -(1.0 / rho) * P.c / P.N + B_T(P, z - lam / rho) / P.N
    return np.minimum(np.maximum(xhat, P.lb), P.ub)


def local_update(P: Problem, x: np.ndarray, lam: np.ndarray, rho: float) -> np.ndarray:
    """Local update (closed_2) for every component:
         d_s = -rho B_s x - lambda_s,   x_s = (1/rho) Abar_s d_s + bbar_s."""
    d = -rho * x[P.gidx] - lam
    z = np.empty(P.L)
    for k, (ss, Ab, slots) in P.buckets.items():
        ds = d[slots]                                  # (cnt, k)
        zs = np.matmul(Ab, ds[:, :, None])[:, :, 0] / rho
        z[slots] = zs
    return z + P.bbar_stacked


def local_update_loop(P: Problem, x: np.ndarray, lam: np.ndarray, rho: float) -> np.ndarray:
    """The same local update, one component at a time (used to check the
    grouped evaluation)."""
    z = np.empty(P.L)
    for s in range(len(P.idx)):
        o = P.offs[s]
        k = len(P.idx[s])
        d = -rho * x[P.idx[s]] - lam[o:o + k]
        z[o:o + k] = (P.Abar[s] @ d) / rho + P.bbar[s]
    return z


def dual_update(P: Problem, x: np.ndarray, z: np.ndarray, lam: np.ndarray, rho: float) -> np.ndarray:
    """lambda_s <- lambda_s + rho (B_s x - x_s)   (ADMM-3 / dual_sparse)."""
    return lam + rho * (x[P.gidx] - z)


def residuals(P: Problem, x, z, z_prev, lam, rho, eps_rel):
    """Primal/dual residuals and tolerances of the termination test."""
    Bx = x[P.gidx]
    pres = math.sqrt(float(np.sum((Bx - z) ** 2)))
    dres = rho * math.sqrt(float(np.sum((z - z_prev) ** 2)))
    eps_prim = eps_rel * max(math.sqrt(float(np.sum(Bx ** 2))), math.sqrt(float(np.sum(z ** 2))))
    eps_dual = eps_rel * math.sqrt(float(np.sum(lam ** 2)))
    return pres, dres, eps_prim, eps_dual


@dataclass
class Result:
    x: np.ndarray
    z: np.ndarray
    lam: np.ndarray
    iterations: int
    converged: bool
    objective: float
    pres: float
    dres: float
    eps_prim: float
    eps_dual: float
    history: np.ndarray       # (iterations, 4): pres, dres, eps_prim, eps_dual


def balance_factor(pres, dres, eps_prim, eps_dual, mu, tau, relative=True):
    """Residual balancing, the first acceleration Section III-D points to
    (Wohlberg): in the relative form the primal and dual residuals are
    compared after each is divided by its tolerance of the termination test,
    in the plain form as they are; the penalty grows by tau when the primal
    one exceeds mu times the dual one, shrinks by tau in the opposite case,
    else stays."""
    if relative:
        rp = pres / eps_prim if eps_prim > 0 else math.inf
        rd = dres / eps_dual if eps_dual > 0 else math.inf
    else:
        rp, rd = pres, dres
    if rp > mu * rd:
        return tau
    if rd > mu * rp:
        return 1.0 / tau
    return 1.0


def solve(P: Problem, rho: float = 100.0, eps_rel: float = 1e-3, max_iter: int = 1_000_000,
          z0=None, lam0=None, fixed_iters: int | None = None, record=True, progress=None,
          balance=None, local_updates: int = 1) -> Result:
    """Algorithm 1: global update, then local and dual updates, until the
    termination test holds (or max_iter / fixed_iters iterations).

    balance = (every, mu, tau, lag, rho_min, rho_max[, relative]) varies the
    penalty by residual balancing: after iteration t with t % every == 0 the
    factor f of balance_factor() on the residuals of t changes the penalty of
    iteration t + lag on, rho_{t+lag} = min(max(rho_{t+lag-1} f, rho_min),
    rho_max); the textbook rule is lag = 1 (the next iteration uses the new
    penalty); relative (default True) selects the form of balance_factor().  Every
    iteration t is one plain ADMM iteration with penalty rho_t: its global,
    local and dual updates and its dual residual all use rho_t.  The duals are
    kept unscaled, so a change of rho needs no rescaling of lambda, and the
    projection factors do not depend on rho.

    local_updates = k repeats, with the global x of the iteration fixed, the
    local update and the dual update k times (several local updates per
    global update, the second acceleration Section III-D points to); the
    residuals compare the local copies of the iteration with those of the
    previous one."""
    if z0 is None:
        z, lam = initial_point(P)
    else:
        z = np.array(z0, dtype=np.float64)
        lam = np.array(lam0, dtype=np.float64)
    hist = []
    rhos = []
    x = np.minimum(np.maximum(np.zeros(P.n), P.lb), P.ub)
    t = 0
    converged = False
    r = (math.nan,) * 4
    limit = fixed_iters if fixed_iters is not None else max_iter
    lag = int(balance[3]) if balance is not None else 1
    if lag < 1:
        raise ValueError("balance lag must be >= 1")
    sched = {k: rho for k in range(1, lag + 1)}       # rho used by iteration k
    while t < limit:
        z_prev = z
        rt = sched[t + 1]
        x = global_update(P, z, lam, rt)
        for _ in range(local_updates):
            z = local_update(P, x, lam, rt)
            lam = dual_update(P, x, z, lam, rt)
        t += 1
        r = residuals(P, x, z, z_prev, lam, rt, eps_rel)
        nxt = sched[t + lag - 1]
        if balance is not None and t % balance[0] == 0:
            rel = bool(balance[6]) if len(balance) > 6 else True
            f = balance_factor(r[0], r[1], r[2], r[3], balance[1], balance[2], rel)
            nxt = min(max(nxt * f, balance[4]), balance[5])
        sched[t + lag] = nxt
        sched.pop(t, None)
        if record:
            hist.append(r)
            rhos.append(rt)
        if progress is not None and t % progress == 0:
            print(f"oracle t={t} pres={r[0]:.3e}/{r[2]:.3e} dres={r[1]:.3e}/{r[3]:.3e}", flush=True)
        if fixed_iters is None and r[0] <= r[2] and r[1] <= r[3]:
            converged = True
            break
    res = Result(x=x, z=z, lam=lam, iterations=t, converged=converged, objective=float(P.c @ x),
                 pres=r[0], dres=r[1], eps_prim=r[2], eps_dual=r[3],
                 history=np.asarray(hist).reshape(-1, 4))
    res.rho_final = sched.get(t + 1, rho)
    res.rho_history = np.asarray(rhos)          # rho used by iterations 1..t (when recorded)
    return res

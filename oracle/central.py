"""ORACLE -- test infrastructure only.

The centralised multi-phase linear OPF of Section II-A (lindist3flow / LP_model)
assembled directly from a feeder, independently of the componentwise builder,
and solved with SciPy's HiGHS as a brute-force reference for the ADMM.

Independence from the componentwise builder is deliberate: the variable order
is different (lines first), the voltage-drop matrices are formed from the
complex closed form Mp = -2 Re(Gamma o conj(Z)), Mq = 2 Im(Gamma o conj(Z)) with
Gamma = alpha alpha^H, alpha = (1, e^{-j2pi/3}, e^{j2pi/3}) instead of the
printed 3x3 entries, and the delta-load block is derived from the per-phase
complex power S^b_phi = V_phi (S_{phi,phi+}/V_{phi,phi+} - S_{phi-,phi}/V_{phi-,phi})
under balanced voltages.  Variable keys use the same tuple names as the
componentwise instance so that the two can be compared.
"""
from __future__ import annotations

import cmath
import math

import numpy as np
import scipy.sparse as sp
from scipy.optimize import linprog

ALPHA = np.array([1.0, cmath.exp(-2j * math.pi / 3), cmath.exp(2j * math.pi / 3)])


def mp_mq_complex(r: np.ndarray, x: np.ndarray):
    """Mp = -2 Re(Gamma o conj(Z)), Mq = 2 Im(Gamma o conj(Z)), Z = r + jx."""
    gamma = np.outer(ALPHA, ALPHA.conj())
    zc = (r - 1j * x)
    prod = gamma * zc
    return -2.0 * prod.real, 2.0 * prod.imag


def delta_block():
    """Linear map from phase-pair consumption (S_ab, S_bc, S_ca) to per-phase
    withdrawals (S_a, S_b, S_c) under balanced unit voltages, as a real 6x6
    matrix acting on (p_ab, p_bc, p_ca, q_ab, q_bc, q_ca) and returning
    (p_a, p_b, p_c, q_a, q_b, q_c)."""
    V = ALPHA
    pairs = [(0, 1), (1, 2), (2, 0)]                # ab, bc, ca
    Vp = [V[i] - V[j] for i, j in pairs]
    M = np.zeros((6, 6))
    for k in range(6):
        s = np.zeros(3, dtype=complex)
        if k < 3:
            s[k] = 1.0
        else:
            s[k - 3] = 1.0j
        out = np.zeros(3, dtype=complex)
        for ph in range(3):
            # current of pair (i, j) flows out of phase i into phase j
            for q, (i, j) in enumerate(pairs):
                if i == ph:
                    out[ph] += V[ph] * s[q] / Vp[q]
                if j == ph:
                    out[ph] -= V[ph] * s[q] / Vp[q]
        M[:3, k] = out.real
        M[3:, k] = out.imag
    return M


class CentralLP:
    def __init__(self, feeder):
        f = feeder
        self.f = f
        keys = []
        lb = []
        ub = []
        cost = []

        def add(key, lo=-np.inf, hi=np.inf, cst=0.0):
            keys.append(key)
            lb.append(lo)
            ub.append(hi)
            cost.append(cst)

        for e, ln in enumerate(f.lines):
            for ph in ln.phases:
                for nm in (("p", e, "ij", ph), ("p", e, "ji", ph), ("q", e, "ij", ph), ("q", e, "ji", ph)):
                    add(nm)
        for l, ld in enumerate(f.loads):
            for ph in ld.phases:
                for nm in ("pd", "qd", "pb", "qb"):
                    add((nm, l, ph))
        for i in range(f.n_bus):
            for ph in f.bus_phases[i]:
                add(("w", i, ph), f.wmin[i, ph], f.wmax[i, ph])
        for k, g in enumerate(f.gens):
            for ph in g.phases:
                add(("pg", k, ph), g.pmin[ph], g.pmax[ph], g.cost)
                add(("qg", k, ph), g.qmin[ph], g.qmax[ph])
        self.keys = keys
        self.pos = {k: i for i, k in enumerate(keys)}
        self.lb = np.array(lb)
        self.ub = np.array(ub)
        self.c = np.array(cost)
        rows, cols, vals, rhs = [], [], [], []
        r = 0

        def eq(co, b):
            nonlocal r
            for key, v in co:
                rows.append(r)
                cols.append(self.pos[key])
                vals.append(v)
            rhs.append(b)
            r += 1

        P = self.pos
        # linearised power flow (no shunts, unit taps)
        for e, ln in enumerate(f.lines):
            mp, mq = mp_mq_complex(ln.r, ln.x)
            for ph in ln.phases:
                eq([(("p", e, "ij", ph), 1.0), (("p", e, "ji", ph), 1.0)], 0.0)
                eq([(("q", e, "ij", ph), 1.0), (("q", e, "ji", ph), 1.0)], 0.0)
                co = [(("w", ln.parent, ph), 1.0), (("w", ln.child, ph), -1.0)]
                for ps in ln.phases:
                    co.append((("p", e, "ij", ps), mp[ph, ps]))
                    co.append((("q", e, "ij", ps), mq[ph, ps]))
                eq(co, 0.0)
        # power balance (lines, loads and generators listed per bus first, in
        # ascending order, so every row holds the same terms in the same order
        # as a scan over all of them)
        at_line = [[] for _ in range(f.n_bus)]
        at_load = [[] for _ in range(f.n_bus)]
        at_gen = [[] for _ in range(f.n_bus)]
        for e, ln in enumerate(f.lines):
            at_line[ln.parent].append(e)
            if ln.child != ln.parent:
                at_line[ln.child].append(e)
        for l, ld in enumerate(f.loads):
            at_load[ld.bus].append(l)
        for k, g in enumerate(f.gens):
            at_gen[g.bus].append(k)
        for i in range(f.n_bus):
            for ph in f.bus_phases[i]:
                for a, gname, bname in (("p", "pg", "pb"), ("q", "qg", "qb")):
                    co = []
                    for e in sorted(at_line[i]):
                        ln = f.lines[e]
                        if ph in ln.phases and ln.parent == i:
                            co.append(((a, e, "ij", ph), 1.0))
                        if ph in ln.phases and ln.child == i:
                            co.append(((a, e, "ji", ph), 1.0))
                    for l in at_load[i]:
                        if ph in f.loads[l].phases:
                            co.append(((bname, l, ph), 1.0))
                    for k in at_gen[i]:
                        if ph in f.gens[k].phases:
                            co.append(((gname, k, ph), -1.0))
                    eq(co, 0.0)
        # loads: voltage-dependent consumption, then wye / delta withdrawal
        D = delta_block()
        for l, ld in enumerate(f.loads):
            scale = 1.0 if ld.conn == "wye" else 3.0
            for ph in ld.phases:
                for nm, ref, ex in (("pd", ld.a[ph], ld.alpha[ph]), ("qd", ld.b[ph], ld.beta[ph])):
                    # d - ref*ex/2*scale*w = ref*(1 - ex/2)
                    eq([((nm, l, ph), 1.0), (("w", ld.bus, ph), -ref * ex / 2.0 * scale)], ref * (1.0 - ex / 2.0))
            if ld.conn == "wye":
                for ph in ld.phases:
                    eq([(("pb", l, ph), 1.0), (("pd", l, ph), -1.0)], 0.0)
                    eq([(("qb", l, ph), 1.0), (("qd", l, ph), -1.0)], 0.0)
            else:
                # (pb, qb) = D (pd, qd): six equations
                src = [("pd", l, 0), ("pd", l, 1), ("pd", l, 2), ("qd", l, 0), ("qd", l, 1), ("qd", l, 2)]
                dst = [("pb", l, 0), ("pb", l, 1), ("pb", l, 2), ("qb", l, 0), ("qb", l, 1), ("qb", l, 2)]
                for o in range(6):
                    co = [(dst[o], 1.0)] + [(src[k], -D[o, k]) for k in range(6)]
                    eq(co, 0.0)
        self.A = sp.csr_matrix((vals, (rows, cols)), shape=(r, len(keys)))
        self.b = np.array(rhs)

    def solve(self):
        res = linprog(self.c, A_eq=self.A, b_eq=self.b, bounds=list(zip(self.lb, self.ub)), method="highs")
        if res.status != 0:
            raise RuntimeError(res.message)
        return res

    def value_range(self, key, objective, tol=1e-9):
        """Min and max of one variable over the optimal face (objective held
        at its optimum within tol, relative) -- certifies uniqueness."""
        k = self.pos[key]
        c = np.zeros(len(self.keys))
        c[k] = 1.0
        A_ub = sp.csr_matrix(self.c.reshape(1, -1))
        bnd = list(zip(self.lb, self.ub))
        lim = [objective + tol * max(1.0, abs(objective))]
        lo = linprog(c, A_ub=A_ub, b_ub=lim, A_eq=self.A, b_eq=self.b, bounds=bnd, method="highs")
        hi = linprog(-c, A_ub=A_ub, b_ub=lim, A_eq=self.A, b_eq=self.b, bounds=bnd, method="highs")
        return lo.fun, -hi.fun

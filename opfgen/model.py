"""Componentwise linear OPF instance (the input of the solver-free ADMM).

Turns a `Feeder` into the data of the reformulated model of Section III-A:
    min c^T x   s.t.  A_s x_s = b_s (each component s),  B_s x = x_s,  lb <= x <= ub
with the global vector x ordered as in the abstract LP form of Section II-A
(generators, voltages, loads, line flows).  Each B_s is a 0/1 selection stored
as the index list idx_s (local slot -> global variable).

Equations follow Section II-A: power balance (balance equations), the
voltage-dependent load model VDLM-1..4, the wye relation VDLM-5, the delta
relations VDLM-6..10 and the linearised power flow (loss equations and the
voltage-magnitude equation with the matrices Mp, Mq).

Decomposition follows Section V-A: one component per bus and per line, except
that a leaf bus is merged into its only line, so S = nodes + lines - leaves.

Readings where the paper is silent (each listed in the design notes):
  * line shunts, bus shunts and tap ratios are absent (g^s = b^s = 0, tau = 1);
  * a variable joins a component only through a nonzero coefficient (so the
    voltage of a bus with only constant-power loads lives in line components);
  * delta loads occur on three-phase buses only; phase pairs d1, d2, d3 are
    ab, bc, ca;
  * the substation's p^g costs 1 per phase, DER p^g costs 0, DER q^g is fixed
    to 0, flows and load variables are unbounded.
This module contains no step of the ADMM itself.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .feeder import Feeder, _mp_mq_explicit

SQ3 = math.sqrt(3.0)

KIND_FREE = 0
KIND_BOUNDED = 1
KIND_VOLTAGE = 2


@dataclass
class Component:
    kind: str                 # "bus", "line" or "leaf+line"
    ident: tuple              # ("bus", i) / ("line", e)
    A: np.ndarray             # (m_s, n_s) float64
    b: np.ndarray             # (m_s,)
    idx: np.ndarray           # (n_s,) int64, sorted global indices


@dataclass
class Instance:
    name: str
    n: int
    c: np.ndarray
    lb: np.ndarray
    ub: np.ndarray
    var_kind: np.ndarray      # uint8: 0 free, 1 bounded, 2 voltage
    var_keys: list
    comps: list               # list[Component]
    feeder: Feeder | None = None

    @property
    def S(self) -> int:
        return len(self.comps)

    @property
    def L(self) -> int:
        return int(sum(len(c.idx) for c in self.comps))

    def flat(self):
        """Concatenated arrays in the layout of the C-ABI problem struct."""
        comp_m = np.array([c.A.shape[0] for c in self.comps], dtype=np.int32)
        comp_n = np.array([c.A.shape[1] for c in self.comps], dtype=np.int32)
        A_vals = np.concatenate([c.A.ravel() for c in self.comps]).astype(np.float64)
        b_vals = np.concatenate([c.b for c in self.comps]).astype(np.float64)
        idx = np.concatenate([c.idx for c in self.comps]).astype(np.int32)
        return comp_m, comp_n, A_vals, b_vals, idx

    def stats(self) -> dict:
        m = np.array([c.A.shape[0] for c in self.comps])
        ns = np.array([c.A.shape[1] for c in self.comps])
        allidx = np.concatenate([c.idx for c in self.comps])
        cnt = np.bincount(allidx, minlength=self.n)
        return dict(S=self.S, n=self.n, L=int(ns.sum()), sum_m=int(m.sum()),
                    m_min=int(m.min()), m_max=int(m.max()), n_min=int(ns.min()), n_max=int(ns.max()),
                    n_mean=float(ns.mean()), n_sd=float(ns.std()), sum_n2=int((ns.astype(np.int64) ** 2).sum()),
                    max_copies=int(cnt.max()), min_copies=int(cnt.min()))


class _Vars:
    def __init__(self):
        self.keys = []
        self.index = {}
        self.lb = []
        self.ub = []
        self.kind = []
        self.cost = []

    def add(self, key, lb=-np.inf, ub=np.inf, kind=None, cost=0.0):
        self.index[key] = len(self.keys)
        self.keys.append(key)
        self.lb.append(lb)
        self.ub.append(ub)
        if kind is None:
            kind = KIND_BOUNDED if (np.isfinite(lb) and np.isfinite(ub)) else KIND_FREE
        self.kind.append(kind)
        self.cost.append(cost)

    def __getitem__(self, key):
        return self.index[key]


def _variables(f: Feeder) -> _Vars:
    V = _Vars()
    for k, g in enumerate(f.gens):
        for ph in g.phases:
            V.add(("pg", k, ph), g.pmin[ph], g.pmax[ph], cost=g.cost)
            V.add(("qg", k, ph), g.qmin[ph], g.qmax[ph])
    for i in range(f.n_bus):
        for ph in f.bus_phases[i]:
            V.add(("w", i, ph), f.wmin[i, ph], f.wmax[i, ph], kind=KIND_VOLTAGE)
    for l, ld in enumerate(f.loads):
        for ph in ld.phases:
            V.add(("pb", l, ph))
            V.add(("qb", l, ph))
            V.add(("pd", l, ph))
            V.add(("qd", l, ph))
    for e, ln in enumerate(f.lines):
        for ph in ln.phases:
            V.add(("p", e, "ij", ph))
            V.add(("q", e, "ij", ph))
            V.add(("p", e, "ji", ph))
            V.add(("q", e, "ji", ph))
    return V


def _equations(f: Feeder, V: _Vars):
    """Yield (owner, coeffs{global index: value}, rhs).  owner is ("bus", i)
    or ("line", e) before leaf merging."""
    eqs = []
    loads_at = [[] for _ in range(f.n_bus)]
    for l, ld in enumerate(f.loads):
        loads_at[ld.bus].append(l)
    gens_at = [[] for _ in range(f.n_bus)]
    for k, g in enumerate(f.gens):
        gens_at[g.bus].append(k)
    lines_at = [[] for _ in range(f.n_bus)]
    for e, ln in enumerate(f.lines):
        lines_at[ln.parent].append((e, "ij"))
        lines_at[ln.child].append((e, "ji"))

    for i in range(f.n_bus):
        own = ("bus", i)
        # power balance, one real and one reactive equation per phase
        for ph in f.bus_phases[i]:
            for pq, gq, lq in (("p", "pg", "pb"), ("q", "qg", "qb")):
                co = {}
                for e, side in lines_at[i]:
                    if ph in f.lines[e].phases:
                        co[V[(pq, e, side, ph)]] = 1.0
                for l in loads_at[i]:
                    if ph in f.loads[l].phases:
                        co[V[(lq, l, ph)]] = 1.0
                for k in gens_at[i]:
                    if ph in f.gens[k].phases:
                        co[V[(gq, k, ph)]] = -1.0
                eqs.append((own, co, 0.0))
        # voltage-dependent load model and the wye / delta relations
        for l in loads_at[i]:
            ld = f.loads[l]
            wmul = 1.0 if ld.conn == "wye" else 3.0
            for ph in ld.phases:
                for dq, ref, ex in (("pd", ld.a[ph], ld.alpha[ph]), ("qd", ld.b[ph], ld.beta[ph])):
                    # d = ref*ex/2 * (wmul*w - 1) + ref
                    co = {V[(dq, l, ph)]: 1.0}
                    cw = -ref * ex / 2.0 * wmul
                    if cw != 0.0:
                        co[V[("w", i, ph)]] = cw
                    eqs.append((own, co, ref - ref * ex / 2.0, ("load", l, dq, ph)))
            if ld.conn == "wye":
                for ph in ld.phases:
                    eqs.append((own, {V[("pb", l, ph)]: 1.0, V[("pd", l, ph)]: -1.0}, 0.0))
                    eqs.append((own, {V[("qb", l, ph)]: 1.0, V[("qd", l, ph)]: -1.0}, 0.0))
            else:
                assert ld.phases == (0, 1, 2), "delta loads are three-phase"
                pb = [V[("pb", l, ph)] for ph in range(3)]
                qb = [V[("qb", l, ph)] for ph in range(3)]
                pd = [V[("pd", l, ph)] for ph in range(3)]
                qd = [V[("qd", l, ph)] for ph in range(3)]
                # VDLM-6
                co = {}
                for ph in range(3):
                    co[pb[ph]] = 1.0
                    co[pd[ph]] = -1.0
                eqs.append((own, co, 0.0))
                co = {}
                for ph in range(3):
                    co[qb[ph]] = 1.0
                    co[qd[ph]] = -1.0
                eqs.append((own, co, 0.0))
                # VDLM-7 .. VDLM-10 (phase 1 -> index 0, etc.)
                eqs.append((own, {pb[1]: 1.5, qb[1]: -SQ3 / 2, pd[1]: -1.0, pd[0]: -0.5, qd[0]: SQ3 / 2}, 0.0))
                eqs.append((own, {pb[1]: SQ3 / 2, qb[1]: 1.5, pd[0]: -SQ3 / 2, qd[0]: -0.5, qd[1]: -1.0}, 0.0))
                eqs.append((own, {qb[1]: SQ3, pb[2]: 1.5, qb[2]: -SQ3 / 2, pd[0]: -0.5, qd[0]: -SQ3 / 2,
                                  pd[2]: -1.0}, 0.0))
                eqs.append((own, {pb[1]: -SQ3, pb[2]: SQ3 / 2, qb[2]: 1.5, pd[0]: SQ3 / 2, qd[0]: -0.5,
                                  qd[2]: -1.0}, 0.0))

    for e, ln in enumerate(f.lines):
        own = ("line", e)
        mp, mq = _mp_mq_explicit(ln.r, ln.x)
        i, j = ln.parent, ln.child
        for ph in ln.phases:
            # losses: p_ij + p_ji = g^s terms (zero), same for q
            eqs.append((own, {V[("p", e, "ij", ph)]: 1.0, V[("p", e, "ji", ph)]: 1.0}, 0.0))
            eqs.append((own, {V[("q", e, "ij", ph)]: 1.0, V[("q", e, "ji", ph)]: 1.0}, 0.0))
        for ph in ln.phases:
            # w_i - tau w_j + sum_psi Mp (p_ij) + sum_psi Mq (q_ij) = 0
            co = {V[("w", i, ph)]: 1.0, V[("w", j, ph)]: -1.0}
            for ps in ln.phases:
                if mp[ph, ps] != 0.0:
                    co[V[("p", e, "ij", ps)]] = co.get(V[("p", e, "ij", ps)], 0.0) + mp[ph, ps]
                if mq[ph, ps] != 0.0:
                    co[V[("q", e, "ij", ps)]] = co.get(V[("q", e, "ij", ps)], 0.0) + mq[ph, ps]
            eqs.append((own, co, 0.0))
    return eqs


def build_instance(f: Feeder) -> Instance:
    V = _variables(f)
    eqs = _equations(f, V)
    deg = f.degree()
    # leaf merging: a degree-1 bus joins the component of its only line
    owner_of_bus = {}
    for e, ln in enumerate(f.lines):
        for b in (ln.parent, ln.child):
            if deg[b] == 1:
                owner_of_bus[b] = ("line", e)
    groups = {}
    order = []
    for own, co, rhs, *tag in eqs:
        if own[0] == "bus" and own[1] in owner_of_bus:
            own = owner_of_bus[own[1]]
        if own not in groups:
            groups[own] = []
            order.append(own)
        groups[own].append((co, rhs, tag[0] if tag else None))
    # components in network order: buses first (by id), then lines (by id)
    order.sort(key=lambda o: (0 if o[0] == "bus" else 1, o[1]))
    comps = []
    load_rows = []          # (row offset in the stacked b, load id) of every VDLM-1/2 row
    boff = 0
    for own in order:
        rows = groups[own]
        cols = sorted({j for co, _, _ in rows for j, v in co.items() if v != 0.0})
        pos = {j: k for k, j in enumerate(cols)}
        A = np.zeros((len(rows), len(cols)))
        b = np.zeros(len(rows))
        for r, (co, rhs, tag) in enumerate(rows):
            for j, v in co.items():
                if v != 0.0:
                    A[r, pos[j]] += v
            b[r] = rhs
            if tag is not None:
                load_rows.append((boff + r, tag[1]))
        boff += len(rows)
        kind = own[0]
        if own[0] == "line":
            ln = f.lines[own[1]]
            if deg[ln.parent] == 1 or deg[ln.child] == 1:
                kind = "leaf+line"
        comps.append(Component(kind=kind, ident=own, A=A, b=b, idx=np.asarray(cols, dtype=np.int64)))
    n = len(V.keys)
    inst = Instance(name=f.name, n=n, c=np.asarray(V.cost, dtype=np.float64),
                    lb=np.asarray(V.lb, dtype=np.float64), ub=np.asarray(V.ub, dtype=np.float64),
                    var_kind=np.asarray(V.kind, dtype=np.uint8), var_keys=list(V.keys), comps=comps,
                    feeder=f)
    inst.load_rows = np.asarray(load_rows, dtype=np.int64).reshape(-1, 2)
    return inst


def scenario_rhs(inst: Instance, bus_factors: np.ndarray) -> np.ndarray:
    """Right-hand sides of load scenarios on one topology: scenario k scales the
    reference powers of every load at bus i by bus_factors[k, i].  Valid for
    constant-power loads (alpha = beta = 0), whose equations then keep the
    same A_s and change only b_s.  Returns [K, sum m_s]."""
    f = inst.feeder
    for ld in f.loads:
        if np.any(ld.alpha != 0) or np.any(ld.beta != 0):
            raise ValueError("load scenarios with a shared A_s need constant-power loads")
    base = np.concatenate([c.b for c in inst.comps])
    K = bus_factors.shape[0]
    out = np.repeat(base[None, :], K, axis=0)
    rows = inst.load_rows[:, 0]
    buses = np.array([f.loads[l].bus for l in inst.load_rows[:, 1]], dtype=np.int64)
    out[:, rows] = base[rows][None, :] * bus_factors[:, buses]
    return out


def scenario_zip(inst: Instance, bus_factors: np.ndarray):
    """Load scenarios on one topology with voltage-dependent (ZIP) loads:
    scenario k scales the reference powers of every load at bus i by
    bus_factors[k, i].  In a load row (VDLM-1/2) both the right-hand side and
    the coefficient on the bus voltage w are proportional to the reference
    power, so a scenario changes b_s and those coefficients only.  Returns
    (b_scen [K, sum m_s], a_pos [nv] flat positions into the stacked A values,
    a_scen [K, nv] their values per scenario)."""
    f = inst.feeder
    base_b = np.concatenate([c.b for c in inst.comps])
    K = bus_factors.shape[0]
    b_scen = np.repeat(base_b[None, :], K, axis=0)
    rows = inst.load_rows[:, 0]
    buses = np.array([f.loads[l].bus for l in inst.load_rows[:, 1]], dtype=np.int64)
    b_scen[:, rows] = base_b[rows][None, :] * bus_factors[:, buses]
    # stacked row -> (component, local row); flat offset of each component's A
    row_comp, row_local, a_off = [], [], []
    off = 0
    for s_, c in enumerate(inst.comps):
        a_off.append(off)
        off += c.A.size
        row_comp.extend([s_] * c.A.shape[0])
        row_local.extend(range(c.A.shape[0]))
    pos, val_base, bus_of = [], [], []
    for r, bus in zip(rows, buses):
        s_ = row_comp[r]
        c = inst.comps[s_]
        i = row_local[r]
        for j in range(c.A.shape[1]):
            key = inst.var_keys[c.idx[j]]
            if c.A[i, j] != 0.0 and key is not None and key[0] == "w":
                pos.append(a_off[s_] + i * c.A.shape[1] + j)
                val_base.append(c.A[i, j])
                bus_of.append(bus)
    a_pos = np.asarray(pos, dtype=np.int64)
    a_scen = np.asarray(val_base)[None, :] * bus_factors[:, np.asarray(bus_of, dtype=np.int64)]
    return b_scen, a_pos, a_scen


def with_rhs(inst: Instance, b: np.ndarray) -> Instance:
    """A copy of the instance whose stacked right-hand side is b."""
    comps = []
    o = 0
    for c in inst.comps:
        m = c.A.shape[0]
        comps.append(Component(kind=c.kind, ident=c.ident, A=c.A, b=np.array(b[o:o + m]), idx=c.idx))
        o += m
    new = Instance(name=inst.name, n=inst.n, c=inst.c, lb=inst.lb, ub=inst.ub, var_kind=inst.var_kind,
                   var_keys=inst.var_keys, comps=comps, feeder=inst.feeder)
    new.load_rows = getattr(inst, "load_rows", None)
    return new


def instance_from_flat(name, n, c, lb, ub, var_kind, comp_m, comp_n, A_vals, b_vals, idx) -> Instance:
    comps = []
    pa = pb = pi = 0
    for m, k in zip(comp_m, comp_n):
        m = int(m)
        k = int(k)
        comps.append(Component(kind="?", ident=("comp", len(comps)), A=np.asarray(A_vals[pa:pa + m * k]).reshape(m, k).copy(),
                               b=np.asarray(b_vals[pb:pb + m]).copy(), idx=np.asarray(idx[pi:pi + k], dtype=np.int64).copy()))
        pa += m * k
        pb += m
        pi += k
    return Instance(name=name, n=int(n), c=np.asarray(c, float), lb=np.asarray(lb, float), ub=np.asarray(ub, float),
                    var_kind=np.asarray(var_kind, np.uint8), var_keys=[None] * int(n), comps=comps)

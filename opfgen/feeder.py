"""Seeded synthetic radial distribution feeders.

This module only draws random network data (topology, phasing, impedances,
loads, distributed generators).  It holds no part of the ADMM arithmetic and no
part of the optimisation model; `opfgen.model` turns a feeder into the
componentwise linear program of the paper (Section II).

The paper evaluates on the IEEE 13/123/8500-bus feeders (Section V-A), which
are not available here.  The generators below produce seeded stand-ins with
the same structure: a three-phase substation, a radial tree, three-phase trunk
and one/two-phase laterals, wye loads with constant-power (or ZIP) behaviour,
optional delta loads on three-phase buses and switchable DERs.

Per-unit convention (the paper does not state one): S_base = 1 MVA,
V_base = V_LL / sqrt(3), Z_base = V_base^2 / S_base.  Powers are per phase in
per unit of S_base, impedances in per unit of Z_base.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

S_BASE_VA = 1.0e6
W_MIN = 0.95 ** 2
W_MAX = 1.05 ** 2


@dataclass
class Line:
    parent: int               # upstream (from) bus i
    child: int                # downstream (to) bus j
    phases: tuple             # subset of (0, 1, 2)
    r: np.ndarray             # 3x3 series resistance, per unit
    x: np.ndarray             # 3x3 series reactance, per unit


@dataclass
class Load:
    bus: int
    phases: tuple
    conn: str                 # "wye" or "delta"
    a: np.ndarray             # reference real power per phase (pu), VDLM-1
    b: np.ndarray             # reference reactive power per phase (pu), VDLM-2
    alpha: np.ndarray         # voltage exponent for real power
    beta: np.ndarray          # voltage exponent for reactive power


@dataclass
class Gen:
    bus: int
    phases: tuple
    pmin: np.ndarray
    pmax: np.ndarray
    qmin: np.ndarray
    qmax: np.ndarray
    cost: float               # objective coefficient on each phase's p^g
    kind: str = "der"         # "substation" or "der"


@dataclass
class Feeder:
    name: str
    seed: int
    n_bus: int
    bus_phases: list          # tuple of phases per bus
    lines: list               # list[Line]; radial tree rooted at bus 0
    loads: list               # list[Load]
    gens: list                # list[Gen]
    wmin: np.ndarray          # (n_bus, 3) lower bound on w (unused phases ignored)
    wmax: np.ndarray          # (n_bus, 3)
    v_ll_kv: float
    kappa: float = 1.0        # load scaling applied for voltage feasibility
    meta: dict = field(default_factory=dict)

    @property
    def root(self) -> int:
        return 0

    def degree(self) -> np.ndarray:
        deg = np.zeros(self.n_bus, dtype=np.int64)
        for ln in self.lines:
            deg[ln.parent] += 1
            deg[ln.child] += 1
        return deg


# ----------------------------------------------------------------------------
# topology
# ----------------------------------------------------------------------------

def random_recursive_tree(n: int, rng: np.random.Generator) -> np.ndarray:
    """parent[k] ~ U{0..k-1} for k >= 1 (parent[0] = -1)."""
    parent = np.full(n, -1, dtype=np.int64)
    for k in range(1, n):
        parent[k] = rng.integers(0, k)
    return parent


def dfs_branching_tree(n: int, rng: np.random.Generator, depth_cap: int | None = None) -> np.ndarray:
    """Depth-first random tree: every expanded bus draws U{1..4} children and
    the first child is expanded before its siblings, under a depth cap.  The
    cap grows until the tree reaches n buses."""
    if n == 1:
        return np.full(1, -1, dtype=np.int64)
    cap = depth_cap or max(2, int(math.ceil(math.log(n) / math.log(2.5))))
    while True:
        parent = [-1]
        depth = [0]
        stack = [0]
        while len(parent) < n and stack:
            u = stack.pop()
            if depth[u] >= cap:
                continue
            k = int(rng.integers(1, 5))
            kids = []
            for _ in range(k):
                if len(parent) >= n:
                    break
                parent.append(u)
                depth.append(depth[u] + 1)
                kids.append(len(parent) - 1)
            stack.extend(reversed(kids))
        if len(parent) >= n:
            return np.asarray(parent, dtype=np.int64)
        cap += 1


def _children(parent: np.ndarray) -> list:
    ch = [[] for _ in range(len(parent))]
    for k in range(1, len(parent)):
        ch[parent[k]].append(k)
    return ch


def _subtree_sizes(parent: np.ndarray) -> np.ndarray:
    size = np.ones(len(parent), dtype=np.int64)
    for k in range(len(parent) - 1, 0, -1):   # children have larger ids than parents
        size[parent[k]] += size[k]
    return size


def assign_phases(parent: np.ndarray, rng: np.random.Generator, trunk_frac: float,
                  p_single: float) -> list:
    """Three-phase trunk (root-connected buses with the largest subtrees, about
    `trunk_frac` of all buses), laterals one-phase with probability `p_single`,
    otherwise two-phase.  Descendants of a lateral root inherit its phases."""
    n = len(parent)
    size = _subtree_sizes(parent)
    # smallest subtree-size threshold whose (root-connected) set of buses is at
    # most trunk_frac of all buses; subtree sizes shrink along every path, so
    # {k : size[k] >= thr} always contains the root and is connected
    target = max(1, int(round(trunk_frac * n)))
    counts = np.bincount(size, minlength=n + 2)[::-1].cumsum()[::-1]   # counts[t] = #{size >= t}
    thr = int(np.argmax(counts <= target))
    phases = [None] * n
    phases[0] = (0, 1, 2)
    for k in range(1, n):
        p = parent[k]
        if phases[p] == (0, 1, 2) and size[k] >= thr:
            phases[k] = (0, 1, 2)
        elif phases[p] == (0, 1, 2):
            if rng.random() < p_single:
                phases[k] = (int(rng.integers(0, 3)),)
            else:
                drop = int(rng.integers(0, 3))
                phases[k] = tuple(ph for ph in (0, 1, 2) if ph != drop)
        else:
            phases[k] = phases[p]
    return phases


# ----------------------------------------------------------------------------
# electrical data
# ----------------------------------------------------------------------------

def random_line_impedance(rng: np.random.Generator, z_base: float):
    """R, X ~ U[0.05, 0.5] ohm/km per entry of the 3x3, symmetrised; length
    ~ U[0.1, 1] km; returned in per unit."""
    length = rng.uniform(0.1, 1.0)
    r = rng.uniform(0.05, 0.5, size=(3, 3))
    x = rng.uniform(0.05, 0.5, size=(3, 3))
    r = 0.5 * (r + r.T) * length / z_base
    x = 0.5 * (x + x.T) * length / z_base
    return r, x


def _pf_q(p: float, pf: float) -> float:
    return p * math.tan(math.acos(pf))


def make_load(bus: int, phases: tuple, p_total_kw: float, pf: float, conn: str = "wye",
              alpha: float = 0.0, beta: float = 0.0) -> Load:
    a = np.zeros(3)
    b = np.zeros(3)
    per = p_total_kw * 1e3 / S_BASE_VA / len(phases)
    for ph in phases:
        a[ph] = per
        b[ph] = _pf_q(per, pf)
    al = np.zeros(3)
    be = np.zeros(3)
    for ph in phases:
        al[ph] = alpha
        be[ph] = beta
    return Load(bus=bus, phases=tuple(phases), conn=conn, a=a, b=b, alpha=al, beta=be)


def substation(phases=(0, 1, 2)) -> Gen:
    inf = np.full(3, np.inf)
    return Gen(bus=0, phases=tuple(phases), pmin=-inf.copy(), pmax=inf.copy(), qmin=-inf.copy(),
               qmax=inf.copy(), cost=1.0, kind="substation")


def make_der(bus: int, phases: tuple, cap_kw: float, on: bool) -> Gen:
    pmax = np.zeros(3)
    if on:
        for ph in phases:
            pmax[ph] = cap_kw * 1e3 / S_BASE_VA / len(phases)
    return Gen(bus=bus, phases=tuple(phases), pmin=np.zeros(3), pmax=pmax, qmin=np.zeros(3),
               qmax=np.zeros(3), cost=0.0, kind="der")


def _build(name, seed, parent, phases, rng, v_ll_kv, loads, gens) -> Feeder:
    n = len(parent)
    v_base = v_ll_kv * 1e3 / math.sqrt(3.0)
    z_base = v_base ** 2 / S_BASE_VA
    lines = []
    for k in range(1, n):
        r, x = random_line_impedance(rng, z_base)
        lines.append(Line(parent=int(parent[k]), child=k, phases=tuple(phases[k]), r=r, x=x))
    wmin = np.full((n, 3), W_MIN)
    wmax = np.full((n, 3), W_MAX)
    wmin[0, :] = 1.0
    wmax[0, :] = 1.0
    f = Feeder(name=name, seed=seed, n_bus=n, bus_phases=[tuple(p) for p in phases], lines=lines,
               loads=loads, gens=gens, wmin=wmin, wmax=wmax, v_ll_kv=v_ll_kv)
    return f


# ----------------------------------------------------------------------------
# voltage feasibility (load scaling kappa)
# ----------------------------------------------------------------------------

def _mp_mq_explicit(r: np.ndarray, x: np.ndarray):
    """The 3x3 voltage-drop coefficient matrices as printed in Section II-A
    (after the linearised power-flow equations)."""
    s3 = math.sqrt(3.0)
    mp = np.array([
        [-2 * r[0, 0], r[0, 1] - s3 * x[0, 1], r[0, 2] + s3 * x[0, 2]],
        [r[1, 0] + s3 * x[1, 0], -2 * r[1, 1], r[1, 2] - s3 * x[1, 2]],
        [r[2, 0] - s3 * x[2, 0], r[2, 1] + s3 * x[2, 1], -2 * r[2, 2]],
    ])
    mq = np.array([
        [-2 * x[0, 0], x[0, 1] + s3 * r[0, 1], x[0, 2] - s3 * r[0, 2]],
        [x[1, 0] - s3 * r[1, 0], -2 * x[1, 1], x[1, 2] + s3 * r[1, 2]],
        [x[2, 0] + s3 * r[2, 0], x[2, 1] - s3 * r[2, 1], -2 * x[2, 2]],
    ])
    return mp, mq


def _sweep_w(f: Feeder, der_on: bool) -> np.ndarray:
    """Voltage profile of constant-power wye loads on the lossless linearised
    model (used only to scale generated loads into the voltage box)."""
    n = f.n_bus
    inj_p = np.zeros((n, 3))
    inj_q = np.zeros((n, 3))
    for ld in f.loads:
        inj_p[ld.bus] += ld.a
        inj_q[ld.bus] += ld.b
    if der_on:
        for g in f.gens:
            if g.kind == "der":
                inj_p[g.bus] -= g.pmax
    flow_p = inj_p.copy()
    flow_q = inj_q.copy()
    # lines in breadth-first order from the substation
    kids = [[] for _ in range(n)]
    for ln in f.lines:
        kids[ln.parent].append(ln)
    order = []
    frontier = [0]
    while frontier:
        nxt = []
        for a in frontier:
            for ln in kids[a]:
                order.append(ln)
                nxt.append(ln.child)
        frontier = nxt
    for ln in reversed(order):
        flow_p[ln.parent] += flow_p[ln.child]
        flow_q[ln.parent] += flow_q[ln.child]
    w = np.ones((n, 3))
    for ln in order:
        mp, mq = _mp_mq_explicit(ln.r, ln.x)
        ph = list(ln.phases)
        P = np.zeros(3)
        Q = np.zeros(3)
        P[ph] = flow_p[ln.child, ph]
        Q[ph] = flow_q[ln.child, ph]
        # w_i = w_j - Mp p_ij - Mq q_ij  ->  w_j = w_i + Mp p + Mq q
        dw = mp[np.ix_(ph, ph)] @ P[ph] + mq[np.ix_(ph, ph)] @ Q[ph]
        w[ln.child, :] = w[ln.parent, :]
        w[ln.child, ph] = w[ln.parent, ph] + dw
    return w


def scale_for_voltage(f: Feeder, lo: float = 0.92, hi: float = 1.08) -> Feeder:
    """Scale all loads and DER capacities by one factor kappa <= 1 so that the
    swept w stays inside [lo, hi] with DERs off and at capacity.  The bounds of
    the model stay [0.95^2, 1.05^2]; the margin keeps them inactive."""
    worst = 0.0
    for der_on in (False, True):
        w = _sweep_w(f, der_on)
        for i in range(f.n_bus):
            for ph in f.bus_phases[i]:
                worst = max(worst, (1.0 - w[i, ph]) / (1.0 - lo), (w[i, ph] - 1.0) / (hi - 1.0))
    kappa = 1.0 if worst <= 1.0 else 1.0 / worst
    if kappa < 1.0:
        for ld in f.loads:
            ld.a *= kappa
            ld.b *= kappa
        for g in f.gens:
            if g.kind == "der":
                g.pmax *= kappa
    f.kappa = kappa
    return f


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def make_13bus(seed: int = 0, zip_variant: bool = False) -> Feeder:
    """13 three-phase buses on a random recursive tree, 12 lines, 8 loads on
    distinct non-root buses with P_total ~ U[20, 400] kW split equally over the
    phases, pf ~ U[0.85, 0.98], constant-power wye.  `zip_variant` draws
    alpha = beta in {0, 1, 2} with probabilities (.6, .2, .2) and makes one
    load a three-phase delta load."""
    rng = np.random.default_rng([13, seed])
    n = 13
    parent = random_recursive_tree(n, rng)
    phases = [(0, 1, 2)] * n
    buses = rng.choice(np.arange(1, n), size=8, replace=False)
    loads = []
    for k, b in enumerate(buses):
        p = rng.uniform(20, 400)
        pf = rng.uniform(0.85, 0.98)
        conn, al = "wye", 0.0
        if zip_variant:
            al = float(rng.choice([0.0, 1.0, 2.0], p=[0.6, 0.2, 0.2]))
            if k == 0:
                conn, al = "delta", 0.0
        loads.append(make_load(int(b), (0, 1, 2), p, pf, conn, al, al))
    gens = [substation()]
    f = _build("13bus" + ("-zip" if zip_variant else ""), seed, parent, phases, rng, 4.16, loads, gens)
    return scale_for_voltage(f)


def make_radial(n_bus: int, seed: int, *, n_loads: int, load_mu_kw: float, load_sigma: float,
                n_der: int, trunk_frac: float, p_single: float, v_ll_kv: float,
                name: str, der_cap=(50.0, 200.0), tag: int = 0, tree: str = "dfs",
                zip_mix: bool = False) -> Feeder:
    """General radial feeder: depth-first branching tree (branching U{1..4})
    or, with tree="recursive", a random recursive tree.  `zip_mix` gives every
    load alpha = beta in {0, 1, 2} with probabilities (.6, .2, .2), drawn from a
    separate stream so that everything else equals the constant-power feeder."""
    rng = np.random.default_rng([n_bus, seed, tag])
    if tree == "dfs":
        parent = dfs_branching_tree(n_bus, rng)
    else:
        parent = random_recursive_tree(n_bus, rng)
    phases = assign_phases(parent, rng, trunk_frac, p_single)
    n_loads = min(n_loads, n_bus - 1)
    buses = rng.choice(np.arange(1, n_bus), size=n_loads, replace=False)
    loads = []
    rng_zip = np.random.default_rng([n_bus, seed, tag, 77])
    for b in buses:
        p = float(rng.lognormal(math.log(load_mu_kw), load_sigma))
        pf = rng.uniform(0.85, 0.98)
        al = float(rng_zip.choice([0.0, 1.0, 2.0], p=[0.6, 0.2, 0.2])) if zip_mix else 0.0
        loads.append(make_load(int(b), phases[b], p, pf, "wye", al, al))
    gens = [substation()]
    if n_der:
        der_buses = rng.choice(np.arange(1, n_bus), size=min(n_der, n_bus - 1), replace=False)
        for b in der_buses:
            cap = rng.uniform(*der_cap)
            on = bool(rng.random() < 0.75)
            gens.append(make_der(int(b), phases[b], cap, on))
    f = _build(name, seed, parent, phases, rng, v_ll_kv, loads, gens)
    return scale_for_voltage(f)


def make_123bus(seed: int = 0, zip_mix: bool = False) -> Feeder:
    """123 buses on a random recursive tree, ~50% three-phase trunk, laterals
    60/40 one-/two-phase (30%/20% of all buses), 85 loads lognormal(ln 40 kW,
    0.6), 4 switchable DERs with capacity U[50, 200] kW, V_LL = 4.16 kV."""
    return make_radial(123, seed, n_loads=85, load_mu_kw=40.0, load_sigma=0.6, n_der=4,
                       trunk_frac=0.5, p_single=0.6, v_ll_kv=4.16, name="123bus" + ("-zip" if zip_mix else ""),
                       tree="recursive", zip_mix=zip_mix)


def make_8500bus(seed: int = 0, n_bus: int = 8500) -> Feeder:
    """~8500 buses, ~60% of them on one-phase laterals, 1200 loads
    lognormal(ln 5 kW, 0.8), 40 DERs with capacity U[50, 200] kW, 12.47 kV."""
    return make_radial(n_bus, seed, n_loads=1200 * n_bus // 8500, load_mu_kw=5.0, load_sigma=0.8,
                       n_der=40 * n_bus // 8500, trunk_frac=0.4, p_single=0.9, v_ll_kv=12.47,
                       name=f"{n_bus}bus")


def make_2500bus(seed: int = 0, zip_mix: bool = False) -> Feeder:
    """One 2500-bus feeder as the 8500-bus generator, ~353 loads, no DERs
    (with `zip_mix`, voltage-dependent loads as in make_radial)."""
    return make_radial(2500, seed, n_loads=353, load_mu_kw=5.0, load_sigma=0.8, n_der=0,
                       trunk_frac=0.4, p_single=0.9, v_ll_kv=12.47, name="2500bus" + ("-zip" if zip_mix else ""),
                       zip_mix=zip_mix)


def scenario_load_factors(f: Feeder, k_scen: int, seed: int, sigma: float = 0.3) -> np.ndarray:
    """Per-scenario, per-bus multiplicative load factors lognormal(0, sigma);
    scenario k uses the stream (seed, k).  Shape (k_scen, n_bus)."""
    out = np.empty((k_scen, f.n_bus))
    for k in range(k_scen):
        rng = np.random.default_rng([seed, k, 4])
        out[k] = rng.lognormal(0.0, sigma, size=f.n_bus)
    return out


def by_name(name: str, seed: int = 0) -> Feeder:
    if name in ("13bus", "c1"):
        return make_13bus(seed)
    if name in ("13bus-zip", "c1z"):
        return make_13bus(seed, zip_variant=True)
    if name in ("123bus", "c2"):
        return make_123bus(seed)
    if name in ("8500bus", "c3"):
        return make_8500bus(seed)
    if name in ("2500bus", "c4"):
        return make_2500bus(seed)
    if name == "2500bus-zip":
        return make_2500bus(seed, zip_mix=True)
    if name == "123bus-zip":
        return make_123bus(seed, zip_mix=True)
    if name.endswith("bus") and name[:-3].isdigit():
        return make_8500bus(seed, n_bus=int(name[:-3]))
    raise KeyError(name)

"""Seeded request streams for the serving runtime.

Feeder families: one base radial feeder per family, with a set of normally
open tie lines between three-phase trunk buses.  A request closes one tie and
opens a trunk line on the loop it creates (the network stays radial), and
draws fresh loads.  Sizes are log-uniform in [13, 8500] buses; arrivals are
a Poisson process.  Only random network data and the componentwise model are
produced here.
"""
from __future__ import annotations

import copy
import hashlib
import math
from dataclasses import dataclass

import numpy as np

from .feeder import Feeder, Line, make_radial, scale_for_voltage
from .model import Instance, build_instance


@dataclass
class Family:
    fid: int
    base: Feeder
    ties: list                     # [(u, v)] trunk bus pairs not joined by a line


def family_size(fid: int, seed: int, lo: int = 13, hi: int = 8500) -> int:
    rng = np.random.default_rng([seed, fid, 55])
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def make_family(fid: int, seed: int = 0, n_bus: int | None = None) -> Family:
    n = n_bus or family_size(fid, seed)
    n = max(n, 4)
    f = make_radial(n, seed, n_loads=max(1, int(0.45 * n)), load_mu_kw=10.0, load_sigma=0.8,
                    n_der=max(0, n // 200), trunk_frac=0.4, p_single=0.9, v_ll_kv=12.47,
                    name=f"family{fid}-{n}bus", tag=1000 + fid)
    rng = np.random.default_rng([seed, fid, 77])
    trunk = [i for i in range(n) if f.bus_phases[i] == (0, 1, 2)]
    adj = {(ln.parent, ln.child) for ln in f.lines} | {(ln.child, ln.parent) for ln in f.lines}
    ties = []
    n_ties = max(1, math.ceil(n / 100))
    tries = 0
    while len(ties) < n_ties and len(trunk) >= 3 and tries < 50 * n_ties:
        tries += 1
        u, v = (int(a) for a in rng.choice(trunk, size=2, replace=False))
        if (u, v) in adj or (u, v) in ties or (v, u) in ties:
            continue
        ties.append((u, v))
    return Family(fid=fid, base=f, ties=ties)


def _tree_path(f: Feeder, u: int, v: int):
    parent = {ln.child: (ln.parent, e) for e, ln in enumerate(f.lines)}

    def up(a):
        out = [a]
        while a in parent:
            a = parent[a][0]
            out.append(a)
        return out
    pu, pv = up(u), up(v)
    common = set(pu) & set(pv)
    lca = next(a for a in pu if a in common)
    edges = []
    for start in (u, v):
        a = start
        while a != lca:
            p, e = parent[a]
            edges.append(e)
            a = p
    return edges


def reconfigure(fam: Family, tie_index: int, rng: np.random.Generator) -> Feeder:
    """Close tie `tie_index` and open a random three-phase line on the loop it
    creates; the result is re-oriented from the substation.  Line ids of lines
    that keep their orientation are preserved (so are their variables)."""
    f = fam.base
    u, v = fam.ties[tie_index % len(fam.ties)]
    loop = [e for e in _tree_path(f, u, v) if f.lines[e].phases == (0, 1, 2)]
    if not loop:
        return copy.deepcopy(f)
    opened = int(rng.choice(loop))
    rz = np.random.default_rng([f.seed, fam.fid, tie_index, 99])
    r = rz.uniform(0.05, 0.5, (3, 3))
    x = rz.uniform(0.05, 0.5, (3, 3))
    zb = (f.v_ll_kv * 1e3 / math.sqrt(3.0)) ** 2 / 1e6
    length = rz.uniform(0.1, 1.0)
    tie_line = Line(parent=u, child=v, phases=(0, 1, 2), r=0.5 * (r + r.T) * length / zb,
                    x=0.5 * (x + x.T) * length / zb)
    edges = [(e, ln) for e, ln in enumerate(f.lines) if e != opened] + [(len(f.lines), tie_line)]
    nbr = {i: [] for i in range(f.n_bus)}
    for e, ln in edges:
        nbr[ln.parent].append((ln.child, e, ln))
        nbr[ln.child].append((ln.parent, e, ln))
    # orient from the substation; a line keeps its position in the list (so
    # its variables keep their names) and the tie takes the opened one's place
    order = [0]
    seen = {0}
    new_lines = {}
    k = 0
    while k < len(order):
        a = order[k]
        k += 1
        for b, e, ln in sorted(nbr[a], key=lambda t: t[1]):
            if b in seen:
                continue
            seen.add(b)
            order.append(b)
            if ln.parent == a:
                new_lines[e] = ln
            else:
                new_lines[e] = Line(parent=a, child=b, phases=ln.phases, r=ln.r.T.copy(), x=ln.x.T.copy())
    lines = [new_lines[e] if e != opened else new_lines[len(f.lines)] for e in range(len(f.lines))]
    g = copy.deepcopy(f)
    g.lines = lines
    g.name = f"{f.name}-tie{tie_index}"
    return g


def with_loads(f: Feeder, rng: np.random.Generator, sigma: float = 0.3) -> Feeder:
    """Fresh loads: every bus's load scaled by lognormal(0, sigma)."""
    g = copy.deepcopy(f)
    fac = rng.lognormal(0.0, sigma, size=f.n_bus)
    for ld in g.loads:
        ld.a = ld.a * fac[ld.bus]
        ld.b = ld.b * fac[ld.bus]
    g.kappa = 1.0
    return scale_for_voltage(g)


def component_keys(inst: Instance) -> np.ndarray:
    """64-bit key per component: a hash of its kind and of the keys of the
    variables it copies (equal keys = same local structure)."""
    out = np.empty(inst.S, dtype=np.uint64)
    for s, comp in enumerate(inst.comps):
        h = hashlib.blake2b(digest_size=8)
        h.update(repr((comp.kind, [inst.var_keys[i] for i in comp.idx], comp.A.shape)).encode())
        h.update(np.ascontiguousarray(comp.A).tobytes())
        out[s] = np.frombuffer(h.digest(), dtype=np.uint64)[0]
    return out


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng([seed, 31])
    return np.cumsum(rng.exponential(1.0 / rate, size=n))

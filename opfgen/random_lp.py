"""Seeded random componentwise LPs for edge-case tests.

Shapes the feeder generator never produces: a component as wide as a
wavefront (64 slots), components without equations, one-slot components, a
redundant (repeated) equation, a variable copied by ten components (more than
a slot keeps in registers), one-sided and infinite bounds.  Each component's
equations are satisfied by one common point x*, so the LP is feasible.  Only
random data and the componentwise layout are produced here.
"""
from __future__ import annotations

import numpy as np

from .model import Component, Instance


def random_instance(seed: int = 0, n: int = 400) -> Instance:
    rng = np.random.default_rng([seed, 6464])
    xstar = rng.uniform(-0.5, 0.5, n)
    comps = []

    def add(idx, m, repeat_row=False):
        idx = np.sort(np.asarray(idx, dtype=np.int64))
        k = len(idx)
        A = rng.normal(0.0, 1.0, (m, k))
        if repeat_row and m >= 1:
            A = np.vstack([A, A[:1]])
        b = A @ xstar[idx]
        comps.append(Component(kind="random", ident=("comp", len(comps)), A=A, b=b, idx=idx))

    add(rng.choice(n, 64, replace=False), 20)                 # a full wavefront
    add(rng.choice(n, 64, replace=False), 0)                  # full width, no equations
    add([3], 0)                                               # one slot, no equations
    add(rng.choice(n, 12, replace=False), 5, repeat_row=True)
    hub = 7
    for _ in range(10):                                       # ten copies of variable `hub`
        others = rng.choice(np.setdiff1d(np.arange(n), [hub]), 5, replace=False)
        add(np.concatenate([[hub], others]), 2)
    while True:                                               # the rest, sizes 2..40
        covered = np.zeros(n, bool)
        for c in comps:
            covered[c.idx] = True
        free = np.nonzero(~covered)[0]
        if len(free) == 0:
            break
        k = int(rng.integers(2, 41))
        pick = rng.choice(free, min(k, len(free)), replace=False)
        extra = rng.choice(n, max(0, k - len(pick)), replace=False)
        idx = np.unique(np.concatenate([pick, extra]))
        add(idx, int(rng.integers(0, max(1, len(idx) // 2))))
    c = np.where(rng.random(n) < 0.3, rng.uniform(-1.0, 1.0, n), 0.0)
    lb = np.full(n, -np.inf)
    ub = np.full(n, np.inf)
    kind = np.zeros(n, np.uint8)
    two = rng.random(n) < 0.4
    lb[two] = xstar[two] - rng.uniform(0.05, 1.0, two.sum())
    ub[two] = xstar[two] + rng.uniform(0.05, 1.0, two.sum())
    kind[two] = 1
    one = (~two) & (rng.random(n) < 0.2)
    lb[one] = xstar[one] - 1.0
    return Instance(name=f"random-lp-{seed}", n=n, c=c, lb=lb, ub=ub, var_kind=kind,
                    var_keys=[None] * n, comps=comps)


def inconsistent_instance(seed: int = 0, n: int = 120) -> Instance:
    """A random feasible LP with two more one-slot components that fix
    variable 0 to +0.5 and to -0.5: every component's equations are
    solvable, their consensus is not (an infeasible LP for the stall watch)."""
    base = random_instance(seed, n)
    comps = list(base.comps)
    for v in (0.5, -0.5):
        comps.append(Component(kind="random", ident=("pin", v), A=np.ones((1, 1)), b=np.array([v]),
                               idx=np.array([0], dtype=np.int64)))
    return Instance(name=f"inconsistent-lp-{seed}", n=n, c=base.c, lb=base.lb, ub=base.ub,
                    var_kind=base.var_kind, var_keys=[None] * n, comps=comps)

"""Pins of the componentwise model builder (the seeded input generator)
against closed forms the paper's model must satisfy.  CPU only."""
import cmath
import math

import numpy as np
import pytest

from opfgen import build_instance, by_name, make_13bus, make_123bus
from opfgen.feeder import _mp_mq_explicit, dfs_branching_tree
from opfgen.model import _equations, _variables
from oracle.central import CentralLP, delta_block, mp_mq_complex


def test_mp_mq_printed_entries_match_complex_closed_form():
    """Section II-A: the printed Mp, Mq equal -2Re(Gamma o conj Z) and
    2Im(Gamma o conj Z) entry by entry (all 18 entries), for arbitrary
    (also non-symmetric) r, x."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        r = rng.uniform(-1, 1, (3, 3))
        x = rng.uniform(-1, 1, (3, 3))
        mp, mq = _mp_mq_explicit(r, x)
        mp2, mq2 = mp_mq_complex(r, x)
        np.testing.assert_allclose(mp, mp2, rtol=0, atol=1e-14)
        np.testing.assert_allclose(mq, mq2, rtol=0, atol=1e-14)


def test_single_phase_voltage_drop_is_distflow():
    """One phase: w_i - w_j = 2 (r p_ij + x q_ij) (the DistFlow drop)."""
    r = np.diag([0.3, 0.0, 0.0])
    x = np.diag([0.2, 0.0, 0.0])
    mp, mq = _mp_mq_explicit(r, x)
    assert mp[0, 0] == -0.6 and mq[0, 0] == -0.4


def _complex_delta(pd, qd):
    """Per-phase withdrawals of a delta load from phase-pair powers
    S_ab, S_bc, S_ca under balanced unit voltages (physics, written out)."""
    a = cmath.exp(-2j * math.pi / 3)
    Va, Vb, Vc = 1.0, a, a.conjugate()
    Sab, Sbc, Sca = (complex(pd[k], qd[k]) for k in range(3))
    Sa = Va * (Sab / (Va - Vb) - Sca / (Vc - Va))
    Sb = Vb * (Sbc / (Vb - Vc) - Sab / (Va - Vb))
    Sc = Vc * (Sca / (Vc - Va) - Sbc / (Vb - Vc))
    return np.array([Sa.real, Sb.real, Sc.real]), np.array([Sa.imag, Sb.imag, Sc.imag])


def test_delta_rows_vdlm6_10_hold_for_physical_delta_powers():
    """VDLM-6..10 are satisfied by the withdrawals that a delta load with
    pair powers (d1, d2, d3) = (ab, bc, ca) draws, and they determine them."""
    f = make_13bus(0, zip_variant=True)
    V = _variables(f)
    eqs = _equations(f, V)
    l = [k for k, ld in enumerate(f.loads) if ld.conn == "delta"][0]
    keys = [(nm, l, ph) for nm in ("pb", "qb", "pd", "qd") for ph in range(3)]
    cols = [V[k] for k in keys]
    wb = {V[(nm, l, ph)] for nm in ("pb", "qb") for ph in range(3)}
    rows = [e[1] for e in eqs if set(e[1]) <= set(cols) and wb & set(e[1])]
    assert len(rows) == 6
    A = np.array([[co.get(c, 0.0) for c in cols] for co in rows])
    rng = np.random.default_rng(1)
    for _ in range(10):
        pd = rng.uniform(-1, 1, 3)
        qd = rng.uniform(-1, 1, 3)
        pb, qb = _complex_delta(pd, qd)
        v = np.concatenate([pb, qb, pd, qd])
        np.testing.assert_allclose(A @ v, 0.0, atol=1e-13)
    # the six rows fix (pb, qb) given (pd, qd)
    assert np.linalg.matrix_rank(A[:, :6]) == 6
    # the oracle's own delta map agrees with the physics as well
    pd = rng.uniform(-1, 1, 3)
    qd = rng.uniform(-1, 1, 3)
    out = delta_block() @ np.concatenate([pd, qd])
    pb, qb = _complex_delta(pd, qd)
    np.testing.assert_allclose(out, np.concatenate([pb, qb]), atol=1e-13)


@pytest.mark.parametrize("name", ["13bus", "13bus-zip", "123bus", "2500bus"])
def test_component_count_identity_and_cover(name):
    """Section V-A / Table 3: S = nodes + lines - leaves; every variable has a
    local copy; each B_s selects distinct variables."""
    f = by_name(name, 0)
    inst = build_instance(f)
    deg = f.degree()
    leaves = int((deg == 1).sum())
    assert inst.S == f.n_bus + len(f.lines) - leaves
    allidx = np.concatenate([c.idx for c in inst.comps])
    assert np.bincount(allidx, minlength=inst.n).min() >= 1
    for c in inst.comps:
        assert len(set(c.idx.tolist())) == len(c.idx)
        assert c.A.shape == (len(c.b), len(c.idx))


@pytest.mark.parametrize("name", ["13bus", "13bus-zip", "123bus"])
def test_stacked_component_rows_span_the_central_model(name):
    """The stacked A_s x_s = b_s define the same affine set as the centralised
    LP assembled independently from the feeder (rank test on [A | b])."""
    f = by_name(name, 0)
    inst = build_instance(f)
    lp = CentralLP(f)
    assert sorted(map(str, inst.var_keys)) == sorted(map(str, lp.keys))
    perm = np.array([lp.pos[k] for k in inst.var_keys])
    rows = []
    for c in inst.comps:
        M = np.zeros((c.A.shape[0], len(lp.keys) + 1))
        M[:, perm[c.idx]] = c.A
        M[:, -1] = c.b
        rows.append(M)
    S = np.vstack(rows)
    C = np.hstack([lp.A.toarray(), lp.b.reshape(-1, 1)])
    rs = np.linalg.matrix_rank(S)
    rc = np.linalg.matrix_rank(C)
    assert rs == rc == np.linalg.matrix_rank(np.vstack([S, C]))
    # the systems are consistent (b in the column space)
    assert np.linalg.matrix_rank(S[:, :-1]) == rs


def test_objective_and_bounds_layout():
    f = by_name("123bus", 0)
    inst = build_instance(f)
    for k, key in enumerate(inst.var_keys):
        if key[0] == "w":
            assert inst.var_kind[k] == 2
            assert 0.9 < inst.lb[k] <= inst.ub[k] < 1.2
        if key[0] == "pg":
            g = f.gens[key[1]]
            assert inst.c[k] == (1.0 if g.kind == "substation" else 0.0)
        if key[0] in ("p", "q", "pb", "qb", "pd", "qd"):
            assert inst.lb[k] == -np.inf and inst.ub[k] == np.inf


def test_tree_generator_is_radial_and_seeded():
    rng = np.random.default_rng(3)
    parent = dfs_branching_tree(500, rng)
    assert parent[0] == -1 and np.all(parent[1:] < np.arange(1, 500))
    a = build_instance(make_123bus(4))
    b = build_instance(make_123bus(4))
    assert a.n == b.n and all(np.array_equal(x.A, y.A) for x, y in zip(a.comps, b.comps))


def test_scenario_rhs_equals_rebuilt_instance():
    """Scaling the loads of a constant-power feeder changes only b_s: the
    scenario right-hand side equals the one of the rebuilt instance."""
    import copy
    from opfgen import scenario_load_factors, scenario_rhs
    f = by_name("123bus", 0)
    inst = build_instance(f)
    fac = scenario_load_factors(f, 2, 5)
    B = scenario_rhs(inst, fac)
    for k in range(2):
        f2 = copy.deepcopy(f)
        for ld in f2.loads:
            ld.a = ld.a * fac[k, ld.bus]
            ld.b = ld.b * fac[k, ld.bus]
        inst2 = build_instance(f2)
        assert all(np.array_equal(c1.A, c2.A) for c1, c2 in zip(inst.comps, inst2.comps))
        np.testing.assert_allclose(np.concatenate([c.b for c in inst2.comps]), B[k], rtol=1e-15, atol=0)


@pytest.mark.parametrize("name", ["13bus-zip", "123bus-zip"])
def test_zip_scenarios_equal_rebuilt_instances(name):
    """The ZIP scenario generator patches b and the load rows' w coefficients;
    the result equals the instance rebuilt from the feeder with the loads of
    every bus scaled by its factor (same component structure)."""
    import copy
    from opfgen import scenario_load_factors, scenario_zip
    f = by_name(name, 0)
    inst = build_instance(f)
    assert any(np.any(ld.alpha != 0) for ld in f.loads)
    fac = scenario_load_factors(f, 3, seed=5)
    b_scen, a_pos, a_scen = scenario_zip(inst, fac)
    assert len(a_pos) > 0
    cm, cn, A, b, idx = inst.flat()
    for k in range(3):
        g = copy.deepcopy(f)
        for ld in g.loads:
            ld.a = ld.a * fac[k, ld.bus]
            ld.b = ld.b * fac[k, ld.bus]
        ref = build_instance(g)
        cm2, cn2, A2, b2, idx2 = ref.flat()
        assert np.array_equal(cm, cm2) and np.array_equal(cn, cn2) and np.array_equal(idx, idx2)
        Ak = A.copy()
        Ak[a_pos] = a_scen[k]
        np.testing.assert_allclose(Ak, A2, rtol=1e-14, atol=0)
        np.testing.assert_allclose(b_scen[k], b2, rtol=1e-14, atol=1e-300)

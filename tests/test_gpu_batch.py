"""Batched same-topology scenarios (shared A_s, per-scenario b_s) on MFMA with
a three-term bfloat16 split and FP32 accumulation, against the FP64 oracle run
on each scenario separately.  Bar: objective and voltages within 1e-4 relative
(the mixed-precision tolerance); early iterates within 1e-5 relative."""
import sys

import numpy as np
import pytest

from opfgen import build_instance, by_name, scenario_load_factors, scenario_rhs, with_rhs
from oracle import admm

pytestmark = pytest.mark.gpu
RHO = 100.0


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _batch(inst, B, **kw):
    from paper_2501_08293_amd import BatchSolver
    return BatchSolver(inst.n, inst.c, inst.lb, inst.ub, inst.var_kind, *inst.flat(), b_scen=B, **kw)


@pytest.fixture(scope="module")
def case123():
    f = by_name("123bus", 0)
    inst = build_instance(f)
    fac = scenario_load_factors(f, 5, seed=11)
    return inst, scenario_rhs(inst, fac)


def test_batch_early_iterates_match_oracle(case123):
    """max_iter = 10 with an unreachable tolerance: every scenario is recorded
    at iteration 10; x agrees with the oracle's 10th iterate of that scenario."""
    inst, B = case123
    _say("[gpu] batch early iterates 123bus K=5 t=10")
    s = _batch(inst, B, rho=RHO, eps_rel=1e-12, max_iter=10, check_every=4)
    out = s.solve()
    s.close()
    assert np.all(out["iterations"] == 10)
    for k in range(B.shape[0]):
        P = admm.setup(with_rhs(inst, B[k]))
        ref = admm.solve(P, rho=RHO, eps_rel=1e-12, fixed_iters=10)
        err = np.max(np.abs(out["x"][k] - ref.x)) / max(1.0, np.max(np.abs(ref.x)))
        assert err < 1e-5, (k, err)


def test_batch_solutions_match_oracle_per_scenario(case123):
    inst, B = case123
    _say("[gpu] batch solve 123bus K=5 eps=1e-4")
    s = _batch(inst, B, rho=RHO, eps_rel=1e-4, check_every=64)
    out = s.solve()
    s.close()
    assert out["status"] == 0 and out["converged"] == B.shape[0]
    vidx = np.nonzero(inst.var_kind == 2)[0]
    for k in range(B.shape[0]):
        P = admm.setup(with_rhs(inst, B[k]))
        ref = admm.solve(P, rho=RHO, eps_rel=1e-4)
        assert abs(out["objective"][k] - ref.objective) <= 1e-4 * abs(ref.objective), k
        rel = np.max(np.abs(out["x"][k][vidx] - ref.x[vidx]) / np.abs(ref.x[vidx]))
        assert rel <= 1e-4, (k, rel)
        assert abs(int(out["iterations"][k]) - ref.iterations) <= 0.02 * ref.iterations + 2, k
        _say(f"  scenario {k}: iterations {out['iterations'][k]} (oracle {ref.iterations}), "
             f"objective rel err {abs(out['objective'][k] - ref.objective) / abs(ref.objective):.2e}, w rel err {rel:.2e}")


def test_identical_scenarios_give_identical_bits():
    """The same right-hand side in several columns of the MFMA tiles (also
    across the 64-scenario chunks) gives the same result bit for bit."""
    f = by_name("13bus", 0)
    inst = build_instance(f)
    b = np.concatenate([c.b for c in inst.comps])
    B = np.repeat(b[None, :], 70, axis=0)
    _say("[gpu] batch identical scenarios 13bus K=70")
    s = _batch(inst, B, rho=RHO, eps_rel=1e-4, check_every=32)
    out = s.solve()
    s.close()
    assert np.all(out["iterations"] == out["iterations"][0])
    assert np.all(out["x"] == out["x"][0][None, :])
    ref = admm.solve(admm.setup(inst), rho=RHO, eps_rel=1e-4)
    assert abs(out["objective"][0] - ref.objective) <= 1e-4 * abs(ref.objective)


def test_two_term_split_runs_and_stays_close():
    """The two-term split is available; it stalls above the dual tolerance on
    this model, so only closeness to the oracle's solution is required."""
    f = by_name("13bus", 0)
    inst = build_instance(f)
    b = np.concatenate([c.b for c in inst.comps])
    _say("[gpu] batch two-term split 13bus")
    s = _batch(inst, b[None, :], rho=RHO, eps_rel=1e-4, max_iter=20000, check_every=64, split_terms=2)
    out = s.solve(raise_on_error=False)
    s.close()
    ref = admm.solve(admm.setup(inst), rho=RHO, eps_rel=1e-4)
    assert abs(out["objective"][0] - ref.objective) <= 1e-3 * abs(ref.objective)


@pytest.mark.parametrize("name", ["13bus-zip", "123bus-zip"])
def test_zip_scenarios_with_per_scenario_factors_match_oracle(name):
    """Voltage-dependent (ZIP) loads: the load rows' voltage coefficients scale
    with each scenario's loads, so those components are factored per scenario
    and run as per-scenario products; every scenario matches the FP64 oracle
    run on that scenario's own A and b: the stop iteration within 2 % of the
    oracle's, and at the GPU's stop iteration the objective and voltages within
    1e-4 relative of the oracle's iterate (near the 1e-4 test the objective
    still moves by more than 1e-4 between stop iterations a few dozen apart,
    so values are compared at the same iteration)."""
    import copy
    from opfgen import scenario_zip
    f = by_name(name, 0)
    inst = build_instance(f)
    fac = scenario_load_factors(f, 6, seed=21)
    b_scen, a_pos, a_scen = scenario_zip(inst, fac)
    _say(f"[gpu] batch ZIP scenarios {name} K=6, {len(a_pos)} varying A entries")
    s = _batch(inst, b_scen, rho=RHO, eps_rel=1e-4, check_every=64, a_pos=a_pos, a_scen=a_scen)
    out = s.solve()
    s.close()
    assert out["status"] == 0 and out["converged"] == 6
    vidx = np.nonzero(inst.var_kind == 2)[0]
    cm, cn, A, b, idx = inst.flat()
    from opfgen import instance_from_flat
    for k in range(6):
        Ak = A.copy()
        Ak[a_pos] = a_scen[k]
        sk = instance_from_flat(name, inst.n, inst.c, inst.lb, inst.ub, inst.var_kind, cm, cn, Ak, b_scen[k], idx)
        Pk = admm.setup(sk)
        ref = admm.solve(Pk, rho=RHO, eps_rel=1e-4, record=False)
        assert abs(int(out["iterations"][k]) - ref.iterations) <= 0.02 * ref.iterations + 2, k
        same = admm.solve(Pk, rho=RHO, eps_rel=1e-4, fixed_iters=int(out["iterations"][k]), record=False)
        assert abs(out["objective"][k] - same.objective) <= 1e-4 * abs(same.objective), k
        rel = np.max(np.abs(out["x"][k][vidx] - same.x[vidx]) / np.abs(same.x[vidx]))
        assert rel <= 1e-4, (k, rel)


def test_zip_scenarios_on_constant_power_equal_shared_path():
    """With no varying entries the extended set-up is the shared-factor path:
    identical bits."""
    f = by_name("13bus", 0)
    inst = build_instance(f)
    B = scenario_rhs(inst, scenario_load_factors(f, 3, seed=2))
    _say("[gpu] batch extended set-up with nothing varying")
    s1 = _batch(inst, B, rho=RHO, eps_rel=1e-4, check_every=32)
    o1 = s1.solve()
    s1.close()
    s2 = _batch(inst, B, rho=RHO, eps_rel=1e-4, check_every=32, a_pos=np.zeros(0, np.int64),
                a_scen=np.zeros((3, 0)))
    o2 = s2.solve()
    s2.close()
    assert np.array_equal(o1["x"], o2["x"]) and np.array_equal(o1["iterations"], o2["iterations"])


@pytest.fixture(scope="module")
def case2500():
    """The benchmark's batch: 2500-bus feeder, 256 load scenarios (stream seed
    1000), four 64-scenario chunks on the MFMA tiles."""
    f = by_name("2500bus", 0)
    inst = build_instance(f)
    return inst, scenario_rhs(inst, scenario_load_factors(f, 256, seed=1000))


def test_full_size_batch_early_iterates_match_oracle(case2500):
    """At the benchmark's size and launch configuration (K = 256): sampled
    scenarios from every 64-scenario chunk after 20 iterations against the
    oracle's 20th iterate of each (1e-5 relative)."""
    inst, B = case2500
    _say("[gpu] batch 2500bus K=256 t=20, scenarios 0, 70, 141, 255 vs oracle")
    s = _batch(inst, B, rho=RHO, eps_rel=1e-12, max_iter=20, check_every=4)
    out = s.solve()
    s.close()
    assert np.all(out["iterations"] == 20)
    for k in (0, 70, 141, 255):
        P = admm.setup(with_rhs(inst, B[k]))
        ref = admm.solve(P, rho=RHO, eps_rel=1e-12, fixed_iters=20, record=False)
        err = np.max(np.abs(out["x"][k] - ref.x)) / max(1.0, np.max(np.abs(ref.x)))
        assert err < 1e-5, (k, err)


def test_full_size_batch_solve_matches_golden_scenario(case2500):
    """The benchmark's batch solved to eps_rel = 1e-4: scenario 3 against the
    oracle's solve of that scenario to the same tolerance (stored golden):
    objective and sampled voltages within 1e-4 relative, stop iteration
    within 2 %; every scenario converges."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "admm_2500bus-scen3_s0_eps0.0001.json")
    if not os.path.exists(path):
        pytest.skip("golden of batch scenario 3 not written yet")
    g = json.load(open(path))
    inst, B = case2500
    _say("[gpu] batch 2500bus K=256 eps=1e-4 (benchmark configuration), scenario 3 vs golden")
    s = _batch(inst, B, rho=RHO, eps_rel=1e-4, check_every=256)
    out = s.solve()
    s.close()
    assert out["status"] == 0 and out["converged"] == 256
    k = 3
    _say(f"  scenario 3: iterations {out['iterations'][k]} (oracle {g['iterations']}), objective "
         f"{out['objective'][k]:.10g} (oracle {g['objective']:.10g})")
    assert abs(out["objective"][k] - g["objective"]) <= 1e-4 * abs(g["objective"])
    w = out["x"][k][g["w_index"]]
    ref_w = np.array(g["w_value"])
    assert np.max(np.abs(w - ref_w) / np.abs(ref_w)) <= 1e-4
    assert abs(int(out["iterations"][k]) - g["iterations"]) <= 0.02 * g["iterations"]

"""The autotuners: every workgroup order of the batched step kernel gives the
same values bit for bit; the batch and single-instance tuners pick a valid
configuration, write it to the decision cache file and read it back."""
import os
import sys

import numpy as np
import pytest

from opfgen import build_instance, by_name, scenario_load_factors, scenario_rhs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _batch(inst, B, **kw):
    from paper_2501_08293_amd import BatchSolver
    return BatchSolver(inst.n, inst.c, inst.lb, inst.ub, inst.var_kind, *inst.flat(), b_scen=B, **kw)


def test_batch_orders_and_autotune_cache(tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("OPF_ADMM_TUNE_CACHE", str(cache))
    f = by_name("123bus", 0)
    inst = build_instance(f)
    B = scenario_rhs(inst, scenario_load_factors(f, 130, seed=21))
    _say("[gpu] batch autotune 123bus K=130 (three 64-scenario chunks)")
    s = _batch(inst, B, rho=100.0, eps_rel=1e-12, max_iter=60, check_every=20, autotune=True)
    order = s.info().batch_order
    tuned = s.solve()
    s.close()
    assert order in (0, 1, 2, 3)
    assert cache.exists() and "batch/" in cache.read_text()
    # a second set-up reads the decision back from the file
    s = _batch(inst, B, rho=100.0, eps_rel=1e-12, max_iter=60, check_every=20, autotune=True)
    assert s.info().batch_order == order
    s.close()
    # every order computes the same values: the default order (no tuning) gives the tuned run's bits
    s = _batch(inst, B, rho=100.0, eps_rel=1e-12, max_iter=60, check_every=20)
    ref = s.solve()
    s.close()
    assert np.array_equal(tuned["x"], ref["x"]) and np.array_equal(tuned["iterations"], ref["iterations"])


@pytest.mark.parametrize("order,groups", [(0, 1), (1, 1), (2, 1), (3, 1), (1, 2), (3, 2)])
def test_each_batch_order_gives_the_same_bits(tmp_path, monkeypatch, order, groups):
    # a cache file holding the order and the number of scenario groups forces them
    # (70 scenarios: two 64-scenario chunks, the second with 6 scenarios)
    f = by_name("13bus", 0)
    inst = build_instance(f)
    B = scenario_rhs(inst, scenario_load_factors(f, 70, seed=5))
    s = _batch(inst, B, rho=100.0, eps_rel=1e-12, max_iter=40, check_every=8)
    ref = s.solve()
    s.close()
    # the problem's cache key, as the tuner writes it, then a fresh cache file
    # (decisions are kept in memory per file) holding the order
    probe = tmp_path / "probe.txt"
    monkeypatch.setenv("OPF_ADMM_TUNE_CACHE", str(probe))
    _batch(inst, B, rho=100.0, eps_rel=1e-12, max_iter=40, check_every=8, autotune=True).close()
    key = [l for l in probe.read_text().splitlines() if l.startswith("batch/")][-1].split("\t")[0]
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{key}\t{order} {groups}\n")
    monkeypatch.setenv("OPF_ADMM_TUNE_CACHE", str(cache))
    _say(f"[gpu] batch order {order}, {groups} scenario groups vs default, 13bus K=70")
    s = _batch(inst, B, rho=100.0, eps_rel=1e-12, max_iter=40, check_every=8, autotune=True)
    info = s.info()
    assert (info.batch_order, info.batch_groups) == (order, groups)
    out = s.solve()
    s.close()
    assert np.array_equal(out["x"], ref["x"])
    assert np.array_equal(out["iterations"], ref["iterations"])


@pytest.mark.parametrize("groups", [2, 4])
def test_scenario_groups_solve_to_tolerance_with_the_same_bits(tmp_path, monkeypatch, groups):
    """Four 64-scenario chunks of the 123-bus feeder iterated as 2 or 4 groups
    on concurrent streams: every scenario stops at the same iteration with the
    same solution as in one group (scenarios are independent), and the batch
    runs until the last group has stopped."""
    f = by_name("123bus", 0)
    inst = build_instance(f)
    B = scenario_rhs(inst, scenario_load_factors(f, 256, seed=7))
    s = _batch(inst, B, rho=100.0, eps_rel=1e-3, check_every=64)
    ref = s.solve()
    s.close()
    probe = tmp_path / "probe.txt"
    monkeypatch.setenv("OPF_ADMM_TUNE_CACHE", str(probe))
    _batch(inst, B, rho=100.0, eps_rel=1e-3, check_every=64, autotune=True).close()
    key = [l for l in probe.read_text().splitlines() if l.startswith("batch/")][-1].split("\t")[0]
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{key}\t1 {groups}\n")
    monkeypatch.setenv("OPF_ADMM_TUNE_CACHE", str(cache))
    _say(f"[gpu] 123bus K=256 to 1e-3: {groups} scenario groups vs one")
    s = _batch(inst, B, rho=100.0, eps_rel=1e-3, check_every=64, autotune=True)
    assert s.info().batch_groups == groups
    out = s.solve()
    s.close()
    assert ref["converged"] == 256 and out["converged"] == 256
    assert np.array_equal(out["iterations"], ref["iterations"])
    assert np.array_equal(out["x"], ref["x"])
    assert np.array_equal(out["objective"], ref["objective"])
    assert out["total_iterations"] >= int(out["iterations"].max())


def test_single_instance_autotune_cache(tmp_path, monkeypatch):
    from paper_2501_08293_amd import Solver
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("OPF_ADMM_TUNE_CACHE", str(cache))
    inst = build_instance(by_name("13bus-zip", 0))
    _say("[gpu] single-instance autotune writes its decision to the cache file")
    s = Solver(inst.n, inst.c, inst.lb, inst.ub, inst.var_kind, *inst.flat(), rho=100.0, eps_rel=1e-4,
               autotune=True)
    info = s.info()
    s.close()
    txt = cache.read_text()
    assert "single/" in txt
    line = [l for l in txt.splitlines() if l.startswith("single/")][-1]
    k, bw = (int(v) for v in line.split("\t")[1].split())
    assert (info.kernel, info.block_waves) == (k, bw)


def test_scenario_groups_with_zip_loads_give_the_same_bits(tmp_path, monkeypatch):
    """ZIP loads (scenario-varying A_s in their own wavefronts, first in every
    group's launch) with the 64-scenario chunks split over two concurrent
    groups: each scenario gets the bits of the one-group run."""
    from opfgen import scenario_zip
    f = by_name("13bus-zip", 0)
    inst = build_instance(f)
    fac = scenario_load_factors(f, 70, seed=11)
    b_scen, a_pos, a_scen = scenario_zip(inst, fac)

    def mk(**kw):
        return _batch(inst, b_scen, rho=100.0, eps_rel=1e-12, max_iter=60, check_every=20, a_pos=a_pos,
                      a_scen=a_scen, **kw)
    s = mk()
    ref = s.solve()
    s.close()
    probe = tmp_path / "probe.txt"
    monkeypatch.setenv("OPF_ADMM_TUNE_CACHE", str(probe))
    mk(autotune=True).close()
    key = [l for l in probe.read_text().splitlines() if l.startswith("batch/")][-1].split("\t")[0]
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{key}\t1 2\n")
    monkeypatch.setenv("OPF_ADMM_TUNE_CACHE", str(cache))
    _say("[gpu] 13bus-zip K=70: two scenario groups vs one")
    s = mk(autotune=True)
    assert s.info().batch_groups == 2
    out = s.solve()
    s.close()
    assert np.array_equal(out["x"], ref["x"])
    assert np.array_equal(out["iterations"], ref["iterations"])

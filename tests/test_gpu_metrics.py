"""Per-solve metrics records (JSON Lines in the file named by
OPF_ADMM_METRICS): one line per single-instance solve, batched solve and
served request, with the values the calls return."""
import json
import sys

import pytest

from opfgen import build_instance, by_name, scenario_load_factors, scenario_rhs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _lines(path):
    return [json.loads(l) for l in open(path).read().splitlines() if l.strip()]


def test_metrics_records(tmp_path, monkeypatch):
    from paper_2501_08293_amd import BatchSolver, Server, Solver
    path = tmp_path / "m.jsonl"
    monkeypatch.setenv("OPF_ADMM_METRICS", str(path))
    inst = build_instance(by_name("13bus", 0))
    args = (inst.n, inst.c, inst.lb, inst.ub, inst.var_kind) + tuple(inst.flat())
    _say("[gpu] metrics: a solve with history, a fixed run, a noalloc solve, a batch and two served requests")
    s = Solver(*args, rho=100.0, eps_rel=1e-4, history_cap=100000)
    out = s.solve()
    s.solve(fixed_iters=50)
    s.solve(noalloc=True)
    info = s.info()
    s.close()
    f = by_name("13bus", 0)
    B = scenario_rhs(inst, scenario_load_factors(f, 5, seed=3))
    b = BatchSolver(inst.n, inst.c, inst.lb, inst.ub, inst.var_kind, *inst.flat(), b_scen=B, rho=100.0,
                    eps_rel=1e-4)
    bout = b.solve()
    b.close()
    srv = Server(rho=100.0, eps_rel=1e-4, iters_per_poll=128)
    ids = [srv.submit(*args, family=1), srv.submit(*args, family=2)]
    got = {}
    while len(got) < 2:
        for r in srv.poll(wait_ms=50):
            got[r["request_id"]] = r
    srv.close()
    L = _lines(path)
    kinds = [l["kind"] for l in L]
    assert kinds.count("solve") == 1 and kinds.count("fixed") == 1 and kinds.count("batch") == 1
    assert kinds.count("served") == 2 and len(L) == 5          # nothing from the allocation-free solve
    sv = [l for l in L if l["kind"] == "solve"][0]
    assert (sv["n"], sv["S"], sv["L"]) == (inst.n, inst.S, inst.L)
    assert sv["iterations"] == out["iterations"] and sv["status"] == out["status"] == 0
    assert sv["objective"] == out["objective"] and sv["pres"] == out["pres"] and sv["dres"] == out["dres"]
    assert sv["block_waves"] == info.block_waves and sv["kernel"] in ("step", "persistent", "tiled")
    assert sv["effective_gbs"] > 0 and sv["iters_per_s"] > 0
    step = sv["history_every"]
    assert len(sv["history"]) == -(-out["iterations"] // step) <= 64
    assert all(p > 0 and d >= 0 for p, d in sv["history"])
    fx = [l for l in L if l["kind"] == "fixed"][0]
    assert fx["iterations"] == 50
    bt = [l for l in L if l["kind"] == "batch"][0]
    assert bt["K"] == 5 and bt["converged"] == int(bout["converged"])
    assert bt["total_iterations"] == int(bout["total_iterations"])
    served = {l["request_id"]: l for l in L if l["kind"] == "served"}
    for i in ids:
        assert served[i]["iterations"] == got[i]["iterations"] and served[i]["status"] == got[i]["status"]
        assert served[i]["latency_ms"] == got[i]["latency_ms"]

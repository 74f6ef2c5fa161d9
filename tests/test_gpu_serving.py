"""Serving runtime: continuous batching of independent solves.

Checks: a solve returns the same bits alone and in a mix of other solves (and
the same bits as the single-instance step kernel with the same workgroup
shape); results match the FP64 oracle; admission respects the arena
footprint and rejects a solve larger than the arena; warm starts from the
resident state of the same family reduce iterations and keep the accuracy."""
import sys
import time

import numpy as np
import pytest

from opfgen import build_instance, by_name
from opfgen.serving import component_keys, make_family, reconfigure, with_loads
from oracle import admm

pytestmark = pytest.mark.gpu
RHO = 100.0


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _args(inst):
    return (inst.n, inst.c, inst.lb, inst.ub, inst.var_kind) + tuple(inst.flat())


def _drain(srv, ids, timeout_s=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(ids):
        for r in srv.poll(max_out=64, wait_ms=50):
            out[r["request_id"]] = r
        assert time.time() - t0 < timeout_s, f"only {len(out)} of {len(ids)} results"
    return out


@pytest.fixture(scope="module")
def mix():
    names = [("13bus", 0), ("13bus", 1), ("123bus", 0), ("13bus-zip", 0), ("123bus", 2), ("13bus", 2)]
    return [build_instance(by_name(n, s)) for n, s in names]


def test_alone_and_in_mix_give_identical_bits(mix):
    from paper_2501_08293_amd import Server, Solver
    _say("[gpu] serving: mix of 6 solves vs each alone vs single-instance step kernel")
    srv = Server(rho=RHO, eps_rel=1e-4, warm_start=False, iters_per_poll=32, arena_bytes=256 << 20)
    ids = [srv.submit(*_args(inst), family=k) for k, inst in enumerate(mix)]
    res = _drain(srv, ids)
    srv.close()
    for k, inst in enumerate(mix):
        r = res[ids[k]]
        assert r["status"] == 0
        alone = Server(rho=RHO, eps_rel=1e-4, warm_start=False, iters_per_poll=16, arena_bytes=64 << 20)
        rid = alone.submit(*_args(inst))
        ra = _drain(alone, [rid])[rid]
        alone.close()
        assert ra["iterations"] == r["iterations"]
        assert np.array_equal(ra["x"], r["x"])
        s = Solver(*_args(inst), rho=RHO, eps_rel=1e-4, kernel=1, block_waves=4)
        one = s.solve()
        s.close()
        assert one["iterations"] == r["iterations"] and np.array_equal(one["x"], r["x"])


def test_served_results_match_oracle(mix):
    from paper_2501_08293_amd import Server
    _say("[gpu] serving: results vs oracle")
    srv = Server(rho=RHO, eps_rel=1e-4, warm_start=False, iters_per_poll=32, arena_bytes=256 << 20)
    ids = [srv.submit(*_args(inst), family=k) for k, inst in enumerate(mix)]
    res = _drain(srv, ids)
    srv.close()
    for k, inst in enumerate(mix):
        ref = admm.solve(admm.setup(inst), rho=RHO, eps_rel=1e-4)
        r = res[ids[k]]
        assert abs(r["iterations"] - ref.iterations) <= 1
        assert abs(r["objective"] - ref.objective) <= 1e-6 * abs(ref.objective)
        vidx = np.nonzero(inst.var_kind == 2)[0]
        assert np.max(np.abs(r["x"][vidx] - ref.x[vidx])) <= 1e-6


def test_admission_by_footprint_and_rejection(mix):
    from paper_2501_08293_amd import Server
    _say("[gpu] serving: small arena admits one by one; oversize request rejected")
    srv = Server(rho=RHO, eps_rel=1e-4, warm_start=False, iters_per_poll=32, arena_bytes=3 << 20)
    big = build_instance(by_name("2500bus", 0))
    ids = [srv.submit(*_args(inst), family=k) for k, inst in enumerate(mix)]
    rid_big = srv.submit(*_args(big), family=99)
    res = _drain(srv, ids + [rid_big])
    st = srv.stats()
    srv.close()
    assert res[rid_big]["status"] == -5          # OPF_ENOMEM: footprint above the arena
    for rid in ids:
        assert res[rid]["status"] == 0
    assert st["arena_used"] == 0 and st["completed"] == len(ids) and st["rejected"] == 1


def test_warm_start_from_resident_family_state():
    from paper_2501_08293_amd import Server
    _say("[gpu] serving: warm start after a tie-switch reconfiguration and new loads")
    fam = make_family(5, 0, n_bus=150)
    rng = np.random.default_rng(3)
    base = build_instance(fam.base)
    nxt = build_instance(with_loads(reconfigure(fam, 0, rng), rng))
    srv = Server(rho=RHO, eps_rel=1e-5, warm_start=True, iters_per_poll=64, arena_bytes=64 << 20)
    r0 = srv.submit(*_args(base), family=5, comp_keys=component_keys(base))
    res0 = _drain(srv, [r0])[r0]
    r1 = srv.submit(*_args(nxt), family=5, comp_keys=component_keys(nxt))
    res1 = _drain(srv, [r1])[r1]
    srv.close()
    cold = Server(rho=RHO, eps_rel=1e-5, warm_start=False, iters_per_poll=64, arena_bytes=64 << 20)
    rc = cold.submit(*_args(nxt), family=5)
    resc = _drain(cold, [rc])[rc]
    cold.close()
    assert res0["status"] == 0 and res1["status"] == 0 and resc["status"] == 0
    assert res1["warm_components"] > 0.8 * nxt.S
    assert res1["iterations"] < resc["iterations"]
    _say(f"  warm {res1['iterations']} iterations ({res1['warm_components']}/{nxt.S} components) vs cold {resc['iterations']}")
    ref = admm.solve(admm.setup(nxt), rho=RHO, eps_rel=1e-8)
    assert abs(res1["objective"] - ref.objective) <= 2e-4 * abs(ref.objective)
    assert abs(resc["objective"] - ref.objective) <= 2e-4 * abs(ref.objective)

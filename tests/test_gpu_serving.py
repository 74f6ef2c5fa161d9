"""Serving runtime: continuous batching of independent solves.

Checks: a solve returns the same bits alone and in a mix of other solves (and
the same bits as the single-instance persistent solve with the same workgroup
shape), in FP64 and in mixed precision (FP32 bulk launch, FP64 polish launch),
also when some of its workgroups exceed the launch's LDS budget; results match
the FP64 oracle, also under admission limits that make solves queue for
either launch; admission respects the arena footprint and rejects a solve
larger than the arena; warm starts from the resident state of the same family
reduce iterations and keep the accuracy; bounded waits that run out end the
round's solves with OPF_EHANG and the device stays usable."""
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


def test_mixed_precision_serving_equals_single_instance_mixed(mix):
    """FP32 bulk phase in the FP32 launch, FP64 polish in the FP64 launch: each
    served solve returns the bits (iterations of both phases, x) of the
    single-instance mixed-precision persistent solve, in a mix and alone, with
    and without polish."""
    from paper_2501_08293_amd import OPF_PREC_MIXED, Server, Solver
    for polish in (True, False):
        _say(f"[gpu] serving mixed precision, polish={polish}: mix vs single-instance")
        srv = Server(rho=RHO, eps_rel=1e-4, warm_start=False, iters_per_poll=32, arena_bytes=256 << 20,
                     precision=OPF_PREC_MIXED, polish=polish)
        ids = [srv.submit(*_args(inst), family=k) for k, inst in enumerate(mix)]
        res = _drain(srv, ids)
        srv.close()
        for k, inst in enumerate(mix):
            r = res[ids[k]]
            s = Solver(*_args(inst), rho=RHO, eps_rel=1e-4, kernel=1, block_waves=4, precision=OPF_PREC_MIXED,
                       polish=polish)
            one = s.solve()
            s.close()
            assert r["status"] == 0 and one["status"] == 0
            assert r["iterations"] == one["iterations"] and r["iterations_fp32"] == one["iterations_fp32"]
            assert r["iterations_fp32"] > 0
            if not polish:
                assert r["iterations"] == r["iterations_fp32"]
            assert np.array_equal(r["x"], one["x"]), k
        srv = Server(rho=RHO, eps_rel=1e-4, warm_start=False, iters_per_poll=16, arena_bytes=64 << 20,
                     precision=OPF_PREC_MIXED, polish=polish)
        rid = srv.submit(*_args(mix[2]))
        ra = _drain(srv, [rid])[rid]
        srv.close()
        assert ra["iterations"] == res[ids[2]]["iterations"] and np.array_equal(ra["x"], res[ids[2]]["x"])


def test_mixed_precision_serving_matches_oracle_under_tight_admission(mix):
    """With room for a single 123-bus solve per launch, solves queue for the
    FP32 launch and for the FP64 polish launch; results keep the bits of the
    unconstrained mix and agree with the FP64 oracle to 1e-4 in the objective."""
    from paper_2501_08293_amd import OPF_PREC_MIXED, Server
    _say("[gpu] serving mixed precision, 16 workgroups per launch, vs oracle")
    kw = dict(rho=RHO, eps_rel=1e-4, warm_start=False, iters_per_poll=32, arena_bytes=256 << 20,
              precision=OPF_PREC_MIXED)
    srv = Server(max_workgroups=16, **kw)
    ids = [srv.submit(*_args(inst), family=k) for k, inst in enumerate(mix)]
    res = _drain(srv, ids)
    srv.close()
    free = Server(**kw)
    fids = [free.submit(*_args(inst), family=k) for k, inst in enumerate(mix)]
    fres = _drain(free, fids)
    free.close()
    for k, inst in enumerate(mix):
        r = res[ids[k]]
        assert r["status"] == 0
        assert r["iterations"] == fres[fids[k]]["iterations"] and np.array_equal(r["x"], fres[fids[k]]["x"])
        ref = admm.solve(admm.setup(inst), rho=RHO, eps_rel=1e-4)
        assert abs(r["objective"] - ref.objective) <= 1e-4 * abs(ref.objective)


def test_serving_bounded_wait_reports_ehang_and_recovers(mix):
    """A spin limit of one poll (forced from the host; every wait still ends)
    makes bounded waits run out: every solve of the round is answered with
    OPF_EHANG or a normal result, and a new server then solves normally."""
    from paper_2501_08293_amd import OPF_PREC_MIXED, Server
    _say("[gpu] serving forced wait timeout, mixed precision")
    srv = Server(rho=RHO, eps_rel=1e-4, warm_start=False, iters_per_poll=32, arena_bytes=256 << 20,
                 precision=OPF_PREC_MIXED, spin_limit=1)
    ids = [srv.submit(*_args(inst), family=k) for k, inst in enumerate(mix[:3])]
    res = _drain(srv, ids)
    srv.close()
    assert all(res[i]["status"] in (0, -8) for i in ids)
    srv = Server(rho=RHO, eps_rel=1e-4, warm_start=False, iters_per_poll=32, arena_bytes=256 << 20,
                 precision=OPF_PREC_MIXED)
    rid = srv.submit(*_args(mix[2]))
    r = _drain(srv, [rid])[rid]
    srv.close()
    assert r["status"] == 0


def test_workgroups_over_the_lds_budget_keep_the_bits():
    """A 254-bus feeder whose largest workgroups hold more factor columns (110)
    than the FP64 serving launch keeps in LDS (96): those workgroups read their
    factors from memory, the others from LDS, and the solve returns the bits of
    the single-instance persistent solve (all factors in LDS)."""
    from paper_2501_08293_amd import Server, Solver
    _say("[gpu] serving: per-workgroup LDS budget, 254-bus feeder, FP64")
    inst = build_instance(make_family(0, 0).base)
    srv = Server(rho=RHO, eps_rel=1e-3, warm_start=False, iters_per_poll=256, arena_bytes=256 << 20)
    rid = srv.submit(*_args(inst))
    r = _drain(srv, [rid])[rid]
    srv.close()
    s = Solver(*_args(inst), rho=RHO, eps_rel=1e-3, kernel=1, block_waves=4)
    one = s.solve()
    s.close()
    assert r["status"] == 0 and one["status"] == 0
    assert r["iterations"] == one["iterations"] and np.array_equal(r["x"], one["x"])


def test_mixed_precision_serving_stall_watch(mix):
    """eps_rel = 1e-9: the served bulk phase is ended by the stall watch at the
    same window boundary as in the single-instance solver, and the polish in
    the FP64 launch reaches 1e-9 with the bits of the single-instance mixed
    solve."""
    from paper_2501_08293_amd import OPF_PREC_MIXED, Server, Solver
    _say("[gpu] serving mixed precision at eps_rel 1e-9")
    srv = Server(rho=RHO, eps_rel=1e-9, warm_start=False, iters_per_poll=64, arena_bytes=64 << 20,
                 precision=OPF_PREC_MIXED)
    ids = [srv.submit(*_args(inst), family=k) for k, inst in enumerate(mix[:2])]
    res = _drain(srv, ids)
    srv.close()
    for k, inst in enumerate(mix[:2]):
        r = res[ids[k]]
        s = Solver(*_args(inst), rho=RHO, eps_rel=1e-9, kernel=1, block_waves=4, precision=OPF_PREC_MIXED)
        one = s.solve()
        s.close()
        assert r["status"] == 0 and 0 < r["iterations_fp32"] < r["iterations"]
        assert r["pres"] <= r["eps_prim"] and r["dres"] <= r["eps_dual"]
        assert r["iterations"] == one["iterations"] and r["iterations_fp32"] == one["iterations_fp32"]
        assert np.array_equal(r["x"], one["x"])


def test_warm_started_solve_alone_and_in_mix_give_identical_bits(mix):
    """A warm start draws on the resident state of its family; with that state
    fixed (the family's previous solve retired before the request arrives),
    the warm-started solve returns the same bits alone and in a mix of other
    solves, in mixed precision."""
    from paper_2501_08293_amd import OPF_PREC_MIXED, Server
    _say("[gpu] serving: warm-started solve alone vs in a mix of six (mixed precision)")
    fam = make_family(7, 0, n_bus=300)
    rng = np.random.default_rng(11)
    base = build_instance(fam.base)
    nxt = build_instance(with_loads(reconfigure(fam, 0, rng), rng))
    kw = dict(rho=RHO, eps_rel=1e-4, warm_start=True, iters_per_poll=64, arena_bytes=256 << 20,
              precision=OPF_PREC_MIXED)
    out = []
    for others in ([], mix):
        srv = Server(**kw)
        r0 = srv.submit(*_args(base), family=7, comp_keys=component_keys(base))
        _drain(srv, [r0])
        r1 = srv.submit(*_args(nxt), family=7, comp_keys=component_keys(nxt))
        ids = [srv.submit(*_args(inst), family=100 + k) for k, inst in enumerate(others)]
        res = _drain(srv, [r1] + ids)
        srv.close()
        assert all(res[i]["status"] == 0 for i in [r1] + ids)
        out.append(res[r1])
    alone, inmix = out
    assert alone["warm_components"] > 0 and alone["warm_components"] == inmix["warm_components"]
    assert alone["iterations"] == inmix["iterations"] and alone["iterations_fp32"] == inmix["iterations_fp32"]
    assert np.array_equal(alone["x"], inmix["x"])


def test_starvation_guard_admits_a_large_solve_ahead_of_later_small_ones():
    """Under a workgroup cap that holds the large solve only beside one small
    one, a stream of small requests would keep the capacity it needs taken;
    with the starvation guard (1 ms) the small requests that arrive after it
    are held back until it is admitted, and every request converges."""
    from paper_2501_08293_amd import Server
    small = [build_instance(by_name("13bus", s)) for s in range(3)]
    big = build_instance(by_name("123bus", 0))
    _say("[gpu] serving: starvation guard, 123bus among 45 13bus requests, max_workgroups 16")
    srv = Server(rho=RHO, eps_rel=1e-4, warm_start=False, iters_per_poll=64, arena_bytes=256 << 20,
                 max_workgroups=16, max_wait_ms=1)
    t_sub = {}
    ids = []
    for k in range(5):
        i = srv.submit(*_args(small[k % 3]), family=100 + k)
        t_sub[i] = time.perf_counter()
        ids.append(i)
    time.sleep(0.005)
    bid = srv.submit(*_args(big), family=1)
    t_sub[bid] = time.perf_counter()
    later = []
    for k in range(40):
        i = srv.submit(*_args(small[k % 3]), family=200 + k)
        t_sub[i] = time.perf_counter()
        later.append(i)
    res = _drain(srv, ids + [bid] + later)
    srv.close()
    assert all(r["status"] == 0 for r in res.values())
    admit = {i: t_sub[i] + res[i]["queue_ms"] * 1e-3 for i in res}
    after = sum(1 for i in later if admit[i] >= admit[bid] - 1e-3)
    _say(f"  large solve queued {res[bid]['queue_ms']:.1f} ms; {after} of 40 later small requests admitted after it")
    assert after >= 30


def test_cancel_queued_and_resident_requests():
    """A request waiting for admission is answered at once with OPF_ECANCELED;
    a resident one ends before the next round with its current iterate; the
    server keeps serving; unknown or answered ids are rejected."""
    from paper_2501_08293_amd import OpfError, Server
    from paper_2501_08293_amd.binding import OPF_ECANCELED, OPF_EINVAL
    big = build_instance(by_name("123bus", 0))
    small = build_instance(by_name("13bus", 0))
    _say("[gpu] serving: cancel a queued and a resident request (one slot)")
    srv = Server(rho=RHO, eps_rel=1e-12, max_iter=200_000, warm_start=False, iters_per_poll=64, max_slots=1,
                 arena_bytes=256 << 20)
    try:
        a = srv.submit(*_args(big), family=1)
        t0 = time.time()
        while srv.stats()["resident"] < 1:
            assert time.time() - t0 < 30
            time.sleep(0.005)
        b = srv.submit(*_args(small), family=2)
        time.sleep(0.05)                       # a few rounds of the resident solve; b is set up meanwhile
        srv.cancel(b)                          # still waiting for the only slot
        rb = _drain(srv, [b])[b]
        assert rb["status"] == OPF_ECANCELED and rb["iterations"] == 0
        srv.cancel(a)
        ra = _drain(srv, [a])[a]
        assert ra["status"] == OPF_ECANCELED
        assert ra["iterations"] > 0 and np.all(np.isfinite(ra["x"]))
        with pytest.raises(OpfError) as e:
            srv.cancel(a)                      # already answered
        assert e.value.code == OPF_EINVAL
        with pytest.raises(OpfError):
            srv.cancel(10 ** 9)                # never submitted
        c = srv.submit(*_args(small), family=3)
        rc = _drain(srv, [c])[c]
        assert rc["status"] in (0, 1) and rc["iterations"] > 0     # served as usual (eps 1e-12: to max_iter or converged)
    finally:
        srv.close()

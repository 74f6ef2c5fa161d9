"""The tiled persistent schedule (fewer co-resident workgroups than the
packing has workgroup tiles; each workgroup takes several tiles in turn every
iteration, state in memory) against the FP64 oracle and against the other
schedules.  Bars as for the other schedules: 1e-9 relative at fixed t in
FP64, the step and persistent schedules' iterates bit for bit, stop iteration
+-1 and objective 1e-6 at termination."""
import json
import os
import sys

import numpy as np
import pytest

from opfgen import build_instance, by_name
from oracle import admm

pytestmark = pytest.mark.gpu
RHO = 100.0
TILED, STEP, PERSIST = 3, 1, 2
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_cache = {}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _inst(name):
    if name not in _cache:
        _cache[name] = build_instance(by_name(name, 0))
    return _cache[name]


def _solver(inst, **kw):
    from paper_2501_08293_amd import Solver
    return Solver(inst.n, inst.c, inst.lb, inst.ub, inst.var_kind, *inst.flat(), **kw)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


def _tiles(info):
    return -(-info.waves // info.block_waves)


def _expect_pair(info, G):
    """The two-tile kernel runs when no workgroup would take more than two
    tiles (small problems: it fits the device)."""
    tiles = _tiles(info)
    return int(tiles >= 2 and (G == 0 or G >= -(-tiles // 2)))


@pytest.mark.parametrize("name,bw,G", [("13bus", 1, 1), ("123bus", 1, 0), ("123bus", 1, 3), ("123bus", 2, 2),
                                       ("13bus-zip", 1, 1)])
@pytest.mark.parametrize("t", [1, 3, 10, 100])
def test_tiled_iterates_match_oracle_fp64(name, bw, G, t):
    _say(f"[gpu] tiled schedule {name} block_waves={bw} workgroups={G or 'auto'} t={t} (FP64)")
    inst = _inst(name)
    ref = admm.solve(admm.setup(inst), rho=RHO, eps_rel=1e-4, fixed_iters=t)
    s = _solver(inst, rho=RHO, eps_rel=1e-4, kernel=TILED, block_waves=bw, tiled_workgroups=G)
    info = s.info()
    out = s.solve(fixed_iters=t)
    s.close()
    assert info.kernel == TILED
    assert info.tiled_pair == _expect_pair(info, G)
    assert out["iterations"] == t
    assert _rel(out["x"], ref.x) < 1e-9
    assert _rel(out["z"], ref.z) < 1e-9
    assert _rel(out["lam"], ref.lam) < 1e-9


@pytest.mark.parametrize("G", [0, 4])
def test_tiled_iterates_equal_persistent_and_step_bitwise(G):
    _say(f"[gpu] tiled = persistent = step bit for bit, 123bus, 300 iterations, workgroups={G or 'auto'}")
    inst = _inst("123bus")
    outs = {}
    for k in (TILED, PERSIST, STEP):
        s = _solver(inst, rho=RHO, eps_rel=1e-4, kernel=k, block_waves=2, tiled_workgroups=G)
        outs[k] = s.solve(fixed_iters=300)
        s.close()
    for k in (PERSIST, STEP):
        for f in ("x", "z", "lam"):
            assert np.array_equal(outs[TILED][f], outs[k][f]), (k, f)


@pytest.mark.parametrize("G", [0, 5])
def test_tiled_solve_matches_golden_fp64(G):
    g = json.load(open(os.path.join(GOLDEN, "admm_123bus_s0_eps0.0001.json")))
    _say(f"[gpu] tiled solve 123bus eps=1e-4 workgroups={G or 'auto'} vs golden (FP64)")
    s = _solver(_inst("123bus"), rho=RHO, eps_rel=1e-4, kernel=TILED, block_waves=1, tiled_workgroups=G)
    out = s.solve()
    s.close()
    assert out["status"] == 0
    assert abs(out["iterations"] - g["iterations"]) <= 1
    assert abs(out["objective"] - g["objective"]) <= 1e-6 * abs(g["objective"])
    assert np.max(np.abs(out["x"][g["w_index"]] - np.array(g["w_value"]))) <= 1e-6


def test_tiled_mixed_precision_matches_oracle():
    from paper_2501_08293_amd import OPF_PREC_MIXED
    g = json.load(open(os.path.join(GOLDEN, "admm_123bus_s0_eps0.0001.json")))
    _say("[gpu] tiled solve 123bus eps=1e-4 mixed precision, 3 workgroups vs golden")
    s = _solver(_inst("123bus"), rho=RHO, eps_rel=1e-4, kernel=TILED, block_waves=1, tiled_workgroups=3,
                precision=OPF_PREC_MIXED)
    out = s.solve()
    s.close()
    assert out["status"] == 0 and out["iterations_fp32"] > 0
    assert abs(out["objective"] - g["objective"]) <= 1e-4 * abs(g["objective"])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_tiled_21000bus_equals_step_schedule(prec):
    """The ~30k-component size, where the persistent grid does not fit: the
    automatic choice is the tiled schedule; its iterates after 50 iterations
    equal the step schedule's bit for bit."""
    from paper_2501_08293_amd import OPF_PREC_FP64, OPF_PREC_MIXED
    p = OPF_PREC_FP64 if prec == "fp64" else OPF_PREC_MIXED
    _say(f"[gpu] 21000bus tiled (auto) vs step, 50 iterations, {prec}")
    inst = _inst("21000bus")
    s = _solver(inst, rho=RHO, eps_rel=1e-4, precision=p)
    info = s.info()
    a = s.solve(fixed_iters=50)
    s.close()
    s = _solver(inst, rho=RHO, eps_rel=1e-4, precision=p, kernel=STEP)
    b = s.solve(fixed_iters=50)
    s.close()
    assert info.kernel == TILED
    _say(f"  tiled: {info.grid_blocks} workgroups, two-tile kernel {info.tiled_pair}")
    if prec == "mixed":
        assert info.tiled_pair == 1 and info.grid_blocks == -(-_tiles(info) // 2)
    for f in ("x", "z", "lam"):
        assert np.array_equal(a[f], b[f]), f


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_tiled_pair_odd_tile_count(prec):
    """The two-tile kernel on an odd number of tiles (the last workgroup
    holds one): iterates at t = 10 and 200 against the oracle (FP64, 1e-9) and
    equal to the step schedule's bit for bit."""
    from paper_2501_08293_amd import OPF_PREC_FP64, OPF_PREC_MIXED
    p = OPF_PREC_FP64 if prec == "fp64" else OPF_PREC_MIXED
    chosen = None
    for name in ("123bus", "13bus", "13bus-zip"):
        for bw in (1, 2, 4):
            s = _solver(_inst(name), rho=RHO, eps_rel=1e-4, kernel=TILED, block_waves=bw, precision=p)
            info = s.info()
            s.close()
            if _tiles(info) % 2 == 1 and _tiles(info) >= 3:
                chosen = (name, bw)
                break
        if chosen:
            break
    if chosen is None:
        pytest.skip("no test feeder packs into an odd number of at least three tiles")
    name, bw = chosen
    inst = _inst(name)
    for t in (10, 200):
        _say(f"[gpu] two-tile kernel, odd tile count: {name} block_waves={bw} t={t} ({prec})")
        s = _solver(inst, rho=RHO, eps_rel=1e-4, kernel=TILED, block_waves=bw, precision=p)
        info = s.info()
        a = s.solve(fixed_iters=t)
        s.close()
        assert info.tiled_pair == 1 and info.grid_blocks == (_tiles(info) + 1) // 2
        s = _solver(inst, rho=RHO, eps_rel=1e-4, kernel=STEP, block_waves=bw, precision=p)
        b = s.solve(fixed_iters=t)
        s.close()
        for f in ("x", "z", "lam"):
            assert np.array_equal(a[f], b[f]), (t, f)
        if prec == "fp64":
            ref = admm.solve(admm.setup(inst), rho=RHO, eps_rel=1e-4, fixed_iters=t)
            assert _rel(a["x"], ref.x) < 1e-9
            assert _rel(a["z"], ref.z) < 1e-9
            assert _rel(a["lam"], ref.lam) < 1e-9


def test_tiled_forced_wait_timeout_reports_ehang():
    """A spin limit of one poll (forced from the host; every wait still ends)
    ends the tiled launch with OPF_EHANG or a normal result, and the next
    solve on the device is normal."""
    _say("[gpu] tiled forced wait timeout 123bus")
    inst = _inst("123bus")
    s = _solver(inst, rho=RHO, eps_rel=1e-4, kernel=TILED, block_waves=1, tiled_workgroups=3, spin_limit=1)
    try:
        out = s.solve(raise_on_error=False)
        assert out["status"] in (0, -8)
    finally:
        s.close()
    s = _solver(inst, rho=RHO, eps_rel=1e-4, kernel=TILED, block_waves=1)
    out = s.solve()
    s.close()
    assert out["status"] == 0

"""Host-side set-up of the HIP library (validation, row reduction, factors,
packing into wavefronts and workgroups, copy and neighbour lists), compiled
with g++ and AddressSanitizer/UBSan and run on the CPU; the layout it builds is
checked against the problem and the oracle's factors."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from opfgen import build_instance, by_name
from oracle import admm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "tests", "native", "layout_driver.cpp"),
       os.path.join(ROOT, "paper_2501_08293_amd", "csrc", "setup.cpp")]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("drv") / "layout_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include")] + SRC + ["-o", out, "-lpthread"]
    subprocess.run(cmd, check=True)
    return out


def _write(path, inst, B):
    cm, cn, A, b, idx = inst.flat()
    with open(path, "wb") as f:
        np.array([inst.n, inst.S, B], np.int32).tofile(f)
        inst.c.astype(np.float64).tofile(f)
        inst.lb.astype(np.float64).tofile(f)
        inst.ub.astype(np.float64).tofile(f)
        inst.var_kind.astype(np.uint8).tofile(f)
        cm.tofile(f)
        cn.tofile(f)
        A.tofile(f)
        b.tofile(f)
        idx.tofile(f)


def _read(path):
    raw = open(path, "rb").read()
    hdr = np.frombuffer(raw[:32], np.int32)
    rc, n, S, L, W, G, B, maxnb = [int(v) for v in hdr]
    out = dict(rc=rc, n=n, S=S, L=L, W=W, G=G, B=B, max_nbrs=maxnb)
    if rc != 0:
        return out
    off = 32
    LP = W * 64

    def take(dt, cnt):
        nonlocal off
        a = np.frombuffer(raw[off:off + cnt * np.dtype(dt).itemsize], dt)
        off += cnt * np.dtype(dt).itemsize
        return a
    for k in ("var", "meta", "user_slot", "copy_start", "copy_cnt"):
        out[k] = take(np.int32, LP)
    out["copy_list"] = take(np.int32, L)
    out["wave_maxn"] = take(np.int32, W)
    out["wave_foff"] = take(np.int64, W)
    nf = int(out["wave_foff"][-1] + out["wave_maxn"][-1] * 64) if W else 0
    out["F"] = take(np.float64, nf)
    out["bbar"] = take(np.float64, LP)
    out["nbr_ptr"] = take(np.int32, G + 1)
    out["nbr_list"] = take(np.int32, int(out["nbr_ptr"][-1]))
    return out


@pytest.mark.parametrize("name,B", [("13bus", 4), ("13bus-zip", 1), ("123bus", 2), ("123bus", 8), ("2500bus", 4)])
def test_layout_invariants(driver, tmp_path, name, B):
    inst = build_instance(by_name(name, 0))
    fin = str(tmp_path / "in.bin")
    fout = str(tmp_path / "out.bin")
    _write(fin, inst, B)
    subprocess.run([driver, fin, fout], check=True)
    lay = _read(fout)
    assert lay["rc"] == 0
    W, G = lay["W"], lay["G"]
    assert W == G * B and lay["B"] == B
    var, meta, us = lay["var"], lay["meta"], lay["user_slot"]
    live = var >= 0
    # every user slot appears exactly once, on a lane copying the right variable
    assert np.array_equal(np.sort(us[live]), np.arange(inst.L))
    gidx = np.concatenate([c.idx for c in inst.comps])
    assert np.array_equal(var[live], gidx[us[live]])
    # components are contiguous inside one wavefront
    offs = np.concatenate([[0], np.cumsum([len(c.idx) for c in inst.comps])])
    P = admm.setup(inst)
    for s, comp in enumerate(inst.comps):
        d = np.nonzero(np.isin(us, np.arange(offs[s], offs[s + 1])))[0]
        assert len(d) == len(comp.idx)
        assert d.max() - d.min() == len(d) - 1 and d.min() // 64 == d.max() // 64
        base = d.min() % 64
        assert np.all(meta[d] & 255 == base) and np.all((meta[d] >> 8) & 255 == len(comp.idx))
        # packed factors equal I - P_s = -Abar_s of the oracle; bbar too
        w = d.min() // 64
        fo = lay["wave_foff"][w]
        for j, dj in enumerate(d):
            row = [lay["F"][fo + k * 64 + (dj % 64)] for k in range(len(comp.idx))]
            np.testing.assert_allclose(row, -P.Abar[s][j], atol=1e-11)
        np.testing.assert_allclose(lay["bbar"][d], P.bbar[s], atol=1e-11)
    # copy lists: all copies of the variable, ascending, one owner per variable
    cl = lay["copy_list"]
    for dd in np.nonzero(live)[0][:: max(1, live.sum() // 400)]:
        lst = cl[lay["copy_start"][dd]: lay["copy_start"][dd] + lay["copy_cnt"][dd]]
        assert np.all(np.diff(lst) > 0) and dd in lst and np.all(var[lst] == var[dd])
    owners = np.nonzero(live & ((meta >> 16) & 1 == 1))[0]
    assert np.array_equal(np.sort(var[owners]), np.arange(inst.n))
    # neighbour lists: symmetric, exclude self, cover every cross-workgroup copy
    nb = [set(lay["nbr_list"][lay["nbr_ptr"][b]: lay["nbr_ptr"][b + 1]].tolist()) for b in range(G)]
    for b in range(G):
        assert b not in nb[b]
        for c in nb[b]:
            assert b in nb[c]
    blk = np.arange(W * 64) // (B * 64)
    for i in range(0, inst.n, max(1, inst.n // 300)):
        ds = np.nonzero(var == i)[0]
        bs = set(blk[ds].tolist())
        for b1 in bs:
            assert (bs - {b1}) <= nb[b1]


def test_layout_rejects_bad_input(driver, tmp_path):
    inst = build_instance(by_name("13bus", 0))
    inst.lb[5] = inst.ub[5] + 1 if np.isfinite(inst.ub[5]) else 0.0
    inst.ub[5] = inst.lb[5] - 1
    fin = str(tmp_path / "in.bin")
    fout = str(tmp_path / "out.bin")
    _write(fin, inst, 4)
    subprocess.run([driver, fin, fout], check=True)
    assert _read(fout)["rc"] == -2

"""ORACLE -- test infrastructure only.

Algorithm 1 with the components split nearly evenly over worker processes,
the way the paper runs it on CPU cores (Section V: components distributed
almost evenly over the processors; the local updates run in parallel, the
global update and the termination test after they are gathered).  Only the
tests and the CPU baseline leg of the benchmark may use this module.

The arithmetic is that of oracle.admm, step for step: the master evaluates
the global update and the residuals with the same functions, each worker
evaluates the local and dual updates of its own components exactly as
admm.local_update / admm.dual_update do for them.  State lives in shared
memory, two buffers per array (iteration parity); two barriers per
iteration separate the master's and the workers' steps.
"""
from __future__ import annotations

import math
import multiprocessing as mp
import os
from multiprocessing import shared_memory

import numpy as np

from . import admm


def split_components(P: admm.Problem, parts: int):
    """Contiguous ranges of components with nearly equal work (sum of n_s^2,
    the local update's multiply-adds)."""
    w = np.array([len(ix) ** 2 for ix in P.idx], dtype=np.float64)
    cut = np.searchsorted(np.cumsum(w), np.linspace(0, w.sum(), parts + 1)[1:-1], side="right")
    bounds = [0] + [int(c) for c in cut] + [len(P.idx)]
    return [(bounds[k], bounds[k + 1]) for k in range(parts)]


def _worker_buckets(P: admm.Problem, lo: int, hi: int):
    """Components lo..hi-1 grouped by size, slots relative to the range."""
    by = {}
    for s in range(lo, hi):
        by.setdefault(len(P.idx[s]), []).append(s)
    base = int(P.offs[lo])
    out = []
    for k, ss in by.items():
        out.append((np.stack([P.Abar[s] for s in ss]), np.stack([P.offs[s] - base + np.arange(k) for s in ss])))
    return out


def _views(shm, L, n):
    buf = np.ndarray((2 * L + 2 * L + n + 2,), dtype=np.float64, buffer=shm.buf)
    z = [buf[0:L], buf[L:2 * L]]
    lam = [buf[2 * L:3 * L], buf[3 * L:4 * L]]
    x = buf[4 * L:4 * L + n]
    ctl = buf[4 * L + n:]              # [stop flag, rho]
    return z, lam, x, ctl


def _work(P, lo, hi, name, bar_x, bar_z):
    os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
    shm = shared_memory.SharedMemory(name=name)
    z, lam, x, ctl = _views(shm, P.L, P.n)
    buckets = _worker_buckets(P, lo, hi)
    sl = slice(int(P.offs[lo]), int(P.offs[hi]))
    g = P.gidx[sl]
    t = 0
    while True:
        bar_x.wait()                   # x of iteration t + 1 is ready (or stop)
        if ctl[0] != 0.0:
            break
        rho = ctl[1]
        src, dst = t & 1, (t + 1) & 1
        d = -rho * x[g] - lam[src][sl]
        zs = np.empty(len(g))
        for Ab, slots in buckets:
            zs[slots] = np.matmul(Ab, d[slots][:, :, None])[:, :, 0] / rho
        zs = zs + P.bbar_stacked[sl]
        z[dst][sl] = zs
        lam[dst][sl] = lam[src][sl] + rho * (x[g] - zs)
        t += 1
        bar_z.wait()
    del z, lam, x, ctl
    shm.close()


def solve_parallel(P: admm.Problem, procs: int, rho: float = 100.0, eps_rel: float = 1e-3,
                   max_iter: int = 1_000_000, fixed_iters: int | None = None):
    """Algorithm 1 on `procs` worker processes (fixed penalty).  Returns
    (x, z, lam, iterations, converged, (pres, dres, eps_prim, eps_dual))."""
    L, n = P.L, P.n
    shm = shared_memory.SharedMemory(create=True, size=8 * (4 * L + n + 2))
    ctx = mp.get_context("fork")
    bar_x = ctx.Barrier(procs + 1)
    bar_z = ctx.Barrier(procs + 1)
    z, lam, x, ctl = _views(shm, L, n)
    z0, l0 = admm.initial_point(P)
    z[0][:] = z0
    lam[0][:] = l0
    ctl[0] = 0.0
    ctl[1] = rho
    workers = [ctx.Process(target=_work, args=(P, lo, hi, shm.name, bar_x, bar_z), daemon=True)
               for lo, hi in split_components(P, procs)]
    for w in workers:
        w.start()
    limit = fixed_iters if fixed_iters is not None else max_iter
    t = 0
    converged = False
    r = (math.nan,) * 4
    try:
        while t < limit:
            src, dst = t & 1, (t + 1) & 1
            x[:] = admm.global_update(P, z[src], lam[src], rho)
            bar_x.wait()
            bar_z.wait()
            t += 1
            r = admm.residuals(P, x, z[dst], z[src], lam[dst], rho, eps_rel)
            if fixed_iters is None and r[0] <= r[2] and r[1] <= r[3]:
                converged = True
                break
        ctl[0] = 1.0
        bar_x.wait()
        for w in workers:
            w.join()
        out = (x.copy(), z[t & 1].copy(), lam[t & 1].copy(), t, converged, r)
    finally:
        for w in workers:
            if w.is_alive():
                w.terminate()
        del z, lam, x, ctl
        shm.close()
        shm.unlink()
    return out

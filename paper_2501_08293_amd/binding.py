"""Python binding of the C ABI in include/opf_admm.h (argument marshalling only).

Every step of the iteration runs in the HIP library `libopf_admm.so`; this
module only converts arrays and structs.  Importing it fails loudly when the
library has not been built; there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libopf_admm.so")

OPF_OK = 0
OPF_NOT_CONVERGED = 1
OPF_EINVAL = -1
OPF_EBOUNDS = -2
OPF_EUNCOVERED = -3
OPF_EINFEASIBLE_COMPONENT = -4
OPF_ENOMEM = -5
OPF_EHIP = -6
OPF_ENUMERIC = -7
OPF_EHANG = -8
OPF_ECANCELED = -9
OPF_STALLED = 2

OPF_PREC_FP64 = 0
OPF_PREC_MIXED = 1

OPF_KERNEL_AUTO = 0
OPF_KERNEL_STEP = 1
OPF_KERNEL_PERSISTENT = 2
OPF_KERNEL_TILED = 3

OPF_RHO_RELATIVE = 0
OPF_RHO_PLAIN = 1
OPF_RHO_LAG = 4

OPF_ADMIT_LARGEST_FIRST = 0
OPF_ADMIT_ARRIVAL = 1

STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", 2: "STALLED", -1: "EINVAL", -2: "EBOUNDS", -3: "EUNCOVERED",
                -4: "EINFEASIBLE_COMPONENT", -5: "ENOMEM", -6: "EHIP", -7: "ENUMERIC", -8: "EHANG",
                -9: "ECANCELED"}

EXPORTED = ["opf_admm_default_options", "opf_admm_setup", "opf_admm_solve", "opf_admm_run_fixed",
            "opf_admm_solve_noalloc",
            "opf_admm_residuals", "opf_admm_get_info", "opf_admm_destroy", "opf_admm_last_error",
            "opf_admm_setup_batch", "opf_admm_setup_batch_ex", "opf_admm_solve_batch", "opf_admm_batch_info", "opf_admm_destroy_batch",
            "opf_admm_batch_last_error", "opf_server_default_options", "opf_server_create", "opf_server_submit", "opf_server_cancel",
            "opf_server_poll", "opf_server_get_stats", "opf_server_destroy", "opf_server_last_error"]


class opf_problem(C.Structure):
    _fields_ = [("n", C.c_int32), ("c", C.POINTER(C.c_double)), ("lb", C.POINTER(C.c_double)),
                ("ub", C.POINTER(C.c_double)), ("var_kind", C.POINTER(C.c_uint8)), ("S", C.c_int32),
                ("comp_m", C.POINTER(C.c_int32)), ("comp_n", C.POINTER(C.c_int32)),
                ("A_vals", C.POINTER(C.c_double)), ("b_vals", C.POINTER(C.c_double)),
                ("idx", C.POINTER(C.c_int32))]


class opf_admm_options(C.Structure):
    _fields_ = [("rho", C.c_double), ("eps_rel", C.c_double), ("max_iter", C.c_int64),
                ("precision", C.c_int32), ("polish", C.c_int32), ("check_every", C.c_int32),
                ("kernel", C.c_int32), ("history_cap", C.c_int32), ("block_waves", C.c_int32),
                ("spin_limit", C.c_int32), ("split_terms", C.c_int32), ("autotune", C.c_int32),
                ("workgroup_order", C.c_int32), ("setup_on_device", C.c_int32), ("rho_every", C.c_int32),
                ("rho_mode", C.c_int32), ("rho_mu", C.c_double), ("rho_tau", C.c_double), ("rho_min", C.c_double),
                ("rho_max", C.c_double), ("local_updates", C.c_int32), ("tiled_workgroups", C.c_int32),
                ("stall_window", C.c_int64), ("stall_delta", C.c_double), ("stall_checks", C.c_int32),
                ("reserved_stall", C.c_int32)]


class opf_warm(C.Structure):
    _fields_ = [("z", C.c_void_p), ("lam", C.c_void_p), ("on_device", C.c_int32)]


class opf_result(C.Structure):
    _fields_ = [("x", C.c_void_p), ("z", C.c_void_p), ("lam", C.c_void_p), ("outputs_on_device", C.c_int32),
                ("status", C.c_int32), ("iterations", C.c_int64), ("iterations_fp32", C.c_int64),
                ("objective", C.c_double), ("pres", C.c_double), ("dres", C.c_double),
                ("eps_prim", C.c_double), ("eps_dual", C.c_double), ("solve_ms", C.c_double),
                ("kernel_ms", C.c_double), ("kernel_ms_fp32", C.c_double), ("kernel_launches", C.c_int64),
                ("rho_final", C.c_double)]


class opf_residuals(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("pres", C.c_double), ("dres", C.c_double),
                ("eps_prim", C.c_double), ("eps_dual", C.c_double)]


class opf_admm_info(C.Structure):
    _fields_ = [("n", C.c_int32), ("S", C.c_int32), ("L", C.c_int32), ("waves", C.c_int32),
                ("lanes", C.c_int32), ("max_ns", C.c_int32), ("max_copies", C.c_int32),
                ("sum_ns2", C.c_int64), ("factor_bytes_fp64", C.c_int64), ("device_bytes", C.c_int64),
                ("setup_ms", C.c_double), ("grid_blocks", C.c_int32), ("block_waves", C.c_int32),
                ("kernel", C.c_int32), ("persistent_capacity", C.c_int32), ("max_neighbours", C.c_int32),
                ("factors_in_lds", C.c_int32), ("batch_order", C.c_int32), ("tiled_pair", C.c_int32),
                ("batch_groups", C.c_int32), ("fp64_lds_workgroups", C.c_int32)]


class opf_batch_result(C.Structure):
    _fields_ = [("x", C.c_void_p), ("outputs_on_device", C.c_int32), ("reserved0", C.c_int32),
                ("iterations", C.POINTER(C.c_int64)), ("objective", C.POINTER(C.c_double)),
                ("status", C.POINTER(C.c_int32)), ("pres", C.POINTER(C.c_double)), ("dres", C.POINTER(C.c_double)),
                ("eps_prim", C.POINTER(C.c_double)), ("eps_dual", C.POINTER(C.c_double)),
                ("total_iterations", C.c_int64), ("converged", C.c_int32), ("reserved1", C.c_int32),
                ("solve_ms", C.c_double)]


class opf_server_options(C.Structure):
    _fields_ = [("admm", opf_admm_options), ("arena_bytes", C.c_int64), ("warm_bytes", C.c_int64),
                ("max_slots", C.c_int32), ("max_workgroups", C.c_int32), ("iters_per_poll", C.c_int32),
                ("setup_threads", C.c_int32), ("warm_start", C.c_int32), ("admission", C.c_int32),
                ("max_wait_ms", C.c_int32), ("reserved", C.c_int32 * 3)]


class opf_served(C.Structure):
    _fields_ = [("request_id", C.c_int64), ("status", C.c_int32), ("warm_components", C.c_int32),
                ("iterations", C.c_int64), ("objective", C.c_double), ("pres", C.c_double),
                ("dres", C.c_double), ("eps_prim", C.c_double), ("eps_dual", C.c_double),
                ("queue_ms", C.c_double), ("latency_ms", C.c_double), ("x", C.c_void_p),
                ("iterations_fp32", C.c_int64)]


class opf_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64),
                ("resident", C.c_int32), ("queued", C.c_int32), ("arena_used", C.c_int64),
                ("arena_bytes", C.c_int64), ("warm_used", C.c_int64), ("launches", C.c_int64),
                ("busy_ms", C.c_double)]


_lib = None

# Handles still open when the interpreter exits are closed by an exit hook that
# runs before the HIP runtime and any profiler attached to it shut down; a
# handle's __del__ makes no HIP call while the interpreter is finalizing.
_live = weakref.WeakSet()


def close_all() -> None:
    """Closes every open Solver, BatchSolver and Server of this process."""
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass


atexit.register(close_all)


def load(path: str = LIB_PATH):
    """Loads the HIP library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run python -m paper_2501_08293_amd.build)")
    # PyTorch ships its own HIP runtime under the same soname; loading PyTorch
    # first makes the library bind to that one, so the process holds a single
    # HIP runtime whose device memory and streams both sides share.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    H = C.c_void_p
    lib.opf_admm_default_options.argtypes = [C.POINTER(opf_admm_options)]
    lib.opf_admm_default_options.restype = None
    lib.opf_admm_setup.argtypes = [C.POINTER(opf_problem), C.POINTER(opf_admm_options), C.c_void_p, C.POINTER(H)]
    lib.opf_admm_setup.restype = C.c_int
    lib.opf_admm_solve.argtypes = [H, C.POINTER(opf_warm), C.POINTER(opf_result)]
    lib.opf_admm_solve.restype = C.c_int
    lib.opf_admm_run_fixed.argtypes = [H, C.POINTER(opf_warm), C.c_int64, C.POINTER(opf_result)]
    lib.opf_admm_run_fixed.restype = C.c_int
    lib.opf_admm_solve_noalloc.argtypes = [H, C.POINTER(opf_warm), C.POINTER(opf_result)]
    lib.opf_admm_solve_noalloc.restype = C.c_int
    lib.opf_admm_residuals.argtypes = [H, C.POINTER(opf_residuals), C.POINTER(C.c_double), C.c_int]
    lib.opf_admm_residuals.restype = C.c_int
    lib.opf_admm_get_info.argtypes = [H, C.POINTER(opf_admm_info)]
    lib.opf_admm_get_info.restype = C.c_int
    lib.opf_admm_destroy.argtypes = [H]
    lib.opf_admm_destroy.restype = None
    lib.opf_admm_last_error.argtypes = [H]
    lib.opf_admm_last_error.restype = C.c_char_p
    lib.opf_admm_setup_batch.argtypes = [C.POINTER(opf_problem), C.POINTER(C.c_double), C.c_int32,
                                         C.POINTER(opf_admm_options), C.c_void_p, C.POINTER(H)]
    lib.opf_admm_setup_batch.restype = C.c_int
    lib.opf_admm_setup_batch_ex.argtypes = [C.POINTER(opf_problem), C.POINTER(C.c_double), C.c_int32, C.c_int64,
                                            C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                            C.POINTER(opf_admm_options), C.c_void_p, C.POINTER(H)]
    lib.opf_admm_setup_batch_ex.restype = C.c_int
    lib.opf_admm_solve_batch.argtypes = [H, C.POINTER(opf_batch_result)]
    lib.opf_admm_solve_batch.restype = C.c_int
    lib.opf_admm_batch_info.argtypes = [H, C.POINTER(opf_admm_info)]
    lib.opf_admm_batch_info.restype = C.c_int
    lib.opf_admm_destroy_batch.argtypes = [H]
    lib.opf_admm_destroy_batch.restype = None
    lib.opf_admm_batch_last_error.argtypes = [H]
    lib.opf_admm_batch_last_error.restype = C.c_char_p
    lib.opf_server_default_options.argtypes = [C.POINTER(opf_server_options)]
    lib.opf_server_default_options.restype = None
    lib.opf_server_create.argtypes = [C.POINTER(opf_server_options), C.c_void_p, C.POINTER(H)]
    lib.opf_server_create.restype = C.c_int
    lib.opf_server_submit.argtypes = [H, C.POINTER(opf_problem), C.c_uint64, C.POINTER(C.c_uint64),
                                      C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.opf_server_submit.restype = C.c_int
    lib.opf_server_poll.argtypes = [H, C.POINTER(opf_served), C.c_int, C.c_int]
    lib.opf_server_poll.restype = C.c_int
    lib.opf_server_cancel.argtypes = [H, C.c_int64]
    lib.opf_server_cancel.restype = C.c_int
    lib.opf_server_get_stats.argtypes = [H, C.POINTER(opf_server_stats)]
    lib.opf_server_get_stats.restype = C.c_int
    lib.opf_server_destroy.argtypes = [H]
    lib.opf_server_destroy.restype = None
    lib.opf_server_last_error.argtypes = [H]
    lib.opf_server_last_error.restype = C.c_char_p
    _lib = lib
    return lib


class OpfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _dev_ptr(t):
    """Device pointer of a torch tensor (or an int address)."""
    if isinstance(t, int):
        return t
    return int(t.data_ptr())


# ---- thin wrappers with the C names ------------------------------------------

def opf_admm_default_options() -> opf_admm_options:
    o = opf_admm_options()
    load().opf_admm_default_options(C.byref(o))
    return o


def opf_admm_setup(problem: opf_problem, options: opf_admm_options, stream: int = 0):
    lib = load()
    h = C.c_void_p()
    rc = lib.opf_admm_setup(C.byref(problem), C.byref(options), C.c_void_p(stream or None), C.byref(h))
    if rc != OPF_OK:
        raise OpfError(rc, lib.opf_admm_last_error(None).decode())
    return h


def opf_admm_solve(h, warm, result: opf_result) -> int:
    return load().opf_admm_solve(h, C.byref(warm) if warm is not None else None, C.byref(result))


def opf_admm_solve_noalloc(h, warm, result: opf_result) -> int:
    return load().opf_admm_solve_noalloc(h, C.byref(warm) if warm is not None else None, C.byref(result))


def opf_admm_run_fixed(h, warm, iters: int, result: opf_result) -> int:
    return load().opf_admm_run_fixed(h, C.byref(warm) if warm is not None else None, int(iters), C.byref(result))


def opf_admm_residuals(h, hist_cap: int = 0):
    res = opf_residuals()
    hist = np.zeros((max(hist_cap, 1), 4))
    rows = load().opf_admm_residuals(h, C.byref(res), _ptr(hist, C.c_double) if hist_cap else None, hist_cap)
    if rows < 0:
        raise OpfError(rows, load().opf_admm_last_error(h).decode())
    return res, hist[:rows]


def opf_admm_get_info(h) -> opf_admm_info:
    info = opf_admm_info()
    load().opf_admm_get_info(h, C.byref(info))
    return info


def opf_admm_destroy(h) -> None:
    load().opf_admm_destroy(h)


def opf_admm_last_error(h=None) -> str:
    return load().opf_admm_last_error(h).decode()


def opf_admm_setup_batch(problem: opf_problem, b_scen: np.ndarray, options: opf_admm_options, stream: int = 0,
                         a_pos=None, a_scen=None):
    lib = load()
    h = C.c_void_p()
    b = np.ascontiguousarray(b_scen, np.float64)
    if a_pos is None:
        rc = lib.opf_admm_setup_batch(C.byref(problem), _ptr(b, C.c_double), int(b.shape[0]), C.byref(options),
                                      C.c_void_p(stream or None), C.byref(h))
    else:
        pos = np.ascontiguousarray(a_pos, np.int64)
        val = np.ascontiguousarray(a_scen, np.float64)
        if val.shape != (b.shape[0], pos.shape[0]):
            raise ValueError("a_scen must be [K, len(a_pos)]")
        rc = lib.opf_admm_setup_batch_ex(C.byref(problem), _ptr(b, C.c_double), int(b.shape[0]), int(pos.shape[0]),
                                         _ptr(pos, C.c_int64), _ptr(val, C.c_double), C.byref(options),
                                         C.c_void_p(stream or None), C.byref(h))
    if rc != OPF_OK:
        raise OpfError(rc, lib.opf_admm_batch_last_error(None).decode())
    return h


def opf_admm_solve_batch(h, result: opf_batch_result) -> int:
    return load().opf_admm_solve_batch(h, C.byref(result))


def opf_admm_batch_info(h) -> opf_admm_info:
    info = opf_admm_info()
    load().opf_admm_batch_info(h, C.byref(info))
    return info


def opf_admm_destroy_batch(h) -> None:
    load().opf_admm_destroy_batch(h)


def opf_admm_batch_last_error(h=None) -> str:
    return load().opf_admm_batch_last_error(h).decode()


# ---- convenience object ---------------------------------------------------------


def _problem(keep, n):
    return opf_problem(n=int(n), c=_ptr(keep["c"], C.c_double), lb=_ptr(keep["lb"], C.c_double),
                       ub=_ptr(keep["ub"], C.c_double), var_kind=_ptr(keep["var_kind"], C.c_uint8),
                       S=len(keep["comp_m"]), comp_m=_ptr(keep["comp_m"], C.c_int32),
                       comp_n=_ptr(keep["comp_n"], C.c_int32), A_vals=_ptr(keep["A"], C.c_double),
                       b_vals=_ptr(keep["b"], C.c_double), idx=_ptr(keep["idx"], C.c_int32))


def _keep(c, lb, ub, var_kind, comp_m, comp_n, A_vals, b_vals, idx):
    return dict(c=np.ascontiguousarray(c, np.float64), lb=np.ascontiguousarray(lb, np.float64),
                ub=np.ascontiguousarray(ub, np.float64), var_kind=np.ascontiguousarray(var_kind, np.uint8),
                comp_m=np.ascontiguousarray(comp_m, np.int32), comp_n=np.ascontiguousarray(comp_n, np.int32),
                A=np.ascontiguousarray(A_vals, np.float64), b=np.ascontiguousarray(b_vals, np.float64),
                idx=np.ascontiguousarray(idx, np.int32))


class BatchSolver:
    """Owns one batched handle: K right-hand sides b_scen[K, sum m_s] on the
    topology and A_s of the given problem arrays."""

    def __init__(self, n, c, lb, ub, var_kind, comp_m, comp_n, A_vals, b_vals, idx, b_scen, *, rho=100.0,
                 eps_rel=1e-4, max_iter=1_000_000, check_every=64, split_terms=3, stream=0, a_pos=None,
                 a_scen=None, autotune=False):
        keep = _keep(c, lb, ub, var_kind, comp_m, comp_n, A_vals, b_vals, idx)
        self.n = int(n)
        self.K = int(np.asarray(b_scen).shape[0])
        o = opf_admm_default_options()
        o.rho = rho
        o.eps_rel = eps_rel
        o.max_iter = max_iter
        o.check_every = check_every
        o.split_terms = split_terms
        o.autotune = int(bool(autotune))
        self.h = opf_admm_setup_batch(_problem(keep, n), b_scen, o, stream, a_pos=a_pos, a_scen=a_scen)
        _live.add(self)

    def close(self):
        if getattr(self, "h", None):
            opf_admm_destroy_batch(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # the default argument keeps the check callable after module teardown
        # has cleared this module's globals
        if getattr(self, "h", None) is None or _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> opf_admm_info:
        return opf_admm_batch_info(self.h)

    def solve(self, x=None, raise_on_error=True):
        K, n = self.K, self.n
        r = opf_batch_result()
        if x is None:
            x = np.zeros((K, n))
        dev = not isinstance(x, np.ndarray)
        r.outputs_on_device = int(dev)
        r.x = _dev_ptr(x) if dev else x.ctypes.data
        it = np.zeros(K, np.int64)
        obj = np.zeros(K)
        st = np.zeros(K, np.int32)
        pres = np.zeros(K)
        dres = np.zeros(K)
        ep = np.zeros(K)
        ed = np.zeros(K)
        r.iterations = _ptr(it, C.c_int64)
        r.objective = _ptr(obj, C.c_double)
        r.status = _ptr(st, C.c_int32)
        r.pres = _ptr(pres, C.c_double)
        r.dres = _ptr(dres, C.c_double)
        r.eps_prim = _ptr(ep, C.c_double)
        r.eps_dual = _ptr(ed, C.c_double)
        rc = opf_admm_solve_batch(self.h, r)
        if rc < 0 and raise_on_error:
            raise OpfError(rc, opf_admm_batch_last_error(self.h))
        return dict(status=rc, x=x, iterations=it, objective=obj, scenario_status=st, pres=pres, dres=dres,
                    eps_prim=ep, eps_dual=ed, total_iterations=r.total_iterations, converged=r.converged,
                    solve_ms=r.solve_ms)


class Solver:
    """Owns one handle.  Arrays are those of the opf_problem struct (the
    componentwise LP of the paper's reformulated model)."""

    def __init__(self, n, c, lb, ub, var_kind, comp_m, comp_n, A_vals, b_vals, idx, *, rho=100.0,
                 eps_rel=1e-3, max_iter=1_000_000, precision=OPF_PREC_FP64, polish=True, check_every=256,
                 kernel=OPF_KERNEL_AUTO, history_cap=0, block_waves=0, spin_limit=0, autotune=False,
                 workgroup_order=0, setup_on_device=False, rho_every=0, rho_mode=OPF_RHO_RELATIVE, rho_mu=0.0,
                 rho_tau=0.0, rho_min=0.0, rho_max=0.0, local_updates=1, tiled_workgroups=0, stall_window=0,
                 stall_checks=0, stall_delta=0.0, stream=0):
        self._keep = dict(
            c=np.ascontiguousarray(c, np.float64), lb=np.ascontiguousarray(lb, np.float64),
            ub=np.ascontiguousarray(ub, np.float64), var_kind=np.ascontiguousarray(var_kind, np.uint8),
            comp_m=np.ascontiguousarray(comp_m, np.int32), comp_n=np.ascontiguousarray(comp_n, np.int32),
            A=np.ascontiguousarray(A_vals, np.float64), b=np.ascontiguousarray(b_vals, np.float64),
            idx=np.ascontiguousarray(idx, np.int32))
        k = self._keep
        self.n = int(n)
        self.L = int(k["comp_n"].sum())
        p = opf_problem(n=self.n, c=_ptr(k["c"], C.c_double), lb=_ptr(k["lb"], C.c_double),
                        ub=_ptr(k["ub"], C.c_double), var_kind=_ptr(k["var_kind"], C.c_uint8),
                        S=len(k["comp_m"]), comp_m=_ptr(k["comp_m"], C.c_int32),
                        comp_n=_ptr(k["comp_n"], C.c_int32), A_vals=_ptr(k["A"], C.c_double),
                        b_vals=_ptr(k["b"], C.c_double), idx=_ptr(k["idx"], C.c_int32))
        o = opf_admm_default_options()
        o.rho = rho
        o.eps_rel = eps_rel
        o.max_iter = max_iter
        o.precision = precision
        o.polish = int(bool(polish))
        o.check_every = check_every
        o.kernel = kernel
        o.history_cap = history_cap
        o.block_waves = block_waves
        o.spin_limit = spin_limit
        o.autotune = int(bool(autotune))
        o.workgroup_order = workgroup_order
        o.setup_on_device = int(bool(setup_on_device))
        o.rho_every = rho_every
        o.rho_mode = rho_mode
        o.rho_mu = rho_mu
        o.rho_tau = rho_tau
        o.rho_min = rho_min
        o.rho_max = rho_max
        o.local_updates = local_updates
        o.tiled_workgroups = tiled_workgroups
        o.stall_window = stall_window
        o.stall_checks = stall_checks
        o.stall_delta = stall_delta
        self.options = o
        self.h = opf_admm_setup(p, o, stream)
        self._keep = None   # the library copied everything it needs
        _live.add(self)

    @classmethod
    def from_arrays(cls, flat, **kw):
        return cls(*flat, **kw)

    def close(self):
        if getattr(self, "h", None):
            opf_admm_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # the default argument keeps the check callable after module teardown
        # has cleared this module's globals
        if getattr(self, "h", None) is None or _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> opf_admm_info:
        return opf_admm_get_info(self.h)

    def _result(self, x, z, lam):
        r = opf_result()
        dev = not isinstance(x, np.ndarray)
        r.outputs_on_device = int(dev)
        if dev:
            r.x = _dev_ptr(x)
            r.z = _dev_ptr(z) if z is not None else None
            r.lam = _dev_ptr(lam) if lam is not None else None
        else:
            r.x = x.ctypes.data
            r.z = z.ctypes.data if z is not None else None
            r.lam = lam.ctypes.data if lam is not None else None
        return r

    def _warm(self, z0, lam0):
        if z0 is None:
            return None
        w = opf_warm()
        if isinstance(z0, np.ndarray):
            self._warm_keep = (np.ascontiguousarray(z0, np.float64), np.ascontiguousarray(lam0, np.float64))
            w.z = self._warm_keep[0].ctypes.data
            w.lam = self._warm_keep[1].ctypes.data
            w.on_device = 0
        else:
            w.z = _dev_ptr(z0)
            w.lam = _dev_ptr(lam0)
            w.on_device = 1
        return w

    def solve(self, x=None, z=None, lam=None, z0=None, lam0=None, fixed_iters=None, raise_on_error=True,
              noalloc=False):
        """Runs Algorithm 1.  Outputs go to the given arrays (numpy = host,
        torch CUDA tensors = device); by default new host arrays are returned.
        noalloc: through opf_admm_solve_noalloc (kernel scratch in the
        library's static device array; not with fixed_iters)."""
        if x is None:
            x = np.zeros(self.n)
            z = np.zeros(self.L) if z is None else z
            lam = np.zeros(self.L) if lam is None else lam
        r = self._result(x, z, lam)
        w = self._warm(z0, lam0)
        if noalloc:
            if fixed_iters is not None:
                raise ValueError("the allocation-free solve runs to the termination test")
            rc = opf_admm_solve_noalloc(self.h, w, r)
        elif fixed_iters is None:
            rc = opf_admm_solve(self.h, w, r)
        else:
            rc = opf_admm_run_fixed(self.h, w, fixed_iters, r)
        if rc < 0 and raise_on_error:
            raise OpfError(rc, opf_admm_last_error(self.h))
        return dict(status=rc, x=x, z=z, lam=lam, iterations=r.iterations, iterations_fp32=r.iterations_fp32,
                    objective=r.objective, pres=r.pres, dres=r.dres, eps_prim=r.eps_prim, eps_dual=r.eps_dual,
                    solve_ms=r.solve_ms, kernel_ms=r.kernel_ms, kernel_ms_fp32=r.kernel_ms_fp32,
                    kernel_launches=r.kernel_launches, rho_final=r.rho_final)

    def residuals(self, hist_cap=0):
        return opf_admm_residuals(self.h, hist_cap)


# ---- serving runtime ----------------------------------------------------------------

def opf_server_default_options() -> opf_server_options:
    o = opf_server_options()
    load().opf_server_default_options(C.byref(o))
    return o


class Server:
    """Owns one serving runtime.  submit() copies the problem arrays; the x
    output buffer of each request is kept alive here until its result is
    polled."""

    def __init__(self, *, rho=100.0, eps_rel=1e-4, max_iter=1_000_000, arena_bytes=4 << 30, warm_bytes=1 << 30,
                 max_slots=256, max_workgroups=8192, iters_per_poll=256, setup_threads=4, warm_start=True,
                 precision=OPF_PREC_FP64, polish=True, spin_limit=0, admission=None, max_wait_ms=None,
                 stream=0):
        lib = load()
        o = opf_server_default_options()
        o.admm.rho = rho
        o.admm.eps_rel = eps_rel
        o.admm.max_iter = max_iter
        o.admm.precision = precision
        o.admm.polish = int(bool(polish))
        o.admm.spin_limit = int(spin_limit)
        o.arena_bytes = int(arena_bytes)
        o.warm_bytes = int(warm_bytes)
        o.max_slots = max_slots
        o.max_workgroups = max_workgroups
        o.iters_per_poll = iters_per_poll
        o.setup_threads = setup_threads
        o.warm_start = int(bool(warm_start))
        if admission is not None:
            o.admission = int(admission)
        if max_wait_ms is not None:
            o.max_wait_ms = int(max_wait_ms)
        h = C.c_void_p()
        rc = lib.opf_server_create(C.byref(o), C.c_void_p(stream or None), C.byref(h))
        if rc != OPF_OK:
            raise OpfError(rc, lib.opf_server_last_error(None).decode())
        self.h = h
        self._pending = {}
        _live.add(self)

    def submit(self, n, c, lb, ub, var_kind, comp_m, comp_n, A_vals, b_vals, idx, family=0, comp_keys=None) -> int:
        keep = _keep(c, lb, ub, var_kind, comp_m, comp_n, A_vals, b_vals, idx)
        x = np.zeros(int(n))
        keys = None if comp_keys is None else np.ascontiguousarray(comp_keys, np.uint64)
        rid = C.c_int64()
        rc = load().opf_server_submit(self.h, C.byref(_problem(keep, n)), C.c_uint64(family),
                                      _ptr(keys, C.c_uint64) if keys is not None else None,
                                      _ptr(x, C.c_double), C.byref(rid))
        if rc != OPF_OK:
            raise OpfError(rc, load().opf_server_last_error(self.h).decode())
        self._pending[rid.value] = x
        return rid.value

    def cancel(self, request_id) -> None:
        """Cancels an unanswered request; its result (status OPF_ECANCELED) comes through poll."""
        rc = load().opf_server_cancel(self.h, C.c_int64(int(request_id)))
        if rc != OPF_OK:
            raise OpfError(rc, load().opf_server_last_error(self.h).decode())

    def poll(self, max_out=64, wait_ms=0):
        buf = (opf_served * max_out)()
        k = load().opf_server_poll(self.h, buf, max_out, int(wait_ms))
        out = []
        for i in range(max(k, 0)):
            r = buf[i]
            out.append(dict(request_id=r.request_id, status=r.status, warm_components=r.warm_components,
                            iterations=r.iterations, iterations_fp32=r.iterations_fp32,
                            objective=r.objective, pres=r.pres, dres=r.dres,
                            eps_prim=r.eps_prim, eps_dual=r.eps_dual, queue_ms=r.queue_ms,
                            latency_ms=r.latency_ms, x=self._pending.pop(r.request_id, None)))
        return out

    def stats(self):
        st = opf_server_stats()
        load().opf_server_get_stats(self.h, C.byref(st))
        return {k: getattr(st, k) for k, _ in opf_server_stats._fields_}

    def close(self):
        if getattr(self, "h", None):
            load().opf_server_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # the default argument keeps the check callable after module teardown
        # has cleared this module's globals
        if getattr(self, "h", None) is None or _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

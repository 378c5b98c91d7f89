"""Python binding of lpk, the MI355X library for interior-point search directions.

Argument marshalling only: every computation runs in the HIP library ``liblpk.so``
(built by ``paper_1604_07491_amd/build.py``).  The names follow the C ABI of
``include/lpk.h``: :func:`lp_create`, :func:`lp_create_dense`, :func:`lp_create_bounded`,
:func:`ipm_step`, :func:`direction_solve`, :func:`lp_solve`, :func:`lp_solve_batch`,
:func:`lp_get_state`, :func:`lp_set_state`, :func:`lp_bounded_solution`,
:func:`lp_footprint_bytes`, :func:`lp_colour_rows`, :func:`lp_presolve_rows`,
:func:`lp_bounds_standard_form`, and the server of ``include/lpk_server.h``.

Arrays may be numpy arrays (host; the library copies them) or torch tensors on the GPU
(``device_io=1``; their ``data_ptr()`` is passed and torch's current stream is used).
Importing this module never falls back to another implementation: if the library is
missing, :func:`lib` raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblpk.so")

LP_OK, LP_EINVAL, LP_EDIM, LP_ENONFINITE, LP_ENOMEM, LP_ETOOBIG, LP_EDEVICE = 0, 1, 2, 3, 4, 5, 6
LP_NOT_CONVERGED, LP_DIVERGED, LP_KRYLOV_MAXIT = 7, 8, 9
LP_FP64, LP_MIXED = 0, 1
LP_ABGMRES, LP_CGNE, LP_MRNE, LP_BAGMRES = 0, 1, 2, 3
LP_NESOR, LP_CIMMINO, LP_NESSOR, LP_GSOR = 0, 1, 2, 3


class LpError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {status_str(status)} ({msg})")
        self.status = status


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("krylov", C.c_int32), ("inner", C.c_int32),
                ("inner_sweeps", C.c_int32), ("omega", C.c_double), ("omega_c", C.c_double),
                ("krylov_max_iter", C.c_int64), ("ipm_max_iter", C.c_int32), ("start", C.c_int32),
                ("eps_out", C.c_double), ("eta", C.c_double), ("phi", C.c_double),
                ("sigma_max", C.c_double), ("eps_in0", C.c_double), ("eps_in_min", C.c_double),
                ("eps_in_max", C.c_double), ("init_tol", C.c_double), ("backtrack", C.c_double),
                ("max_backtrack", C.c_int32), ("device_io", C.c_int32), ("stream", C.c_void_p),
                ("poll_every", C.c_int32), ("use_graphs", C.c_int32), ("schedule", C.c_int32),
                ("max_correctors", C.c_int32)]


class KrylovInfo(C.Structure):
    _fields_ = [("iters", C.c_int64), ("beta", C.c_double), ("res_est", C.c_double),
                ("res_true", C.c_double), ("failed", C.c_int32), ("pad0", C.c_int32)]


class IterInfo(C.Structure):
    _fields_ = [(f, C.c_double) for f in ("mu", "gamma", "gamma_rel", "rp_rel", "rd_rel", "gap_rel",
                                          "pobj", "dobj", "alpha_p", "alpha_d", "sigma", "eps_in",
                                          "res_af", "res_cc")] + \
               [("k_af", C.c_int64), ("k_cc", C.c_int64), ("fail_af", C.c_int32),
                ("fail_cc", C.c_int32), ("backtracks", C.c_int32), ("converged", C.c_int32),
                ("correctors", C.c_int32), ("pad0", C.c_int32), ("k_mcc", C.c_int64)]


class IpmState(C.Structure):
    _fields_ = [("eps_in", C.c_double), ("k", C.c_int32), ("fail_prev", C.c_int32)]


class KernelStat(C.Structure):
    _fields_ = [("cls", C.c_int32), ("pad0", C.c_int32), ("launches", C.c_int64),
                ("ms_total", C.c_double), ("bytes_total", C.c_double), ("flops_total", C.c_double),
                ("name", C.c_char * 32)]


LP_K_SWEEP, LP_K_SPMV_CSR, LP_K_SPMV_CSC, LP_K_GS_DOTS, LP_K_GS_UPDATE, LP_K_GRAM = 0, 1, 2, 3, 4, 5
LP_K_CG_VEC, LP_K_COUNT = 6, 7


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32)] + \
               [(f, C.c_double) for f in ("gamma", "gamma_rel", "pobj", "dobj", "rp_rel", "rd_rel",
                                          "gap_rel")] + \
               [("krylov_iters", C.c_int64), ("seconds", C.c_double)]


class ServerOptions(C.Structure):
    _fields_ = [("slots", C.c_int32), ("max_skip", C.c_int32), ("lanes", C.c_int32), ("pad0", C.c_int32),
                ("hbm_budget", C.c_uint64), ("solver", Options)]


class Completion(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("status", C.c_int32), ("iters", C.c_int32),
                ("pobj", C.c_double), ("dobj", C.c_double), ("gamma_rel", C.c_double),
                ("krylov_iters", C.c_int64), ("t_submit", C.c_double), ("t_start", C.c_double),
                ("t_done", C.c_double), ("footprint", C.c_uint64)]


# every entry point declared in include/lpk.h and include/lpk_server.h, with its signature
_P = C.c_void_p
SIGNATURES = {
    "lp_options_default": (C.c_int, [C.POINTER(Options)]),
    "lp_create": (C.c_int, [C.c_int64, C.c_int64, C.c_int64, _P, _P, _P, _P, _P, C.POINTER(Options),
                            C.POINTER(C.c_void_p)]),
    "lp_create_dense": (C.c_int, [C.c_int64, C.c_int64, _P, C.c_int64, _P, _P, C.POINTER(Options),
                                  C.POINTER(C.c_void_p)]),
    "lp_create_bounded": (C.c_int, [C.c_int64, C.c_int64, C.c_int64, _P, _P, _P, _P, _P, _P, _P,
                                    C.POINTER(Options), C.POINTER(C.c_void_p)]),
    "lp_bounded_solution": (C.c_int, [_P, _P, _P, C.POINTER(C.c_double)]),
    "lp_bounds_standard_form": (C.c_int, [C.c_int64, C.c_int64, _P, _P, _P, _P, _P, _P, _P,
                                          C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                          _P, _P, _P, _P, _P, C.POINTER(C.c_double)]),
    "lp_presolve_rows": (C.c_int, [C.c_int64, C.c_int64, _P, _P, _P, _P, C.c_double, _P, C.POINTER(C.c_int64)]),
    "lp_presolve_dependent_rows": (C.c_int, [C.c_int64, C.c_int64, _P, _P, _P, _P, C.c_double, _P,
                                             C.POINTER(C.c_int64)]),
    "lp_destroy": (None, [_P]),
    "ipm_step": (C.c_int, [_P, C.POINTER(IterInfo)]),
    "direction_solve": (C.c_int, [_P, _P, _P, C.c_double, _P, _P, C.POINTER(KrylovInfo)]),
    "direction_solve_noalloc": (C.c_int, [_P, _P, _P, C.c_double, _P, _P, C.POINTER(KrylovInfo)]),
    "lp_solve": (C.c_int, [_P, C.POINTER(Result)]),
    "lp_get_state": (C.c_int, [_P, _P, _P, _P, C.POINTER(IpmState)]),
    "lp_set_state": (C.c_int, [_P, _P, _P, _P, C.POINTER(IpmState)]),
    "lp_get_log": (C.c_int, [_P, C.POINTER(IterInfo), C.c_int32, C.POINTER(C.c_int32)]),
    "lp_footprint_bytes": (C.c_int, [C.c_int64, C.c_int64, C.c_int64, C.POINTER(Options),
                                     C.POINTER(C.c_uint64)]),
    "lp_colouring": (C.c_int, [_P, C.POINTER(C.c_int32), _P, C.c_int32]),
    "lp_sweep_layout": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "lp_colour_rows": (C.c_int, [C.c_int64, C.c_int64, _P, _P, _P, _P, C.POINTER(C.c_int32)]),
    "lp_profile": (C.c_int, [_P, C.c_uint32]),
    "lp_profile_read": (C.c_int, [_P, C.POINTER(KernelStat), C.c_int32, C.POINTER(C.c_int32)]),
    "lp_solve_batch": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.c_int32, C.POINTER(Result)]),
    "lp_server_options_default": (C.c_int, [C.POINTER(ServerOptions)]),
    "lp_server_create": (C.c_int, [C.POINTER(ServerOptions), C.POINTER(C.c_void_p)]),
    "lp_server_submit": (C.c_int, [_P, C.c_int64, C.c_int64, C.c_int64, _P, _P, _P, _P, _P,
                                   C.POINTER(C.c_uint64)]),
    "lp_server_poll": (C.c_int, [_P, C.POINTER(Completion), C.c_int32, C.POINTER(C.c_int32)]),
    "lp_server_wait": (C.c_int, [_P, C.c_int32, C.c_double]),
    "lp_server_result": (C.c_int, [_P, C.c_uint64, _P, _P, _P]),
    "lp_server_stats": (C.c_int, [_P, C.POINTER(C.c_uint64), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "lp_server_destroy": (C.c_int, [_P]),
    "lp_time_kernel": (C.c_int, [_P, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "lp_time_batch_kernel": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.c_int32, C.c_int32,
                                       C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(C.c_int32)]),
    "lp_status_str": (C.c_char_p, [C.c_int]),
    "lp_last_error": (C.c_char_p, []),
    "lp_version": (C.c_char_p, []),
}

_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1604_07491_amd/build.py")
        # torch ships its own HIP runtime under the same soname; loading torch first makes
        # the library bind to that one runtime, so torch's device pointers and streams are
        # valid in the library and both see the GPU
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_str(s: int) -> str:
    return lib().lp_status_str(int(s)).decode()


def last_error() -> str:
    return lib().lp_last_error().decode()


def _check(rc: int, where: str, ok=(LP_OK,)):
    if rc not in ok:
        raise LpError(rc, where, last_error())
    return rc


def options(**kw) -> Options:
    o = Options()
    lib().lp_options_default(C.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp64": LP_FP64, "mixed": LP_MIXED}[v]
        if k == "inner" and isinstance(v, str):
            v = {"nesor": LP_NESOR, "cimmino": LP_CIMMINO, "nessor": LP_NESSOR, "gsor": LP_GSOR}[v]
        if k == "krylov" and isinstance(v, str):
            v = {"abgmres": LP_ABGMRES, "cgne": LP_CGNE, "mrne": LP_MRNE, "bagmres": LP_BAGMRES}[v]
        setattr(o, k, v)
    return o


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _ptr(a, dtype):
    """Device pointer of a torch tensor or host pointer of a numpy array (no copy made
    unless the dtype or layout must change)."""
    if a is None:
        return None, None
    if _is_torch(a):
        import torch
        tdt = {np.float64: torch.float64, np.int64: torch.int64, np.int32: torch.int32}[dtype]
        t = a.to(tdt).contiguous()
        return t.data_ptr(), t
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr.ctypes.data, arr


def _dict(s: C.Structure):
    return {k: getattr(s, k) for k, _ in s._fields_ if not k.startswith("pad")}


class Problem:
    """An LP resident on the device (wraps an ``lp_problem*``)."""

    def __init__(self, handle: int, m: int, n: int, opts: Options):
        self.h = C.c_void_p(handle)
        self.m, self.n, self.opts = m, n, opts

    def close(self):
        if self.h:
            lib().lp_destroy(self.h)
            self.h = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # host/device output buffers following device_io
    def _out(self, size):
        if self.opts.device_io:
            import torch
            t = torch.empty(size, dtype=torch.float64, device="cuda")
            return t, t.data_ptr()
        a = np.zeros(size)
        return a, a.ctypes.data

    def sweep_layout(self):
        """(fp32, kind): the sweeps run in FP32; kind 2 one workgroup from LDS alone, 1 one
        workgroup with the rows read from memory, 0 colour by colour."""
        f, k = C.c_int32(0), C.c_int32(0)
        _check(lib().lp_sweep_layout(self.h, C.byref(f), C.byref(k)), "lp_sweep_layout")
        return int(f.value), int(k.value)

    def colouring(self):
        nc = C.c_int32(0)
        _check(lib().lp_colouring(self.h, C.byref(nc), None, 0), "lp_colouring")
        sizes = np.zeros(nc.value, np.int32)
        _check(lib().lp_colouring(self.h, C.byref(nc), sizes.ctypes.data, nc.value), "lp_colouring")
        return sizes


def lp_create(m, n, row_ptr, col_idx, val, b, c, opts: Optional[Options] = None, **kw) -> Problem:
    """``lp_create`` of the C ABI (introduction: min c^T x s.t. A x = b, x >= 0)."""
    o = opts if opts is not None else options(**kw)
    keep = []
    if not o.stream:
        import torch
        if torch.cuda.is_available():
            o.stream = torch.cuda.current_stream().cuda_stream
    if _is_torch(val):
        import torch
        o.device_io = 1
        if not o.stream:
            o.stream = torch.cuda.current_stream().cuda_stream
    ptrs = []
    for a, dt in ((row_ptr, np.int64), (col_idx, np.int32), (val, np.float64), (b, np.float64), (c, np.float64)):
        p_, k_ = _ptr(a, dt)
        ptrs.append(p_)
        keep.append(k_)
    nnz = int(row_ptr[-1])
    h = C.c_void_p(None)
    _check(lib().lp_create(int(m), int(n), nnz, *ptrs, C.byref(o), C.byref(h)), "lp_create")
    return Problem(h.value, int(m), int(n), o)


def lp_create_dense(A, b, c, opts: Optional[Options] = None, **kw) -> Problem:
    o = opts if opts is not None else options(**kw)
    m, n = A.shape
    keep = []
    pa, ka = _ptr(A, np.float64)
    pb, kb = _ptr(b, np.float64)
    pc, kc = _ptr(c, np.float64)
    keep += [ka, kb, kc]
    if _is_torch(A):
        import torch
        o.device_io = 1
        if not o.stream:
            o.stream = torch.cuda.current_stream().cuda_stream
    h = C.c_void_p(None)
    _check(lib().lp_create_dense(int(m), int(n), pa, int(n), pb, pc, C.byref(o), C.byref(h)), "lp_create_dense")
    return Problem(h.value, int(m), int(n), o)


def from_lp(lp, opts: Optional[Options] = None, device=False, **kw) -> Problem:
    """lp_create from a generator LP (synth.LP); device=True passes torch CUDA tensors."""
    if device:
        import torch
        t = lambda a: torch.as_tensor(np.asarray(a)).cuda()
        return lp_create(lp.m, lp.n, t(lp.row_ptr), t(lp.col_idx), t(lp.val), t(lp.b), t(lp.c), opts, **kw)
    return lp_create(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.val, lp.b, lp.c, opts, **kw)


def lp_bounds_standard_form(m, n, row_ptr, col_idx, val, b, c, lo, hi) -> dict:
    """``lp_bounds_standard_form``: the standard form of min c^T x, A x = b, lo <= x <= hi
    built on the host (host arrays)."""
    arrs = [np.ascontiguousarray(a, dt) for a, dt in ((row_ptr, np.int64), (col_idx, np.int32),
                                                     (val, np.float64), (b, np.float64), (c, np.float64),
                                                     (lo, np.float64), (hi, np.float64))]
    ms, ns, nz = C.c_int64(0), C.c_int64(0), C.c_int64(0)
    ptrs = [a.ctypes.data for a in arrs]
    _check(lib().lp_bounds_standard_form(int(m), int(n), *ptrs, C.byref(ms), C.byref(ns), C.byref(nz),
                                         None, None, None, None, None, None), "lp_bounds_standard_form")
    rp = np.zeros(ms.value + 1, np.int64)
    ci = np.zeros(nz.value, np.int32)
    v = np.zeros(nz.value)
    bs = np.zeros(ms.value)
    cs = np.zeros(ns.value)
    off = C.c_double(0.0)
    _check(lib().lp_bounds_standard_form(int(m), int(n), *ptrs, C.byref(ms), C.byref(ns), C.byref(nz),
                                         rp.ctypes.data, ci.ctypes.data, v.ctypes.data, bs.ctypes.data,
                                         cs.ctypes.data, C.byref(off)), "lp_bounds_standard_form")
    return dict(m=ms.value, n=ns.value, row_ptr=rp, col_idx=ci, val=v, b=bs, c=cs, offset=off.value)


def lp_presolve_rows(m, n, row_ptr, col_idx, val, b, tol: float = 1e-12):
    """``lp_presolve_rows``: a 0/1 mask of the rows to keep (rows that are scalar multiples
    of an earlier row are dropped)."""
    arrs = [np.ascontiguousarray(a, dt) for a, dt in ((row_ptr, np.int64), (col_idx, np.int32),
                                                     (val, np.float64), (b, np.float64))]
    keep = np.zeros(int(m), np.int32)
    mk = C.c_int64(0)
    _check(lib().lp_presolve_rows(int(m), int(n), *[a.ctypes.data for a in arrs], float(tol), keep.ctypes.data,
                                  C.byref(mk)), "lp_presolve_rows")
    return keep.astype(bool)


def lp_presolve_dependent_rows(m, n, row_ptr, col_idx, val, b, tol: float = 1e-9):
    """``lp_presolve_dependent_rows``: a 0/1 mask of the rows to keep (the rows in the span
    of the rows before them are dropped: the kept rows are the first row basis)."""
    arrs = [np.ascontiguousarray(a, dt) for a, dt in ((row_ptr, np.int64), (col_idx, np.int32),
                                                     (val, np.float64), (b, np.float64))]
    keep = np.zeros(int(m), np.int32)
    mk = C.c_int64(0)
    _check(lib().lp_presolve_dependent_rows(int(m), int(n), *[a.ctypes.data for a in arrs], float(tol),
                                            keep.ctypes.data, C.byref(mk)), "lp_presolve_dependent_rows")
    assert mk.value == int(keep.sum())
    return keep.astype(bool)


def lp_create_bounded(m, n, row_ptr, col_idx, val, b, c, lo, hi, opts: Optional[Options] = None,
                      **kw) -> Problem:
    """``lp_create_bounded`` (general bounds, reduced to the standard form on the host).
    The returned Problem's m and n are the standard form's; m0 and n0 the caller's."""
    o = opts if opts is not None else options(**kw)
    host = [np.asarray(a.cpu() if _is_torch(a) else a) for a in (row_ptr, col_idx, val, b, c, lo, hi)]
    sf = lp_bounds_standard_form(m, n, *host)   # sizes of the standard form
    keep = []
    if not o.stream:
        import torch
        if torch.cuda.is_available():
            o.stream = torch.cuda.current_stream().cuda_stream
    if _is_torch(val):
        import torch
        o.device_io = 1
        if not o.stream:
            o.stream = torch.cuda.current_stream().cuda_stream
    ptrs = []
    for a, dt in ((row_ptr, np.int64), (col_idx, np.int32), (val, np.float64), (b, np.float64), (c, np.float64),
                  (lo, np.float64), (hi, np.float64)):
        p_, k_ = _ptr(a, dt)
        ptrs.append(p_)
        keep.append(k_)
    h = C.c_void_p(None)
    _check(lib().lp_create_bounded(int(m), int(n), int(host[0][-1]), *ptrs, C.byref(o), C.byref(h)),
           "lp_create_bounded")
    p = Problem(h.value, sf["m"], sf["n"], o)
    p.m0, p.n0 = int(m), int(n)
    return p


def from_bounded_lp(lp, lo, hi, opts: Optional[Options] = None, device=False, **kw) -> Problem:
    """lp_create_bounded from a bounded generator LP (synth.bounded_lp)."""
    if device:
        import torch
        t = lambda a: torch.as_tensor(np.asarray(a)).cuda()
        return lp_create_bounded(lp.m, lp.n, t(lp.row_ptr), t(lp.col_idx), t(lp.val), t(lp.b), t(lp.c), t(lo),
                                 t(hi), opts, **kw)
    return lp_create_bounded(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.val, lp.b, lp.c, lo, hi, opts, **kw)


def lp_bounded_solution(p: Problem):
    """(x, y, obj) of a bounded problem in the caller's variables and rows."""
    x, px = p._out(getattr(p, "n0", p.n))
    y, py = p._out(getattr(p, "m0", p.m))
    obj = C.c_double(0.0)
    _check(lib().lp_bounded_solution(p.h, px, py, C.byref(obj)), "lp_bounded_solution")
    return x, y, obj.value


def ipm_step(p: Problem) -> dict:
    info = IterInfo()
    _check(lib().ipm_step(p.h, C.byref(info)), "ipm_step")
    return _dict(info)


def direction_solve(p: Problem, d, f, tol: float):
    """(dw, dy, info) of min ||dw|| s.t. (A diag(d)) dw = f (eq. minnrmprob); d None: current D."""
    pd, kd = _ptr(d, np.float64)
    pf, kf = _ptr(f, np.float64)
    dw, pdw = p._out(p.n)
    dy, pdy = p._out(p.m)
    ki = KrylovInfo()
    _check(lib().direction_solve(p.h, pd, pf, float(tol), pdw, pdy, C.byref(ki)), "direction_solve")
    return dw, dy, _dict(ki)


def direction_solve_noalloc(p: Problem, d, f, tol: float, dw, dy=None) -> dict:
    """direction_solve with no device allocation in the call; returns the info dict.  d
    (n, or None: current D), f (m) and the outputs dw (n), dy (m or None) are the caller's
    contiguous float64 CUDA tensors; dw and dy are written in place."""
    def dev(t, size, name):
        if t is None:
            return None
        import torch
        if not (_is_torch(t) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                and t.numel() == size):
            raise ValueError(f"{name}: a contiguous float64 CUDA tensor of {size} entries is needed")
        return t.data_ptr()
    pd, pf = dev(d, p.n, "d"), dev(f, p.m, "f")
    pdw, pdy = dev(dw, p.n, "dw"), dev(dy, p.m, "dy")
    if pf is None or pdw is None:
        raise ValueError("f and dw are needed")
    ki = KrylovInfo()
    _check(lib().direction_solve_noalloc(p.h, pd, pf, float(tol), pdw, pdy, C.byref(ki)), "direction_solve_noalloc")
    return _dict(ki)


def lp_solve(p: Problem) -> dict:
    r = Result()
    rc = lib().lp_solve(p.h, C.byref(r))
    _check(rc, "lp_solve", ok=(LP_OK, LP_NOT_CONVERGED, LP_DIVERGED))
    out = _dict(r)
    out["status"] = rc
    return out


def lp_get_state(p: Problem):
    x, px = p._out(p.n)
    y, py = p._out(p.m)
    s, ps = p._out(p.n)
    st = IpmState()
    _check(lib().lp_get_state(p.h, px, py, ps, C.byref(st)), "lp_get_state")
    return x, y, s, _dict(st)


def lp_set_state(p: Problem, x, y, s, state: Optional[dict] = None):
    px, kx = _ptr(x, np.float64)
    py, ky = _ptr(y, np.float64)
    ps, ks = _ptr(s, np.float64)
    st = None
    if state is not None:
        st = IpmState(state["eps_in"], state["k"], state["fail_prev"])
    _check(lib().lp_set_state(p.h, px, py, ps, C.byref(st) if st is not None else None), "lp_set_state")


def lp_get_log(p: Problem):
    n = C.c_int32(0)
    _check(lib().lp_get_log(p.h, None, 0, C.byref(n)), "lp_get_log")
    arr = (IterInfo * max(1, n.value))()
    _check(lib().lp_get_log(p.h, arr, n.value, C.byref(n)), "lp_get_log")
    return [_dict(arr[i]) for i in range(n.value)]


def lp_footprint_bytes(m, n, nnz, opts: Optional[Options] = None) -> int:
    b = C.c_uint64(0)
    _check(lib().lp_footprint_bytes(int(m), int(n), int(nnz), C.byref(opts) if opts else None, C.byref(b)),
           "lp_footprint_bytes")
    return int(b.value)


def lp_colour_rows(m, n, row_ptr, col_idx):
    """Host greedy colouring: (colour[m], perm[m], ncolours)."""
    rp = np.ascontiguousarray(row_ptr, np.int64)
    ci = np.ascontiguousarray(col_idx, np.int32)
    col = np.zeros(m, np.int32)
    perm = np.zeros(m, np.int32)
    nc = C.c_int32(0)
    _check(lib().lp_colour_rows(int(m), int(n), rp.ctypes.data, ci.ctypes.data, col.ctypes.data,
                                perm.ctypes.data, C.byref(nc)), "lp_colour_rows")
    return col, perm, int(nc.value)


def lp_profile(p: Problem, mask: int):
    """Enable per-launch HIP-event timing for the kernel classes in mask (0: off)."""
    _check(lib().lp_profile(p.h, int(mask)), "lp_profile")


def lp_profile_read(p: Problem):
    """{class name: dict(launches, ms_total, bytes_total)} since lp_profile."""
    arr = (KernelStat * LP_K_COUNT)()
    n = C.c_int32(0)
    _check(lib().lp_profile_read(p.h, arr, LP_K_COUNT, C.byref(n)), "lp_profile_read")
    return {arr[i].name.decode(): dict(launches=arr[i].launches, ms_total=arr[i].ms_total,
                                       bytes_total=arr[i].bytes_total, flops_total=arr[i].flops_total)
            for i in range(n.value)}


def lp_solve_batch(problems, width: int):
    """Solve created problems, up to `width` of them in lockstep (one launch per phase)."""
    arr = (C.c_void_p * len(problems))(*[p.h.value for p in problems])
    res = (Result * max(1, len(problems)))()
    _check(lib().lp_solve_batch(arr, len(problems), int(width), res), "lp_solve_batch")
    return [_dict(res[i]) for i in range(len(problems))]


class Server:
    """The request server of include/lpk_server.h (lockstep batch, continuous admission by
    HBM footprint)."""

    def __init__(self, slots=32, max_skip=8, hbm_budget=0, solver: Optional[Options] = None, lanes=1, **kw):
        o = ServerOptions()
        lib().lp_server_options_default(C.byref(o))
        o.slots, o.max_skip, o.hbm_budget, o.lanes = int(slots), int(max_skip), int(hbm_budget), int(lanes)
        o.solver = solver if solver is not None else options(**kw)
        h = C.c_void_p(None)
        _check(lib().lp_server_create(C.byref(o), C.byref(h)), "lp_server_create")
        self.h = h
        self.sizes = {}

    def submit(self, lp) -> int:
        t = C.c_uint64(0)
        arrs = [np.ascontiguousarray(lp.row_ptr, np.int64), np.ascontiguousarray(lp.col_idx, np.int32),
                np.ascontiguousarray(lp.val, np.float64), np.ascontiguousarray(lp.b, np.float64),
                np.ascontiguousarray(lp.c, np.float64)]
        _check(lib().lp_server_submit(self.h, lp.m, lp.n, int(arrs[0][-1]), *[a.ctypes.data for a in arrs],
                                      C.byref(t)), "lp_server_submit")
        self.sizes[t.value] = (lp.m, lp.n)
        return t.value

    def wait(self, count: int, timeout: float = 600.0) -> bool:
        return lib().lp_server_wait(self.h, int(count), float(timeout)) == LP_OK

    def poll(self, cap: int = 4096):
        arr = (Completion * cap)()
        n = C.c_int32(0)
        _check(lib().lp_server_poll(self.h, arr, cap, C.byref(n)), "lp_server_poll")
        return [_dict(arr[i]) for i in range(n.value)]

    def result(self, ticket: int):
        m, n = self.sizes[ticket]
        x, y, s = np.zeros(n), np.zeros(m), np.zeros(n)
        _check(lib().lp_server_result(self.h, C.c_uint64(ticket), x.ctypes.data, y.ctypes.data, s.ctypes.data),
               "lp_server_result")
        return x, y, s

    def stats(self):
        b, q, r = C.c_uint64(0), C.c_int32(0), C.c_int32(0)
        _check(lib().lp_server_stats(self.h, C.byref(b), C.byref(q), C.byref(r)), "lp_server_stats")
        return dict(bytes_in_use=b.value, queued=q.value, running=r.value)

    def close(self):
        if self.h:
            lib().lp_server_destroy(self.h)
            self.h = C.c_void_p(None)

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def lp_time_kernel(p: Problem, cls: int, reps: int = 200):
    """Replay-timed mean launch duration (us) and algorithmic bytes/flops per launch."""
    us, by, fl, nl = C.c_double(0), C.c_double(0), C.c_double(0), C.c_int32(0)
    _check(lib().lp_time_kernel(p.h, int(cls), int(reps), C.byref(us), C.byref(by), C.byref(fl), C.byref(nl)),
           "lp_time_kernel")
    return dict(us_per_launch=us.value, bytes_per_launch=by.value, flops_per_launch=fl.value,
                launches_per_group=nl.value)


def lp_time_batch_kernel(problems, cls: int, reps: int = 200):
    """lp_time_kernel over a batch: one launch covers every problem; bytes/flops summed."""
    arr = (C.c_void_p * len(problems))(*[p.h.value for p in problems])
    us, by, fl, nl = C.c_double(0), C.c_double(0), C.c_double(0), C.c_int32(0)
    _check(lib().lp_time_batch_kernel(arr, len(problems), int(cls), int(reps), C.byref(us), C.byref(by),
                                      C.byref(fl), C.byref(nl)), "lp_time_batch_kernel")
    return dict(us_per_launch=us.value, bytes_per_launch=by.value, flops_per_launch=fl.value,
                launches_per_group=nl.value)

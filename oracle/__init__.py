"""CPU FP64 oracle -- TEST INFRASTRUCTURE ONLY.

ctypes binding of ``oracle/oracle.c``, a plain single-threaded FP64 implementation of the
interior-point search-direction path of Cui, Morikuni, Tsuchiya and Hayami (Mehrotra's
predictor-corrector method with the w-recurrence, the row-scaled min-norm problem solved
by AB-GMRES / CGNE / MRNE preconditioned by NE-SOR / NE-SSOR / Cimmino inner iterations).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library.

Each wrapper names the part of the paper it follows; see ``oracle.c`` for the arithmetic.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# status codes
OK, EINVAL, ENOMEM, NOT_CONVERGED, DIVERGED = 0, 1, 4, 7, 8
NESOR, CIMMINO, NESSOR = 0, 1, 2
ABGMRES, CGNE, MRNE, BAGMRES = 0, 1, 2, 3
ORDER_COLOUR, ORDER_NATURAL = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fused multiply-add, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class SolverOpts(C.Structure):
    _fields_ = [("krylov", C.c_int32), ("inner", C.c_int32), ("ell", C.c_int32),
                ("order", C.c_int32), ("flexible", C.c_int32), ("pad0", C.c_int32),
                ("omega", C.c_double), ("omega_c", C.c_double), ("kmax", C.c_int64)]


class KrylovInfo(C.Structure):
    _fields_ = [("iters", C.c_int64), ("beta", C.c_double), ("res_est", C.c_double),
                ("res_true", C.c_double), ("failed", C.c_int32), ("pad0", C.c_int32),
                ("omega_c", C.c_double)]


class IpmOpts(C.Structure):
    _fields_ = [("solver", SolverOpts), ("max_iter", C.c_int32), ("start", C.c_int32),
                ("eps_out", C.c_double), ("eta", C.c_double), ("phi", C.c_double),
                ("sigma_max", C.c_double), ("eps_in0", C.c_double), ("eps_in_min", C.c_double),
                ("eps_in_max", C.c_double), ("init_tol", C.c_double), ("backtrack", C.c_double),
                ("max_backtrack", C.c_int32), ("max_correctors", C.c_int32)]


class IterLog(C.Structure):
    _fields_ = [(f, C.c_double) for f in ("mu", "gamma", "gamma_rel", "rp_rel", "rd_rel", "gap_rel",
                                          "pobj", "dobj", "alpha_p", "alpha_d", "sigma", "eps_in",
                                          "res_af", "res_cc")] + \
               [("k_af", C.c_int64), ("k_cc", C.c_int64), ("fail_af", C.c_int32),
                ("fail_cc", C.c_int32), ("backtracks", C.c_int32), ("correctors", C.c_int32)]


class IpmState(C.Structure):
    _fields_ = [("eps_in", C.c_double), ("fail_prev", C.c_int32), ("k", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = C.CDLL(_LIB)
        _lib.orc_power_lambda.restype = C.c_double
    return _lib


def _p(a, dt):
    if a is None:
        return None
    assert a.dtype == dt and a.flags.c_contiguous, (a.dtype, dt)
    return a.ctypes.data_as(C.c_void_p)


def _csr(lp_or_tuple):
    if isinstance(lp_or_tuple, tuple):
        m, n, rp, ci, val = lp_or_tuple
    else:
        m, n, rp, ci, val = lp_or_tuple.m, lp_or_tuple.n, lp_or_tuple.row_ptr, lp_or_tuple.col_idx, lp_or_tuple.val
    return (int(m), int(n), np.ascontiguousarray(rp, np.int64), np.ascontiguousarray(ci, np.int32),
            np.ascontiguousarray(val, np.float64))


def solver_opts(krylov=ABGMRES, inner=NESOR, ell=2, order=ORDER_COLOUR, flexible=0, omega=1.0,
                omega_c=0.0, kmax=0) -> SolverOpts:
    return SolverOpts(krylov, inner, ell, order, flexible, 0, omega, omega_c, kmax)


def ipm_opts(**kw) -> IpmOpts:
    o = IpmOpts()
    lib().orc_ipm_opts_default(C.byref(o))
    solver = kw.pop("solver", None)
    if solver is not None:
        o.solver = solver
    for k, v in kw.items():
        setattr(o, k, v)
    return o


# ------------------------------------------------------------------------------------
def csr_mv(A, x):
    m, n, rp, ci, val = _csr(A)
    x = np.ascontiguousarray(x, np.float64)
    y = np.zeros(m)
    lib().orc_csr_mv(C.c_int64(m), _p(rp, np.int64), _p(ci, np.int32), _p(val, np.float64),
                     _p(x, np.float64), _p(y, np.float64))
    return y


def csr_tmv(A, x):
    m, n, rp, ci, val = _csr(A)
    x = np.ascontiguousarray(x, np.float64)
    y = np.zeros(n)
    lib().orc_csr_tmv(C.c_int64(m), C.c_int64(n), _p(rp, np.int64), _p(ci, np.int32),
                      _p(val, np.float64), _p(x, np.float64), _p(y, np.float64))
    return y


def colour(A):
    """Greedy row colouring; returns (colour[m], perm[m], ncolours)."""
    m, n, rp, ci, _ = _csr(A)
    col = np.zeros(m, np.int32)
    perm = np.zeros(m, np.int32)
    nc = C.c_int32(0)
    rc = lib().orc_colour(C.c_int64(m), C.c_int64(n), _p(rp, np.int64), _p(ci, np.int32),
                          _p(col, np.int32), _p(perm, np.int32), C.byref(nc))
    assert rc == OK
    return col, perm, int(nc.value)


def nesor(A, g, omega=1.0, ell=2, perm=None, rn2=None, ssor=False):
    """NE-SOR (or NE-SSOR) inner iterations from zero; returns (z = A^T p, p)."""
    m, n, rp, ci, val = _csr(A)
    g = np.ascontiguousarray(g, np.float64)
    z = np.zeros(n)
    p = np.zeros(m)
    pp = None if perm is None else np.ascontiguousarray(perm, np.int32)
    rr = None if rn2 is None else np.ascontiguousarray(rn2, np.float64)
    fn = lib().orc_nessor if ssor else lib().orc_nesor
    fn(C.c_int64(m), C.c_int64(n), _p(rp, np.int64), _p(ci, np.int32), _p(val, np.float64),
       _p(rr, np.float64), _p(g, np.float64), C.c_double(omega), C.c_int32(ell), _p(pp, np.int32),
       _p(z, np.float64), _p(p, np.float64))
    return z, p


def cimmino(A, g, omega_c, ell=2):
    m, n, rp, ci, val = _csr(A)
    g = np.ascontiguousarray(g, np.float64)
    z = np.zeros(n)
    p = np.zeros(m)
    lib().orc_cimmino(C.c_int64(m), C.c_int64(n), _p(rp, np.int64), _p(ci, np.int32),
                      _p(val, np.float64), _p(g, np.float64), C.c_double(omega_c), C.c_int32(ell),
                      _p(z, np.float64), _p(p, np.float64))
    return z, p


def power_lambda(A, iters=20):
    m, n, rp, ci, val = _csr(A)
    return float(lib().orc_power_lambda(C.c_int64(m), C.c_int64(n), _p(rp, np.int64),
                                        _p(ci, np.int32), _p(val, np.float64), C.c_int32(iters)))


def scale(A, d=None):
    """(rho, ahat_values) of the row-scaled A D."""
    m, n, rp, ci, val = _csr(A)
    rho = np.zeros(m)
    ah = np.zeros(len(val))
    dd = None if d is None else np.ascontiguousarray(d, np.float64)
    rc = lib().orc_scale(C.c_int64(m), _p(rp, np.int64), _p(ci, np.int32), _p(val, np.float64),
                         _p(dd, np.float64), _p(rho, np.float64), _p(ah, np.float64))
    assert rc == OK
    return rho, ah


def dirsolve(A, d, f, eps, opts: Optional[SolverOpts] = None):
    """Min-norm solve of (A D) dw = f; returns (dw, dy, info dict)."""
    m, n, rp, ci, val = _csr(A)
    o = opts if opts is not None else solver_opts()
    f = np.ascontiguousarray(f, np.float64)
    dd = None if d is None else np.ascontiguousarray(d, np.float64)
    dw = np.zeros(n)
    dy = np.zeros(m)
    info = KrylovInfo()
    rc = lib().orc_dirsolve(C.c_int64(m), C.c_int64(n), _p(rp, np.int64), _p(ci, np.int32),
                            _p(val, np.float64), _p(dd, np.float64), _p(f, np.float64),
                            C.c_double(eps), C.byref(o), _p(dw, np.float64), _p(dy, np.float64),
                            C.byref(info))
    assert rc == OK, rc
    return dw, dy, {k: getattr(info, k) for k, _ in KrylovInfo._fields_ if k != "pad0"}


def affine_direction(lp, x, y, s, eps, opts=None):
    m, n, rp, ci, val = _csr(lp)
    o = opts if opts is not None else solver_opts()
    dx, dy, ds = np.zeros(n), np.zeros(m), np.zeros(n)
    info = KrylovInfo()
    args = [np.ascontiguousarray(v, np.float64) for v in (lp.b, lp.c, x, y, s)]
    rc = lib().orc_affine_direction(C.c_int64(m), C.c_int64(n), _p(rp, np.int64), _p(ci, np.int32),
                                    _p(val, np.float64), *[_p(a, np.float64) for a in args],
                                    C.c_double(eps), C.byref(o), _p(dx, np.float64),
                                    _p(dy, np.float64), _p(ds, np.float64), C.byref(info))
    assert rc == OK, rc
    return dx, dy, ds, info.iters


def corrector_direction(lp, x, s, dx_af, ds_af, sigma_mu, eps, opts=None):
    m, n, rp, ci, val = _csr(lp)
    o = opts if opts is not None else solver_opts()
    dx, dy, ds = np.zeros(n), np.zeros(m), np.zeros(n)
    info = KrylovInfo()
    args = [np.ascontiguousarray(v, np.float64) for v in (x, s, dx_af, ds_af)]
    rc = lib().orc_corrector_direction(C.c_int64(m), C.c_int64(n), _p(rp, np.int64),
                                       _p(ci, np.int32), _p(val, np.float64),
                                       *[_p(a, np.float64) for a in args], C.c_double(sigma_mu),
                                       C.c_double(eps), C.byref(o), _p(dx, np.float64),
                                       _p(dy, np.float64), _p(ds, np.float64), C.byref(info))
    assert rc == OK, rc
    return dx, dy, ds, info.iters


def centrality_target(x, s, dx, ds, tp, td, sigma_mu):
    """Complementarity target r of a centrality corrector at the trial point (x + tp dx,
    s + td ds): the products moved into [0.1, 10] sigma mu, decreases capped at 10 sigma mu."""
    n = len(x)
    arrs = [np.ascontiguousarray(a, np.float64) for a in (x, s, dx, ds)]
    r = np.zeros(n)
    lib().orc_centrality_target(C.c_int64(n), *[_p(a, np.float64) for a in arrs], C.c_double(tp),
                                C.c_double(td), C.c_double(sigma_mu), _p(r, np.float64))
    return r


def centrality_direction(lp, x, s, r, eps, opts: Optional[SolverOpts] = None):
    """(dx, dy, ds, info) with A dx = 0, A^T dy + ds = 0, S dx + X ds = r (multiple
    centrality correctors), by the corrector's min-norm solve."""
    m, n, rp, ci, val = _csr(lp)
    o = opts if opts is not None else solver_opts()
    xx, ss, rr = (np.ascontiguousarray(a, np.float64) for a in (x, s, r))
    dx, dy, ds = np.zeros(n), np.zeros(m), np.zeros(n)
    info = KrylovInfo()
    rc = lib().orc_centrality_direction(C.c_int64(m), C.c_int64(n), _p(rp, np.int64), _p(ci, np.int32),
                                        _p(val, np.float64), _p(xx, np.float64), _p(ss, np.float64),
                                        _p(rr, np.float64), C.c_double(eps), C.byref(o), _p(dx, np.float64),
                                        _p(dy, np.float64), _p(ds, np.float64), C.byref(info))
    assert rc == OK, rc
    return dx, dy, ds, {k: getattr(info, k) for k, _ in KrylovInfo._fields_ if k != "pad0"}


def init_point(lp, opts=None, tol=1e-10):
    m, n, rp, ci, val = _csr(lp)
    o = opts if opts is not None else solver_opts()
    x, y, s = np.zeros(n), np.zeros(m), np.zeros(n)
    b = np.ascontiguousarray(lp.b, np.float64)
    c = np.ascontiguousarray(lp.c, np.float64)
    rc = lib().orc_init_point(C.c_int64(m), C.c_int64(n), _p(rp, np.int64), _p(ci, np.int32),
                              _p(val, np.float64), _p(b, np.float64), _p(c, np.float64),
                              C.byref(o), C.c_double(tol), _p(x, np.float64), _p(y, np.float64),
                              _p(s, np.float64))
    assert rc == OK, rc
    return x, y, s


def _log_dicts(log, count):
    names = [f for f, _ in IterLog._fields_ if f != "pad0"]
    return [{k: getattr(log[i], k) for k in names} for i in range(count)]


def ipm(lp, opts: Optional[IpmOpts] = None, x=None, y=None, s=None, pairs=None):
    """Whole interior-point solve; returns dict(status, x, y, s, iters, gamma, gamma_rel, log).
    pairs: (k, 2) column indices of split free variables to recentre after the starting
    point and every step (the bounded-variable reduction)."""
    m, n, rp, ci, val = _csr(lp)
    o = opts if opts is not None else ipm_opts()
    xx = np.zeros(n) if x is None else np.array(x, np.float64)
    yy = np.zeros(m) if y is None else np.array(y, np.float64)
    ss = np.zeros(n) if s is None else np.array(s, np.float64)
    if x is not None:
        o.start = 1
    b = np.ascontiguousarray(lp.b, np.float64)
    c = np.ascontiguousarray(lp.c, np.float64)
    log = (IterLog * (o.max_iter + 1))()
    iters = C.c_int32(0)
    g = C.c_double(0)
    gr = C.c_double(0)
    pr = np.ascontiguousarray(np.zeros((0, 2)) if pairs is None else pairs, np.int64).reshape(-1, 2)
    rc = lib().orc_ipm_pairs(C.c_int64(m), C.c_int64(n), _p(rp, np.int64), _p(ci, np.int32),
                             _p(val, np.float64), _p(b, np.float64), _p(c, np.float64), C.byref(o),
                             C.c_int64(pr.shape[0]), _p(pr, np.int64) if pr.size else None,
                             _p(xx, np.float64), _p(yy, np.float64), _p(ss, np.float64), log,
                             C.byref(iters), C.byref(g), C.byref(gr))
    return dict(status=int(rc), x=xx, y=yy, s=ss, iters=int(iters.value), gamma=g.value,
                gamma_rel=gr.value, log=_log_dicts(log, int(iters.value) + 1),
                pobj=float(c @ xx), dobj=float(b @ yy))


def ipm_iterate(lp, x, y, s, state: IpmState, opts: Optional[IpmOpts] = None):
    """One Mehrotra iteration in place; returns (rc, done, log dict)."""
    m, n, rp, ci, val = _csr(lp)
    o = opts if opts is not None else ipm_opts()
    b = np.ascontiguousarray(lp.b, np.float64)
    c = np.ascontiguousarray(lp.c, np.float64)
    L = IterLog()
    done = C.c_int32(0)
    rc = lib().orc_ipm_iterate(C.c_int64(m), C.c_int64(n), _p(rp, np.int64), _p(ci, np.int32),
                               _p(val, np.float64), _p(b, np.float64), _p(c, np.float64),
                               C.byref(o), _p(x, np.float64), _p(y, np.float64), _p(s, np.float64),
                               C.byref(state), C.byref(L), C.byref(done))
    return int(rc), int(done.value), _log_dicts([L], 1)[0]


def new_state(eps_in0=1e-6) -> IpmState:
    return IpmState(eps_in0, 0, 0)

"""Bounded variables l <= x <= u, oracle side -- TEST INFRASTRUCTURE ONLY.

The method of the paper is stated for the standard form of its introduction
(min c^T x, A x = b, x >= 0).  For test problems with general bounds, the experiments on
typical LPs (Sec. 4.3) transform them first, as LIPSOL does.  This module writes that
transform out plainly on a dense copy of A, solves the standard-form LP with the oracle's
interior-point method, and maps the solution back.  Per original variable x_j:

* l finite, u = +inf (lower):  x_j = l_j + x'_j.
* l, u finite, l < u (box):     x_j = l_j + x'_j and one more constraint
  x'_j + w_j = u_j - l_j with a slack w_j >= 0.
* l = -inf, u finite (upper):   x_j = u_j - x'_j (the column and its cost change sign).
* l = -inf, u = +inf (free):    x_j = x+_j - x-_j (a second column -a_j, cost -c_j).
* l = u (fixed):                x_j = l_j; the column leaves the problem.

The two parts of a split free variable grow without bound along the central path (their
dual slacks must both vanish), so the solve recentres each pair after the starting point
and after every step: a smaller part above (1 + |x+ - x-|) / 2 is lowered by the excess,
both parts by the same amount (x, A x and c^T x unchanged).

Column order of the standard form: the kept original columns in their order, then the
negative parts of the free variables, then the slacks; rows: the original rows, then one
row per box variable.  b' = b - sum_j a_j shift_j over the shifted, reflected and fixed
variables, and the objective gains the constant sum_j c_j shift_j.  A row left with no
entry (every variable in it fixed) is rejected.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this.
It shares no code with the GPU library.
"""
from __future__ import annotations

import dataclasses
import types

import numpy as np

from . import ipm, ipm_opts

LOWER, BOX, UPPER, FREE, FIXED = 0, 1, 2, 3, 4


@dataclasses.dataclass
class BoundMap:
    m0: int
    n0: int
    kind: np.ndarray     # per original variable
    shift: np.ndarray    # l_j (lower, box), u_j (upper), the fixed value; 0 for free
    col: np.ndarray      # standard-form column of x'_j or x+_j; -1 when fixed
    col2: np.ndarray     # free: column of x-_j; else -1
    offset: float        # objective constant sum_j c_j shift_j


def classify(lo, hi):
    """Kind of every variable; raises ValueError on l > u, NaN, l = +inf or u = -inf."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    if np.isnan(lo).any() or np.isnan(hi).any():
        raise ValueError("NaN bound")
    if (lo == np.inf).any() or (hi == -np.inf).any() or (lo > hi).any():
        raise ValueError("empty bound interval")
    kind = np.empty(lo.size, np.int64)
    for j in range(lo.size):
        lf, uf = np.isfinite(lo[j]), np.isfinite(hi[j])
        if lf and uf:
            kind[j] = FIXED if lo[j] == hi[j] else BOX
        elif lf:
            kind[j] = LOWER
        elif uf:
            kind[j] = UPPER
        else:
            kind[j] = FREE
    return kind


def standard_form(A, b, c, lo, hi):
    """The standard-form LP (a namespace with m, n, row_ptr, col_idx, val, b, c, and the
    dense matrix as ``dense_A``) and the BoundMap.  A is a dense m0 x n0 array."""
    A = np.asarray(A, np.float64)
    b = np.asarray(b, np.float64)
    c = np.asarray(c, np.float64)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    m0, n0 = A.shape
    kind = classify(lo, hi)
    shift = np.zeros(n0)
    for j in range(n0):
        if kind[j] in (LOWER, BOX, FIXED):
            shift[j] = lo[j]
        elif kind[j] == UPPER:
            shift[j] = hi[j]
    kept = [j for j in range(n0) if kind[j] != FIXED]
    free = [j for j in range(n0) if kind[j] == FREE]
    box = [j for j in range(n0) if kind[j] == BOX]
    n1 = len(kept) + len(free) + len(box)
    m1 = m0 + len(box)
    col = -np.ones(n0, np.int64)
    col2 = -np.ones(n0, np.int64)
    for t, j in enumerate(kept):
        col[j] = t
    for t, j in enumerate(free):
        col2[j] = len(kept) + t
    As = np.zeros((m1, n1))
    cs = np.zeros(n1)
    for j in kept:
        sign = -1.0 if kind[j] == UPPER else 1.0
        As[:m0, col[j]] = sign * A[:, j]
        cs[col[j]] = sign * c[j]
    for j in free:
        As[:m0, col2[j]] = -A[:, j]
        cs[col2[j]] = -c[j]
    bs = np.zeros(m1)
    bs[:m0] = b - A @ shift
    for t, j in enumerate(box):
        As[m0 + t, col[j]] = 1.0
        As[m0 + t, len(kept) + len(free) + t] = 1.0
        bs[m0 + t] = hi[j] - lo[j]
    empty = np.flatnonzero(~(As != 0).any(axis=1))
    if empty.size:
        raise ValueError(f"row {int(empty[0])} has only fixed variables")
    rows, cols = np.nonzero(As)   # row-major: columns ascending inside each row
    row_ptr = np.zeros(m1 + 1, np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    lp = types.SimpleNamespace(m=m1, n=n1, row_ptr=row_ptr, col_idx=cols.astype(np.int32),
                               val=As[rows, cols].copy(), b=bs, c=cs, dense_A=As)
    bmap = BoundMap(m0, n0, kind, shift, col, col2, float(c @ shift))
    return lp, bmap


def to_standard_point(bmap: BoundMap, x, hi):
    """The standard-form point of an original point x inside the bounds (the inverse map:
    x' = x - l, u - x, or the positive and negative parts; w = u - x)."""
    x = np.asarray(x, np.float64)
    n1 = int(max(bmap.col.max(), bmap.col2.max())) + 1 + int((bmap.kind == BOX).sum())
    xs = np.zeros(n1)
    nb = n1 - int((bmap.kind == BOX).sum())
    t = 0
    for j in range(bmap.n0):
        k = bmap.kind[j]
        if k in (LOWER, BOX):
            xs[bmap.col[j]] = x[j] - bmap.shift[j]
        elif k == UPPER:
            xs[bmap.col[j]] = bmap.shift[j] - x[j]
        elif k == FREE:
            xs[bmap.col[j]] = max(x[j], 0.0)
            xs[bmap.col2[j]] = max(-x[j], 0.0)
        if k == BOX:
            xs[nb + t] = hi[j] - x[j]
            t += 1
    return xs


def recover(bmap: BoundMap, xs, ys):
    """Original x (n0) and the duals y of the original rows (m0) from a standard-form point."""
    xs = np.asarray(xs, np.float64)
    x = np.empty(bmap.n0)
    for j in range(bmap.n0):
        k = bmap.kind[j]
        if k in (LOWER, BOX):
            x[j] = bmap.shift[j] + xs[bmap.col[j]]
        elif k == UPPER:
            x[j] = bmap.shift[j] - xs[bmap.col[j]]
        elif k == FREE:
            x[j] = xs[bmap.col[j]] - xs[bmap.col2[j]]
        else:
            x[j] = bmap.shift[j]
    return x, np.asarray(ys, np.float64)[:bmap.m0].copy()


def free_pairs(bmap: BoundMap):
    """(k, 2) standard-form columns (x+_j, x-_j) of the free variables, in variable order."""
    free = np.flatnonzero(bmap.kind == FREE)
    return np.stack([bmap.col[free], bmap.col2[free]], axis=1).astype(np.int64)


def ipm_bounded(A, b, c, lo, hi, opts=None):
    """Solve min c^T x, A x = b, lo <= x <= hi through the standard form; returns the
    oracle's result dict for the standard form plus x, y and obj in the original space."""
    lp, bmap = standard_form(A, b, c, lo, hi)
    r = ipm(lp, opts if opts is not None else ipm_opts(), pairs=free_pairs(bmap))
    x, y = recover(bmap, r["x"], r["y"])
    out = dict(r)
    out.update(x_std=r["x"], y_std=r["y"], x=x, y=y, obj=float(np.asarray(c, np.float64) @ x), lp=lp, bmap=bmap)
    return out

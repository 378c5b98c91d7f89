"""Seeded synthetic LP generators shared by the tests, the smoke check and the benchmark.

This module only draws random problem data (it contains no step of the interior-point
method, the Krylov solver or the inner iterations).  Every problem is in standard form
``min c^T x  s.t.  A x = b, x >= 0`` with A given as 0-based CSR (sorted, unique column
indices per row), the form assumed by the primal-dual pair of the paper's introduction.

Each generator builds a strictly feasible primal point x0 > 0 and dual point (y0, s0 > 0)
first and forms ``b = A x0`` and ``c = A^T y0 + s0`` from them (or uses a closed-form
construction for the transportation and basis-pursuit families), so that an optimal
solution exists, as the paper assumes.

Workload families (sizes are the defaults; every one takes a seed):

* ``sparse_lp``: random sparse A with a fixed number of nonzeros per column at distinct
  uniform rows, N(0,1) values, plus duplicated rows (rank deficiency), optionally with
  columns scaled by 10^U(-e, e).  Stands in for the sparse Netlib-like problems.
* ``transport_lp``: the node-arc incidence matrix of a complete bipartite
  sources x sinks network (a transportation problem), integer supplies, demands and costs.
  Stands in for the network-flow problems (ken family) of the paper.
* ``basis_pursuit_lp``: A = [Phi, -Phi] with a dense Gaussian Phi, b = Phi x_true for a
  sparse +-1 signal and c = 1.  Stands in for the dense basis-pursuit problems.
* ``serving_mix``: a list of sparse LPs of random sizes with Poisson arrival times.
* ``bounded_lp``: a ``sparse_lp`` matrix with general bounds lo <= x <= hi (lower-bounded,
  boxed, upper-bounded only, free and fixed variables in stated fractions); the LP is
  given in that bounded form, not in standard form.  Stands in for the typical LPs with
  general bounds of the paper's experiments.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class LP:
    """One standard-form LP; A in CSR (row_ptr int64, col_idx int32, val float64)."""

    m: int
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray
    b: np.ndarray
    c: np.ndarray
    name: str = ""
    seed: int = 0
    x0: Optional[np.ndarray] = None
    y0: Optional[np.ndarray] = None
    s0: Optional[np.ndarray] = None
    dense: Optional[np.ndarray] = None  # row-major m x n copy for dense families
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_dense(self) -> np.ndarray:
        if self.dense is not None:
            return self.dense
        A = np.zeros((self.m, self.n))
        for i in range(self.m):
            s, e = self.row_ptr[i], self.row_ptr[i + 1]
            A[i, self.col_idx[s:e]] = self.val[s:e]
        return A


def _csr_from_coo(m: int, n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray):
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int64)
    return row_ptr, cols.astype(np.int32), vals.astype(np.float64)


def csr_matvec(lp: LP, x: np.ndarray) -> np.ndarray:
    """A @ x for a generator's own use (forming b); not part of the method."""
    rows = np.repeat(np.arange(lp.m), np.diff(lp.row_ptr))
    out = np.zeros(lp.m)
    np.add.at(out, rows, lp.val * x[lp.col_idx])
    return out


def csr_rmatvec(lp: LP, y: np.ndarray) -> np.ndarray:
    """A^T @ y for a generator's own use (forming c); not part of the method."""
    rows = np.repeat(np.arange(lp.m), np.diff(lp.row_ptr))
    out = np.zeros(lp.n)
    np.add.at(out, lp.col_idx, lp.val * y[rows])
    return out


def sparse_lp(m_base: int = 198, n: int = 500, nnz_per_col: int = 6, n_dup: int = 2,
              seed: int = 0, col_scale_exp: float = 0.0, name: str = "") -> LP:
    """Random sparse LP: ``m_base`` independent rows plus ``n_dup`` duplicated rows.

    Each column receives ``nnz_per_col`` distinct rows drawn uniformly from the base rows,
    with N(0,1) values.  ``n_dup`` distinct base rows are copied and appended, so
    m = m_base + n_dup and rank(A) <= m_base.  With ``col_scale_exp`` = e > 0 column j is
    multiplied by 10^u_j, u_j ~ U(-e, e), before b and c are formed.  The draw is repeated
    (same generator stream) until no base row is empty.
    """
    rng = np.random.default_rng(seed)
    k = nnz_per_col
    while True:
        # k distinct rows per column: argpartition of uniform keys (vectorised sampling
        # without replacement)
        if m_base <= 4096:
            keys = rng.random((n, m_base))
            rows = np.argpartition(keys, k - 1, axis=1)[:, :k].astype(np.int64)
        else:
            rows = rng.integers(0, m_base, size=(n, k), dtype=np.int64)
            for _ in range(64):
                srt = np.sort(rows, axis=1)
                bad = np.any(srt[:, 1:] == srt[:, :-1], axis=1)
                if not bad.any():
                    break
                rows[bad] = rng.integers(0, m_base, size=(int(bad.sum()), k), dtype=np.int64)
            else:  # pragma: no cover - vanishingly unlikely
                raise RuntimeError("could not draw distinct rows")
        cols = np.repeat(np.arange(n, dtype=np.int64), k)
        rows = rows.reshape(-1)
        vals = rng.standard_normal(n * k)
        counts = np.bincount(rows, minlength=m_base)
        if counts.min() > 0:
            break
    if col_scale_exp > 0:
        u = rng.uniform(-col_scale_exp, col_scale_exp, size=n)
        vals = vals * (10.0 ** u)[cols]
    dup = rng.choice(m_base, size=n_dup, replace=False) if n_dup > 0 else np.zeros(0, np.int64)
    # appended copies of the chosen base rows
    row_list = [rows]
    col_list = [cols]
    val_list = [vals]
    if n_dup > 0:
        # entries of each base row in their original order (stable sort by row)
        order = np.argsort(rows, kind="stable")
        start = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=m_base))])
        for t, r in enumerate(dup):
            sel = order[start[r]:start[r + 1]]
            row_list.append(np.full(sel.size, m_base + t, dtype=np.int64))
            col_list.append(cols[sel])
            val_list.append(vals[sel])
    m = m_base + n_dup
    row_ptr, col_idx, val = _csr_from_coo(m, n, np.concatenate(row_list),
                                          np.concatenate(col_list), np.concatenate(val_list))
    lp = LP(m=m, n=n, row_ptr=row_ptr, col_idx=col_idx, val=val, b=np.zeros(m), c=np.zeros(n),
            name=name or f"sparse_{m}x{n}", seed=seed)
    x0 = rng.uniform(0.5, 1.5, size=n)
    y0 = rng.standard_normal(m)
    s0 = rng.uniform(0.5, 1.5, size=n)
    lp.b = csr_matvec(lp, x0)
    lp.c = csr_rmatvec(lp, y0) + s0
    lp.x0, lp.y0, lp.s0 = x0, y0, s0
    lp.meta = dict(family="sparse", m_base=m_base, nnz_per_col=k, n_dup=n_dup,
                   dup_rows=[int(r) for r in dup], col_scale_exp=col_scale_exp)
    return lp


def transport_lp(n_src: int = 300, n_snk: int = 300, seed: int = 1) -> LP:
    """Transportation LP on the complete bipartite network sources x sinks.

    Arc (i, j) is column i*n_snk + j with +1 in row i (supply node) and +1 in row
    n_src + j (demand node); rows are the flow-conservation equalities
    sum_j x_ij = supply_i and sum_i x_ij = demand_j.  Supplies and the first
    n_snk - 1 demands are U{50..150}; the last demand balances the totals and the
    demand draw is repeated until it is >= 1.  Costs are U{1..100}.  rank(A) = m - 1.
    """
    rng = np.random.default_rng(seed)
    supply = rng.integers(50, 151, size=n_src).astype(np.float64)
    for _ in range(10000):
        dem = rng.integers(50, 151, size=n_snk - 1).astype(np.float64)
        last = supply.sum() - dem.sum()
        if last >= 1:
            break
    else:
        raise ValueError("supplies and demands cannot be balanced for these sizes")
    demand = np.concatenate([dem, [last]])
    cost = rng.integers(1, 101, size=n_src * n_snk).astype(np.float64)
    m, n = n_src + n_snk, n_src * n_snk
    arcs = np.arange(n, dtype=np.int64)
    src = arcs // n_snk
    snk = arcs % n_snk
    rows = np.concatenate([src, n_src + snk])
    cols = np.concatenate([arcs, arcs])
    vals = np.ones(2 * n)
    row_ptr, col_idx, val = _csr_from_coo(m, n, rows, cols, vals)
    lp = LP(m=m, n=n, row_ptr=row_ptr, col_idx=col_idx, val=val,
            b=np.concatenate([supply, demand]), c=cost, name=f"transport_{n_src}x{n_snk}", seed=seed)
    lp.meta = dict(family="transport", n_src=n_src, n_snk=n_snk)
    return lp


def basis_pursuit_lp(m: int = 1024, N: int = 8192, k: int = 64, seed: int = 2) -> LP:
    """Basis-pursuit LP  min 1^T (u+v)  s.t.  [Phi, -Phi][u; v] = Phi x_true, u, v >= 0.

    Phi_ij ~ N(0,1)/sqrt(m); x_true has k entries of +-1 at random positions.  A is
    stored dense (row-major) and also as CSR with every entry present.
    """
    rng = np.random.default_rng(seed)
    Phi = rng.standard_normal((m, N)) / np.sqrt(m)
    pos = rng.choice(N, size=k, replace=False)
    xt = np.zeros(N)
    xt[pos] = rng.choice([-1.0, 1.0], size=k)
    A = np.concatenate([Phi, -Phi], axis=1)
    b = Phi @ xt
    n = 2 * N
    row_ptr = (np.arange(m + 1, dtype=np.int64) * n)
    col_idx = np.tile(np.arange(n, dtype=np.int32), m)
    lp = LP(m=m, n=n, row_ptr=row_ptr, col_idx=col_idx, val=A.reshape(-1).copy(), b=b,
            c=np.ones(n), name=f"basis_pursuit_{m}x{n}", seed=seed, dense=A)
    lp.meta = dict(family="basis_pursuit", N=N, k=k, x_true=xt, support=np.sort(pos))
    return lp


def tiny_lp(m: int, n: int, seed: int, density: float = 0.6, n_dup: int = 0) -> LP:
    """Tiny dense-ish LP for brute-force checks (m <= 6, n <= 12)."""
    rng = np.random.default_rng(seed)
    while True:
        A = rng.standard_normal((m, n)) * (rng.random((m, n)) < density)
        if np.all(np.abs(A).sum(axis=1) > 0) and np.all(np.abs(A).sum(axis=0) > 0):
            break
    if n_dup:
        A = np.concatenate([A, A[:n_dup]], axis=0)
    mm = A.shape[0]
    x0 = rng.uniform(0.5, 1.5, size=n)
    y0 = rng.standard_normal(mm)
    s0 = rng.uniform(0.5, 1.5, size=n)
    return from_dense(A, A @ x0, A.T @ y0 + s0, name=f"tiny_{mm}x{n}_{seed}", seed=seed,
                      x0=x0, y0=y0, s0=s0)


def from_dense(A: np.ndarray, b: np.ndarray, c: np.ndarray, name: str = "", seed: int = 0,
               x0=None, y0=None, s0=None) -> LP:
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    rows, cols = np.nonzero(A)
    row_ptr, col_idx, val = _csr_from_coo(m, n, rows.astype(np.int64), cols.astype(np.int64), A[rows, cols])
    return LP(m=m, n=n, row_ptr=row_ptr, col_idx=col_idx, val=val, b=np.asarray(b, np.float64),
              c=np.asarray(c, np.float64), name=name, seed=seed, x0=x0, y0=y0, s0=s0)


def config(idx: int) -> LP:
    """The five workload configurations (indices 0-4; 4 returns the first serving LP)."""
    if idx == 0:
        return sparse_lp(198, 500, 6, 2, seed=0, name="sparse_200x500")
    if idx == 1:
        return transport_lp(300, 300, seed=1)
    if idx == 2:
        return basis_pursuit_lp(1024, 8192, 64, seed=2)
    if idx == 3:
        return sparse_lp(119_900, 434_580, 8, 100, seed=3, col_scale_exp=3.0, name="sparse_120000x434580")
    if idx == 4:
        return serving_mix(1)[0][0]
    raise ValueError(idx)


def streaming_lp(scale: int = 10, seed: int = 3) -> LP:
    """The config-3 generator scaled ``scale`` times in m and n (8 nonzeros per column,
    columns scaled by 10^U(-3,3), 100 * scale duplicated rows): an instance whose matrix
    does not fit the 256 MB Infinity Cache, for kernel bandwidth measurements."""
    return sparse_lp(119_900 * scale, 434_580 * scale, 8, 100 * scale, seed=seed, col_scale_exp=3.0,
                     name=f"sparse_{120_000 * scale}x{434_580 * scale}")


def serving_mix(count: int = 256, m_lo: int = 200, m_hi: int = 20_000, seed0: int = 1000,
                rate: float = 1.0, arrival_seed: int = 4242):
    """``count`` sparse LPs (instance i uses seed seed0+i) with Poisson arrival times.

    m ~ U{m_lo..m_hi} (including 2 duplicated rows), n = round(m * U(2, 4)), nonzeros per
    column ~ U{4..10}.  Arrival gaps are exponential with the given rate (per second).
    Returns (list of LP, arrival times in seconds from 0).
    """
    lps: List[LP] = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        m = int(rng.integers(m_lo, m_hi + 1))
        n = int(round(m * rng.uniform(2.0, 4.0)))
        k = int(rng.integers(4, 11))
        lps.append(sparse_lp(m - 2, n, k, 2, seed=seed0 + i, name=f"serve_{i}_{m}x{n}"))
    arng = np.random.default_rng(arrival_seed)
    gaps = arng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    return lps, arrivals


def bounded_lp(m_base: int = 198, n: int = 500, nnz_per_col: int = 6, n_dup: int = 2, seed: int = 0,
               frac_box: float = 0.3, frac_upper: float = 0.1, frac_free: float = 0.1,
               frac_fixed: float = 0.02):
    """``min c^T x  s.t.  A x = b, lo <= x <= hi`` on the matrix of ``sparse_lp``.

    Returns ``(lp, lo, hi)``; ``lp`` carries A, b and c of the bounded problem (its ``b``
    and ``c`` are those of this LP, not of a standard form).  Variable kinds are drawn in
    the stated fractions, the rest lower-bounded: lower l ~ U(-2, 2); box l ~ U(-2, 2),
    u = l + U(1, 3); upper-only u ~ U(-2, 2); free; fixed l = u ~ U(-1, 1).  A strictly
    interior x0 (fixed variables at their value) gives b = A x0, and a dual point y0 with
    reduced costs of the right sign (> 0 for lower-bounded, < 0 for upper-only, 0 for
    free, any for box and fixed) gives c, so a bounded optimum exists.  A row whose
    variables would all be fixed gets one of them boxed instead.
    """
    lp = sparse_lp(m_base, n, nnz_per_col, n_dup, seed=seed, name=f"bounded_{m_base + n_dup}x{n}")
    rng = np.random.default_rng(seed + 7919)
    kinds = np.zeros(n, np.int64)   # 0 lower, 1 box, 2 upper, 3 free, 4 fixed
    order = rng.permutation(n)
    counts = [int(round(f * n)) for f in (frac_box, frac_upper, frac_free, frac_fixed)]
    start = 0
    for k, cnt in zip((1, 2, 3, 4), counts):
        kinds[order[start:start + cnt]] = k
        start += cnt
    for i in range(lp.m):
        cols = lp.col_idx[lp.row_ptr[i]:lp.row_ptr[i + 1]]
        if np.all(kinds[cols] == 4):
            kinds[cols[0]] = 1
    lo = np.full(n, -np.inf)
    hi = np.full(n, np.inf)
    x0 = np.zeros(n)
    r = np.zeros(n)
    for j in range(n):
        k = kinds[j]
        if k == 0:
            lo[j] = rng.uniform(-2, 2)
            x0[j] = lo[j] + rng.uniform(0.5, 1.5)
            r[j] = rng.uniform(0.5, 1.5)
        elif k == 1:
            lo[j] = rng.uniform(-2, 2)
            hi[j] = lo[j] + rng.uniform(1, 3)
            x0[j] = lo[j] + (hi[j] - lo[j]) * rng.uniform(0.25, 0.75)
            r[j] = rng.uniform(-1, 1)
        elif k == 2:
            hi[j] = rng.uniform(-2, 2)
            x0[j] = hi[j] - rng.uniform(0.5, 1.5)
            r[j] = -rng.uniform(0.5, 1.5)
        elif k == 3:
            x0[j] = rng.standard_normal()
        else:
            lo[j] = hi[j] = rng.uniform(-1, 1)
            x0[j] = lo[j]
            r[j] = rng.standard_normal()
    y0 = rng.standard_normal(lp.m)
    lp.b = csr_matvec(lp, x0)
    lp.c = csr_rmatvec(lp, y0) + r
    lp.x0, lp.y0, lp.s0 = x0, y0, None
    lp.meta = dict(lp.meta, family="bounded", kinds=[int(np.sum(kinds == k)) for k in range(5)])
    return lp, lo, hi

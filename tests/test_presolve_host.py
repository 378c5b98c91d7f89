"""Presolve of dependent rows (``lp_presolve_rows``, host only): rows that are scalar
multiples of an earlier row.  Pinned against hand-built cases and against linear algebra:
on the generator's sparse family every dependency is a duplicated row, so the kept rows
number rank(A) and span the same row space; the reduced LP has the optimum of the full one
(HiGHS on both)."""
import numpy as np
import pytest
from scipy.optimize import linprog

import paper_1604_07491_amd as lpk
from paper_1604_07491_amd import synth


def _keep(A, b, tol=1e-12):
    lp = synth.from_dense(np.asarray(A, float), np.asarray(b, float), np.ones(np.shape(A)[1]))
    return lpk.lp_presolve_rows(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.val, lp.b, tol)


def test_hand_built_multiples_and_duplicates():
    A = [[1.0, 2.0, 0.0, 0.0],
         [2.0, 4.0, 0.0, 0.0],     # 2 x row 0
         [0.0, 1.0, 1.0, 0.0],
         [1.0, 2.0, 0.0, 0.0],     # row 0 again
         [-0.5, -1.0, 0.0, 0.0],   # -0.5 x row 0
         [1.0, 2.0, 0.0, 1.0]]     # same leading entries, other pattern
    b = [3.0, 6.0, 1.0, 3.0, -1.5, 4.0]
    assert list(_keep(A, b)) == [True, False, True, False, False, True]
    # a contradicting right-hand side makes the LP infeasible
    with pytest.raises(lpk.LpError) as e:
        _keep(A, [3.0, 6.5, 1.0, 3.0, -1.5, 4.0])
    assert e.value.status == lpk.LP_EINVAL
    # tolerance: ratios equal to 1e-9 are multiples at tol 1e-8, not at tol 0
    A2 = [[1.0, 3.0], [2.0, 6.0 * (1 + 1e-9)]]
    assert list(_keep(A2, [1.0, 2.0], 1e-8)) == [True, False]
    assert list(_keep(A2, [1.0, 2.0], 0.0)) == [True, True]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_duplicated_rows_of_the_sparse_family(seed):
    lp = synth.sparse_lp(120, 300, 5, 4, seed=seed)
    keep = lpk.lp_presolve_rows(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.val, lp.b)
    A = lp.to_dense()
    r = np.linalg.matrix_rank(A)
    assert keep.sum() == r == 120
    assert np.linalg.matrix_rank(A[keep]) == r
    # every dropped row is one of the appended copies
    assert keep[:120].all() and not keep[120:].any()
    ref = linprog(lp.c, A_eq=A, b_eq=lp.b, bounds=[(0, None)] * lp.n, method="highs")
    red = linprog(lp.c, A_eq=A[keep], b_eq=lp.b[keep], bounds=[(0, None)] * lp.n, method="highs")
    assert ref.status == red.status == 0
    assert abs(ref.fun - red.fun) <= 1e-9 * max(1.0, abs(ref.fun))


def test_transport_dependency_is_left_in_place():
    """The transportation matrix's dependency (supply rows and demand rows sum to the same
    vector) involves every row; no row is a multiple of another."""
    lp = synth.transport_lp(12, 10, seed=3)
    keep = lpk.lp_presolve_rows(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.val, lp.b)
    assert keep.all()
    assert np.linalg.matrix_rank(lp.to_dense()) == lp.m - 1


def test_invalid_arguments():
    lp = synth.sparse_lp(20, 50, 3, 1, seed=0)
    with pytest.raises(lpk.LpError):
        lpk.lp_presolve_rows(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.val, lp.b, -1.0)
    b = lp.b.copy()
    b[0] = np.nan
    with pytest.raises(lpk.LpError):
        lpk.lp_presolve_rows(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.val, b)


# ---- general dependent rows (lp_presolve_dependent_rows) ---------------------------------

def _rank_increments(A, tol=1e-9):
    """keep[k] by brute force: row k raises the rank of the rows before it (SVD rank)."""
    keep, r = [], 0
    for k in range(A.shape[0]):
        rk = np.linalg.matrix_rank(A[:k + 1], tol=tol * max(1.0, np.abs(A[:k + 1]).max()))
        keep.append(rk > r)
        r = rk
    return np.array(keep)


def _planted(seed, m0=40, n=90, extra=20, per=(2, 4)):
    """A sparse LP whose extra rows are random combinations of 2-4 earlier rows (b combined
    alike, so the LP stays feasible), interleaved at random positions, plus a duplicate."""
    base = synth.sparse_lp(m0, n, 4, 0, seed=seed)
    A = base.to_dense()
    b = base.b.copy()
    rng = np.random.default_rng(100 + seed)
    rows, rhs = [A[i] for i in range(m0)], [b[i] for i in range(m0)]
    for _ in range(extra):
        pos = int(rng.integers(per[1], len(rows) + 1))
        idx = rng.choice(pos, size=int(rng.integers(per[0], per[1] + 1)), replace=False)
        w = rng.normal(size=len(idx))
        rows.insert(pos, sum(wi * rows[i] for wi, i in zip(w, idx)))
        rhs.insert(pos, sum(wi * rhs[i] for wi, i in zip(w, idx)))
    rows.append(rows[3].copy())
    rhs.append(rhs[3])
    return synth.from_dense(np.array(rows), np.array(rhs), base.c), base


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_general_dependencies_are_the_rank_increments(seed):
    """The kept rows are exactly those that raise the rank of the rows before them (numpy
    SVD rank), and they number rank(A)."""
    lp, _ = _planted(seed)
    keep = lpk.lp_presolve_dependent_rows(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.val, lp.b)
    A = lp.to_dense()
    assert np.array_equal(keep, _rank_increments(A))
    assert keep.sum() == np.linalg.matrix_rank(A) == 40
    # the pairwise pass finds only the duplicate
    pair = lpk.lp_presolve_rows(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.val, lp.b)
    assert (~pair).sum() == 1 and not keep[~pair].any()


def test_transport_dependency_is_found():
    """The transportation matrix has rank m - 1: the supply rows and the demand rows sum to
    the same vector.  In row order the last demand row is the dependent one."""
    for ns, nt in ((12, 10), (7, 7), (20, 3)):
        lp = synth.transport_lp(ns, nt, seed=3)
        keep = lpk.lp_presolve_dependent_rows(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.val, lp.b)
        assert keep.sum() == lp.m - 1 == np.linalg.matrix_rank(lp.to_dense())
        assert not keep[-1] and keep[:-1].all()
        assert np.array_equal(keep, _rank_increments(lp.to_dense()))


def test_general_presolve_keeps_the_optimum():
    """HiGHS reaches the same optimum on the reduced LP as on the full one."""
    for seed in (0, 1):
        lp, _ = _planted(seed)
        keep = lpk.lp_presolve_dependent_rows(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.val, lp.b)
        A = lp.to_dense()
        ref = linprog(lp.c, A_eq=A, b_eq=lp.b, bounds=[(0, None)] * lp.n, method="highs")
        red = linprog(lp.c, A_eq=A[keep], b_eq=lp.b[keep], bounds=[(0, None)] * lp.n, method="highs")
        assert ref.status == red.status == 0
        assert abs(ref.fun - red.fun) <= 1e-8 * max(1.0, abs(ref.fun))


def test_general_presolve_infeasible_and_tolerance():
    lp, _ = _planted(0)
    A = lp.to_dense()
    dep = np.flatnonzero(~_rank_increments(A))
    b = lp.b.copy()
    b[dep[0]] += 1e-3 * max(1.0, abs(b[dep[0]]))       # a dependent row with another rhs
    with pytest.raises(lpk.LpError) as e:
        lpk.lp_presolve_dependent_rows(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.val, b)
    assert e.value.status == lpk.LP_EINVAL
    # a combination perturbed by 1e-6 relative is independent at tol 1e-9, dependent at 1e-4
    A2 = A.copy()
    k = dep[0]
    A2[k] = A2[k] * (1 + 1e-6 * np.sign(A2[k]))
    lp2 = synth.from_dense(A2, lp.b, lp.c)
    k2 = lpk.lp_presolve_dependent_rows(lp2.m, lp2.n, lp2.row_ptr, lp2.col_idx, lp2.val, lp2.b, 1e-9)
    assert k2[k]
    k4 = lpk.lp_presolve_dependent_rows(lp2.m, lp2.n, lp2.row_ptr, lp2.col_idx, lp2.val, lp2.b, 1e-4)
    assert not k4[k]
    with pytest.raises(lpk.LpError):
        lpk.lp_presolve_dependent_rows(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.val, lp.b, -1.0)


def test_general_presolve_at_size():
    """Transportation 300 x 300 (m = 600, 180,000 nonzeros) and the sparse 200 x 500 family:
    the dependency search runs in well under a second and finds rank(A) rows."""
    import time
    lp = synth.transport_lp(300, 300, seed=1)
    t = time.perf_counter()
    keep = lpk.lp_presolve_dependent_rows(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.val, lp.b)
    assert time.perf_counter() - t < 2.0
    assert keep.sum() == 599 and not keep[-1]
    lp = synth.sparse_lp(198, 500, 6, 2, seed=0)
    keep = lpk.lp_presolve_dependent_rows(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.val, lp.b)
    assert keep.sum() == np.linalg.matrix_rank(lp.to_dense()) == 198


def test_general_presolve_dense_fallback():
    """A random sparse LP of 2,000 rows fills under elimination past the cap, so the search
    runs on the dense Gram matrix: the 10 planted combinations (of 3 earlier rows each) are
    exactly the rows dropped, and their right-hand sides pass."""
    import scipy.sparse as sp
    base = synth.sparse_lp(2000, 5600, 6, 0, seed=11)
    A = sp.csr_matrix((base.val, base.col_idx, base.row_ptr), shape=(base.m, base.n))
    rng = np.random.default_rng(5)
    rows, rhs, planted = [A[i] for i in range(base.m)], list(base.b), []
    for _ in range(10):
        pos = int(rng.integers(100, len(rows) + 1))
        idx = rng.choice(pos, 3, replace=False)
        w = rng.normal(size=3)
        rows.insert(pos, sum(wi * rows[i] for wi, i in zip(w, idx)))
        rhs.insert(pos, sum(wi * rhs[i] for wi, i in zip(w, idx)))
        planted = [p + (p >= pos) for p in planted] + [pos]
    M = sp.vstack(rows).tocsr()
    M.sort_indices()
    keep = lpk.lp_presolve_dependent_rows(M.shape[0], M.shape[1], M.indptr.astype(np.int64), M.indices,
                                          M.data, np.array(rhs))
    assert sorted(np.flatnonzero(~keep)) == sorted(planted)
    bad = np.array(rhs)
    bad[planted[0]] += 1.0
    with pytest.raises(lpk.LpError):
        lpk.lp_presolve_dependent_rows(M.shape[0], M.shape[1], M.indptr.astype(np.int64), M.indices, M.data, bad)

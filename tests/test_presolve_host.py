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

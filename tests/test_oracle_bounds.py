"""Pins of the oracle's bounded-variable transform (the LIPSOL-style reduction to the
standard form used for the typical LPs of Sec. 4.3), against its definition (a hand-built
example, the inverse map of feasible points) and against an independent LP solver (HiGHS
through scipy.optimize.linprog) on the original bounded problems."""
import numpy as np
import pytest
from scipy.optimize import linprog

import oracle
from oracle import bounds
from paper_1604_07491_amd import synth

INF = np.inf


def test_hand_built_example_has_the_stated_layout():
    # x0 lower [1, inf), x1 box [-1, 2], x2 upper (-inf, 3], x3 free, x4 fixed at 0.5
    A = np.array([[1.0, 2.0, 3.0, 4.0, 5.0],
                  [0.0, 1.0, 0.0, -1.0, 2.0]])
    b = np.array([10.0, 1.0])
    c = np.array([1.0, -2.0, 3.0, -4.0, 5.0])
    lo = np.array([1.0, -1.0, -INF, -INF, 0.5])
    hi = np.array([INF, 2.0, 3.0, INF, 0.5])
    lp, bm = bounds.standard_form(A, b, c, lo, hi)
    # columns: x0', x1', x2', x3+ (kept, in order), x3- (free part), w1 (slack of x1)
    expect_A = np.array([[1.0, 2.0, -3.0, 4.0, -4.0, 0.0],
                         [0.0, 1.0, 0.0, -1.0, 1.0, 0.0],
                         [0.0, 1.0, 0.0, 0.0, 0.0, 1.0]])
    np.testing.assert_array_equal(lp.dense_A, expect_A)
    # b' = b - A (1, -1, 3, 0, 0.5); box row: u - l = 3
    np.testing.assert_array_equal(lp.b, [10.0 - (1 - 2 + 9 + 2.5), 1.0 - (-1 + 1.0), 3.0])
    np.testing.assert_array_equal(lp.c, [1.0, -2.0, -3.0, -4.0, 4.0, 0.0])
    assert bm.offset == 1.0 * 1 + (-2.0) * (-1) + 3.0 * 3 + 5.0 * 0.5
    assert list(bm.kind) == [bounds.LOWER, bounds.BOX, bounds.UPPER, bounds.FREE, bounds.FIXED]
    assert (lp.m, lp.n) == (3, 6)
    # CSR rows hold ascending columns
    for i in range(lp.m):
        seg = lp.col_idx[lp.row_ptr[i]:lp.row_ptr[i + 1]]
        assert np.all(np.diff(seg) > 0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_feasible_points_map_to_feasible_points(seed):
    lp0, lo, hi = synth.bounded_lp(28, 80, 4, 2, seed=seed)
    A = lp0.to_dense()
    lp, bm = bounds.standard_form(A, lp0.b, lp0.c, lo, hi)
    x = lp0.x0
    xs = bounds.to_standard_point(bm, x, hi)
    assert np.all(xs >= 0)
    np.testing.assert_allclose(lp.dense_A @ xs, lp.b, rtol=1e-12, atol=1e-12 * np.abs(lp0.b).max())
    assert abs(lp.c @ xs + bm.offset - lp0.c @ x) <= 1e-12 * (1 + abs(lp0.c @ x))
    xr, _ = bounds.recover(bm, xs, np.zeros(lp.m))
    np.testing.assert_allclose(xr, x, rtol=0, atol=1e-14 * (1 + np.abs(x).max()))


def test_plain_nonnegativity_is_the_identity_transform():
    lp0 = synth.sparse_lp(28, 80, 4, 2, seed=4)
    A = lp0.to_dense()
    lp, bm = bounds.standard_form(A, lp0.b, lp0.c, np.zeros(lp0.n), np.full(lp0.n, INF))
    np.testing.assert_array_equal(lp.dense_A, A)
    np.testing.assert_array_equal(lp.b, lp0.b)
    np.testing.assert_array_equal(lp.c, lp0.c)
    assert bm.offset == 0.0


def _highs(A, b, c, lo, hi):
    bnds = [(None if not np.isfinite(l) else l, None if not np.isfinite(u) else u) for l, u in zip(lo, hi)]
    r = linprog(c, A_eq=A, b_eq=b, bounds=bnds, method="highs")
    assert r.status == 0, r.message
    return r


@pytest.mark.parametrize("shape", [(28, 80, 4, 2, 0), (60, 150, 5, 0, 1), (198, 500, 6, 2, 2)])
def test_bounded_optimum_matches_highs(shape):
    mb, n, k, dup, seed = shape
    lp0, lo, hi = synth.bounded_lp(mb, n, k, dup, seed=seed)
    A = lp0.to_dense()
    ref = _highs(A, lp0.b, lp0.c, lo, hi)
    r = bounds.ipm_bounded(A, lp0.b, lp0.c, lo, hi)
    assert r["status"] == oracle.OK
    assert abs(r["obj"] - ref.fun) <= 1e-7 * max(1.0, abs(ref.fun))
    x = r["x"]
    scale = 1.0 + np.abs(x).max()
    assert np.all(x >= lo - 1e-7 * scale) and np.all(x <= hi + 1e-7 * scale)
    assert np.linalg.norm(A @ x - lp0.b) <= 1e-7 * (1 + np.linalg.norm(lp0.b))
    # the standard form's objective plus the constant is the original objective
    assert abs(r["pobj"] + r["bmap"].offset - r["obj"]) <= 1e-8 * max(1.0, abs(r["obj"]))


@pytest.mark.parametrize("seed", [6, 8, 43, 56, 60])
def test_split_free_variables_reach_the_highs_optimum(seed):
    """LPs of the 200 x 500 bounded family on which the split free variables grew without
    bound (gamma_rel 1e18 and worse after 99 steps) before the pairs were recentred."""
    lp0, lo, hi = synth.bounded_lp(198, 500, 6, 2, seed=seed)
    A = lp0.to_dense()
    ref = _highs(A, lp0.b, lp0.c, lo, hi)
    r = bounds.ipm_bounded(A, lp0.b, lp0.c, lo, hi)
    assert r["status"] == oracle.OK and r["iters"] <= 30
    assert abs(r["obj"] - ref.fun) <= 1e-7 * max(1.0, abs(ref.fun))
    # a split pair keeps its smaller part at most (1 + |x|) / 2 (recentred after each step)
    xs = r["x_std"]
    pr = bounds.free_pairs(r["bmap"])
    a, b = xs[pr[:, 0]], xs[pr[:, 1]]
    assert np.all(np.minimum(a, b) <= 0.5 * (1 + np.abs(a - b)) * (1 + 1e-12))


def test_invalid_bounds_are_rejected():
    A = np.array([[1.0, 1.0]])
    with pytest.raises(ValueError):
        bounds.standard_form(A, [1.0], [1.0, 1.0], [0.0, 2.0], [1.0, 1.0])      # l > u
    with pytest.raises(ValueError):
        bounds.standard_form(A, [1.0], [1.0, 1.0], [0.0, np.nan], [1.0, 1.0])
    with pytest.raises(ValueError):
        bounds.standard_form(A, [1.0], [1.0, 1.0], [0.0, INF], [1.0, INF])      # l = +inf
    with pytest.raises(ValueError):                                             # every variable fixed
        bounds.standard_form(A, [1.0], [1.0, 1.0], [0.5, 0.5], [0.5, 0.5])

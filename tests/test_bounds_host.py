"""The library's bounded-variable reduction (``lp_bounds_standard_form``, host only) against
the oracle's, which is pinned in test_oracle_bounds.py.  The structure and values of the
standard form must be identical; b' = b - A s is summed in a different order on the two
sides, so it is compared to 1e-14 relative."""
import numpy as np
import pytest

import paper_1604_07491_amd as lpk
from oracle import bounds
from paper_1604_07491_amd import synth

INF = np.inf


def _both(A_lp, lo, hi):
    sf = lpk.lp_bounds_standard_form(A_lp.m, A_lp.n, A_lp.row_ptr, A_lp.col_idx, A_lp.val, A_lp.b, A_lp.c, lo, hi)
    olp, bm = bounds.standard_form(A_lp.to_dense(), A_lp.b, A_lp.c, lo, hi)
    return sf, olp, bm


@pytest.mark.parametrize("shape", [(28, 80, 4, 2, 0), (60, 150, 5, 0, 1), (198, 500, 6, 2, 2)])
def test_standard_form_equals_the_oracles(shape):
    mb, n, k, dup, seed = shape
    lp0, lo, hi = synth.bounded_lp(mb, n, k, dup, seed=seed)
    sf, olp, bm = _both(lp0, lo, hi)
    assert (sf["m"], sf["n"]) == (olp.m, olp.n)
    np.testing.assert_array_equal(sf["row_ptr"], olp.row_ptr)
    np.testing.assert_array_equal(sf["col_idx"], olp.col_idx)
    np.testing.assert_array_equal(sf["val"], olp.val)
    np.testing.assert_array_equal(sf["c"], olp.c)
    np.testing.assert_allclose(sf["b"], olp.b, rtol=1e-14, atol=1e-14 * np.abs(lp0.b).max())
    assert abs(sf["offset"] - bm.offset) <= 1e-13 * (1 + abs(bm.offset))


def test_hand_built_example():
    A = np.array([[1.0, 2.0, 3.0, 4.0, 5.0],
                  [0.0, 1.0, 0.0, -1.0, 2.0]])
    lp0 = synth.from_dense(A, np.array([10.0, 1.0]), np.array([1.0, -2.0, 3.0, -4.0, 5.0]))
    lo = np.array([1.0, -1.0, -INF, -INF, 0.5])
    hi = np.array([INF, 2.0, 3.0, INF, 0.5])
    sf, olp, bm = _both(lp0, lo, hi)
    dense = np.zeros((sf["m"], sf["n"]))
    for i in range(sf["m"]):
        s, e = sf["row_ptr"][i], sf["row_ptr"][i + 1]
        dense[i, sf["col_idx"][s:e]] = sf["val"][s:e]
    np.testing.assert_array_equal(dense, olp.dense_A)
    np.testing.assert_array_equal(sf["b"], olp.b)


def test_invalid_bounds_are_rejected_on_the_host():
    A = np.array([[1.0, 1.0]])
    lp0 = synth.from_dense(A, np.array([1.0]), np.array([1.0, 1.0]))
    for lo, hi in (([0.0, 2.0], [1.0, 1.0]), ([0.0, np.nan], [1.0, 1.0]), ([0.0, INF], [1.0, INF]),
                   ([0.0, 0.0], [1.0, -INF]), ([0.5, 0.5], [0.5, 0.5])):
        with pytest.raises(lpk.LpError) as e:
            lpk.lp_bounds_standard_form(1, 2, lp0.row_ptr, lp0.col_idx, lp0.val, lp0.b, lp0.c, lo, hi)
        assert e.value.status == lpk.LP_EINVAL


def test_bounded_create_checks_bounds_before_the_device():
    A = np.array([[1.0, 1.0]])
    lp0 = synth.from_dense(A, np.array([1.0]), np.array([1.0, 1.0]))
    with pytest.raises(lpk.LpError) as e:
        lpk.from_bounded_lp(lp0, np.array([0.0, 2.0]), np.array([1.0, 1.0]))
    assert e.value.status == lpk.LP_EINVAL
    import torch
    if not torch.cuda.is_available():
        with pytest.raises(lpk.LpError) as e:
            lpk.from_bounded_lp(lp0, np.array([0.0, -1.0]), np.array([1.0, 1.0]))
        assert e.value.status == lpk.LP_EDEVICE

"""Pins of the oracle's multiple centrality correctors (the multi-corrector interior-point
framework the paper contrasts with its single corrector), against closed forms, a dense
direct solve of the corrector's Newton system and an independent LP solver (HiGHS)."""
import numpy as np
import pytest
from scipy.optimize import linprog

import oracle
from paper_1604_07491_amd import synth


def test_target_moves_products_into_the_box():
    smu = 2.0
    x = np.array([1.0, 1.0, 1.0, 1.0, 4.0])
    s = np.array([0.05, 1.0, 30.0, 100.0, 1.0])
    z = np.zeros(5)
    r = oracle.centrality_target(x, s, z, z, 0.5, 0.5, smu)
    # products 0.05 (below 0.2 -> +0.15), 1 (inside -> 0), 30 (above 20 -> -10),
    # 100 (above: 20 - 100 = -80, capped at -20), 4 (inside -> 0)
    np.testing.assert_array_equal(r, [0.2 - 0.05, 0.0, 20.0 - 30.0, -20.0, 0.0])
    # the trial point moves along (dx, ds) with separate step lengths
    dx = np.array([2.0, 0, 0, 0, 0])
    ds = np.array([0.0, 0, 0, 0, 4.0])
    r = oracle.centrality_target(x, s, dx, ds, 0.5, 0.25, smu)
    assert r[0] == pytest.approx(0.2 - 2.0 * 0.05)       # (1 + 1)(0.05) = 0.1 -> 0.2
    assert r[4] == pytest.approx(0.0)                     # 4 * (1 + 1) = 8, inside


@pytest.mark.parametrize("seed", [0, 1])
def test_direction_solves_the_newton_system(seed):
    lp = synth.sparse_lp(28, 80, 4, 0, seed=seed)
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.1, 2.0, lp.n)
    s = rng.uniform(0.1, 2.0, lp.n)
    r = rng.standard_normal(lp.n)
    dx, dy, ds, info = oracle.centrality_direction(lp, x, s, r, 1e-13)
    A = lp.to_dense()
    m, n = A.shape
    # dense direct solve of  A dx = 0,  A^T dy + ds = 0,  S dx + X ds = r  (full row rank)
    K = np.zeros((m + 2 * n, 2 * n + m))
    K[:m, :n] = A
    K[m:m + n, n:n + m] = A.T
    K[m:m + n, n + m:] = np.eye(n)
    K[m + n:, :n] = np.diag(s)
    K[m + n:, n + m:] = np.diag(x)
    rhs = np.concatenate([np.zeros(m + n), r])
    sol = np.linalg.solve(K, rhs)
    np.testing.assert_allclose(dx, sol[:n], rtol=1e-8, atol=1e-9 * np.abs(sol[:n]).max())
    np.testing.assert_allclose(ds, sol[n + m:], rtol=1e-8, atol=1e-9 * np.abs(sol[n + m:]).max())
    np.testing.assert_allclose(A.T @ dy, A.T @ sol[n:n + m], rtol=1e-8, atol=1e-9)
    assert not info["failed"]


def test_zero_correctors_is_mehrotras_method():
    lp = synth.sparse_lp(60, 150, 5, 0, seed=3)
    a = oracle.ipm(lp)
    b = oracle.ipm(lp, oracle.ipm_opts(max_correctors=0))
    assert a["iters"] == b["iters"]
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["y"], b["y"])
    assert all(L["correctors"] == 0 for L in a["log"])


def _highs(lp):
    r = linprog(lp.c, A_eq=lp.to_dense(), b_eq=lp.b, bounds=[(0, None)] * lp.n, method="highs")
    assert r.status == 0
    return r.fun


@pytest.mark.parametrize("K", [1, 2, 3])
def test_correctors_reach_the_highs_optimum_in_fewer_steps(K):
    its0, itsk = 0, 0
    for seed in range(4):
        lp = synth.sparse_lp(60, 150, 5, 1, seed=seed)
        ref = _highs(lp)
        o0 = oracle.ipm(lp)
        ok = oracle.ipm(lp, oracle.ipm_opts(max_correctors=K))
        assert ok["status"] == oracle.OK
        assert abs(ok["pobj"] - ref) <= 1e-7 * max(1.0, abs(ref))
        assert all(0 <= L["correctors"] <= K for L in ok["log"])
        assert sum(L["correctors"] for L in ok["log"]) > 0
        its0 += o0["iters"]
        itsk += ok["iters"]
    assert itsk < its0

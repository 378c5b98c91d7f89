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


def _mehrotra_step_dense(A, b, c, x, y, s, eta=0.9995, phi=1e-5, sigma_max=0.208, bt=0.95, max_bt=200):
    """One step of Mehrotra's predictor-corrector method (Sec. 2.1) from dense Newton solves
    of the full system (eq. SE1): the predictor with right-hand side (r_p, r_d, -XSe), step
    lengths by the ratio test (eq. steplength), sigma from mu_af (or 10 Gamma late), the
    corrector with (0, 0, sigma mu e - dX_af dS_af e), the sum, back-tracking to the
    centrality condition, the update."""
    m, n = A.shape
    rp = b - A @ x
    rd = c - A.T @ y - s
    mu = x @ s / n
    gam = max(mu, np.linalg.norm(rp) / max(np.linalg.norm(b), 1.0), np.linalg.norm(rd) / max(np.linalg.norm(c), 1.0))
    K = np.zeros((m + 2 * n, 2 * n + m))
    K[:m, :n] = A
    K[m:m + n, n:n + m] = A.T
    K[m:m + n, n + m:] = np.eye(n)
    K[m + n:, :n] = np.diag(s)
    K[m + n:, n + m:] = np.diag(x)

    def newton(r1, r2, r3):
        z = np.linalg.solve(K, np.concatenate([r1, r2, r3]))
        return z[:n], z[n:n + m], z[n + m:]

    def ratio(v, dv):
        neg = dv < 0
        return min(1.0, eta * np.min(-v[neg] / dv[neg])) if neg.any() else 1.0

    dx, dy, ds = newton(rp, rd, -x * s)
    ap, ad = ratio(x, dx), ratio(s, ds)
    sigma = 0.0
    if ap < 1.0 or ad < 1.0:
        mu_af = (x + ap * dx) @ (s + ad * ds) / n
        sigma = min(sigma_max, (mu_af / mu) ** 2 if gam > 1e-3 else 10.0 * gam)
        cx, cy, cs = newton(np.zeros(m), np.zeros(n), sigma * mu - dx * ds)
        dx, dy, ds = dx + cx, dy + cy, ds + cs
    ap, ad = ratio(x, dx), ratio(s, ds)
    for _ in range(max_bt):
        pr = (x + ap * dx) * (s + ad * ds)
        if pr.min() >= phi * pr.sum() / n:
            break
        ap, ad = ap * bt, ad * bt
    return x + ap * dx, y + ad * dy, s + ad * ds, sigma


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("K", [None, 0])
def test_zero_correctors_is_mehrotras_method(seed, K):
    """With no centrality corrector (the default, and max_correctors = 0) an oracle step
    equals Mehrotra's step computed independently from dense Newton solves, from the
    starting point and from a later iterate."""
    lp = synth.sparse_lp(30, 80, 4, 0, seed=seed)
    A = lp.to_dense()
    opts = oracle.ipm_opts() if K is None else oracle.ipm_opts(max_correctors=K)
    x, y, s = oracle.init_point(lp, tol=1e-14)
    sigmas = []
    for step in range(3):
        xr, yr, sr, sig = _mehrotra_step_dense(A, lp.b, lp.c, x, y, s)
        st = oracle.new_state(eps_in0=1e-14)     # first-iteration state: no eps_in update
        rc, done, L = oracle.ipm_iterate(lp, x, y, s, st, opts)
        assert rc == oracle.OK and not done and L["correctors"] == 0
        assert L["sigma"] == pytest.approx(sig, rel=1e-8, abs=1e-14)
        for got, ref in ((x, xr), (y, yr), (s, sr)):
            np.testing.assert_allclose(got, ref, rtol=1e-8, atol=1e-9 * np.abs(ref).max())
        sigmas.append(sig)
        x, y, s = xr.copy(), yr.copy(), sr.copy()
    assert max(sigmas) > 0            # the corrector stage ran


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

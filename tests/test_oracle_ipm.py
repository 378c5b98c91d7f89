"""Pins of the oracle's interior-point recurrence and its end result (CPU only).

* the w-recurrence (eq. step_predictor / step_corrector) against a dense solve of the
  full Newton system (eq. SE1);
* LP optima against brute-force vertex enumeration (tiny LPs), HiGHS (scipy), an exact
  integer min-cost-flow solve (transportation), and the closed-form basis-pursuit
  optimum ||x_true||_1;
* invariances: row sign flip (bitwise), duplicated rows, column scaling;
* the failure paths of Sec. 4.2: eps_in x1.5 after a failed solve, the iteration cap.
"""
import itertools

import numpy as np
import pytest
from scipy.optimize import linprog

import oracle
from paper_1604_07491_amd import synth


# ---------------------------------------------------------------- Newton system (SE1)
def _newton(A, x, s, rd, rp, rc):
    m, n = A.shape
    K = np.zeros((m + 2 * n, m + 2 * n))
    K[:n, n:n + m] = A.T
    K[:n, n + m:] = np.eye(n)
    K[n:n + m, :n] = A
    K[n + m:, :n] = np.diag(s)
    K[n + m:, n + m:] = np.diag(x)
    rhs = np.concatenate([rd, rp, rc])
    sol = np.linalg.lstsq(K, rhs, rcond=None)[0]
    return sol[:n], sol[n:n + m], sol[n + m:]


@pytest.mark.parametrize("seed,dup", [(0, 0), (1, 2), (2, 1)])
def test_w_recurrence_solves_newton_system(seed, dup):
    lp = synth.tiny_lp(5, 11, seed, density=0.7, n_dup=dup)
    A = lp.to_dense()
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.1, 3.0, lp.n)
    s = rng.uniform(0.1, 3.0, lp.n)
    y = rng.standard_normal(lp.m)
    rd = lp.c - A.T @ y - s
    rp = lp.b - A @ x
    dx, dy, ds, _ = oracle.affine_direction(lp, x, y, s, 1e-14)
    rdx, rdy, rds = _newton(A, x, s, rd, rp, -x * s)
    np.testing.assert_allclose(dx, rdx, rtol=1e-9, atol=1e-10 * np.abs(rdx).max())
    np.testing.assert_allclose(ds, rds, rtol=1e-9, atol=1e-10 * np.abs(rds).max())
    np.testing.assert_allclose(A.T @ dy, A.T @ rdy, rtol=1e-9, atol=1e-10 * np.abs(A.T @ rdy).max())
    sigma_mu = 0.3 * (x @ s) / lp.n
    cx, cy, cs, _ = oracle.corrector_direction(lp, x, s, dx, ds, sigma_mu, 1e-14)
    rcx, rcy, rcs = _newton(A, x, s, np.zeros(lp.n), np.zeros(lp.m), -dx * ds + sigma_mu)
    np.testing.assert_allclose(cx, rcx, rtol=1e-9, atol=1e-10 * np.abs(rcx).max())
    np.testing.assert_allclose(cs, rcs, rtol=1e-9, atol=1e-10 * np.abs(rcs).max())
    np.testing.assert_allclose(A.T @ cy, A.T @ rcy, rtol=1e-9, atol=1e-10 * np.abs(A.T @ rcy).max())


# ---------------------------------------------------------------- brute force
def brute_force_lp(A, b, c):
    """min c^T x over the basic feasible solutions of A x = b, x >= 0."""
    m, n = A.shape
    r = np.linalg.matrix_rank(A)
    best = np.inf
    for cols in itertools.combinations(range(n), r):
        B = A[:, cols]
        if np.linalg.matrix_rank(B) < r:
            continue
        xb = np.linalg.lstsq(B, b, rcond=None)[0]
        if np.linalg.norm(B @ xb - b) > 1e-9 * max(1, np.linalg.norm(b)) or xb.min() < -1e-10:
            continue
        best = min(best, float(c[list(cols)] @ xb))
    return best


@pytest.mark.parametrize("m,n,seed,dup", [(3, 7, 0, 0), (4, 9, 1, 0), (5, 12, 2, 1), (4, 10, 3, 2), (6, 12, 4, 0)])
def test_ipm_matches_vertex_enumeration(m, n, seed, dup):
    lp = synth.tiny_lp(m, n, seed, density=0.7, n_dup=dup)
    A = lp.to_dense()
    ref = brute_force_lp(A, lp.b, lp.c)
    r = oracle.ipm(lp)
    assert r["status"] == oracle.OK, r["status"]
    assert abs(r["pobj"] - ref) <= 1e-8 * max(1.0, abs(ref))
    assert np.all(r["x"] > 0) and np.all(r["s"] > 0)
    assert np.linalg.norm(A @ r["x"] - lp.b) <= 1e-8 * max(1, np.linalg.norm(lp.b))


# ---------------------------------------------------------------- HiGHS
def test_ipm_config0_matches_highs():
    lp = synth.config(0)
    r = oracle.ipm(lp)
    assert r["status"] == oracle.OK and r["gamma_rel"] <= 1e-8
    h = linprog(lp.c, A_eq=lp.to_dense(), b_eq=lp.b, bounds=(0, None), method="highs")
    assert abs(r["pobj"] - h.fun) <= 1e-8 * abs(h.fun)
    assert abs(r["dobj"] - h.fun) <= 1e-8 * abs(h.fun)


def transport_min_cost(supply, demand, cost):
    """Exact integer optimum of the transportation problem by successive shortest paths
    (Dijkstra with node potentials on the residual bipartite network)."""
    S, T = cost.shape
    x = np.zeros((S, T), np.int64)
    sup = supply.astype(np.int64).copy()
    dem = demand.astype(np.int64).copy()
    pot_s = np.zeros(S)
    pot_t = np.zeros(T)
    while sup.sum() > 0:
        ds = np.where(sup > 0, 0.0, np.inf)
        dt = np.full(T, np.inf)
        done_s = np.zeros(S, bool)
        done_t = np.zeros(T, bool)
        pred_t = np.full(T, -1)
        pred_s = np.full(S, -1)
        target = -1
        while True:
            cs = np.where(done_s, np.inf, ds)
            ct = np.where(done_t, np.inf, dt)
            i, j = int(np.argmin(cs)), int(np.argmin(ct))
            if cs[i] <= ct[j]:
                if not np.isfinite(cs[i]):
                    raise RuntimeError("infeasible")
                done_s[i] = True
                nd = ds[i] + cost[i] + pot_s[i] - pot_t
                upd = (~done_t) & (nd < dt)
                dt[upd] = nd[upd]
                pred_t[upd] = i
            else:
                done_t[j] = True
                if dem[j] > 0:
                    target = j
                    break
                back = x[:, j] > 0
                nd = dt[j] - cost[:, j] + pot_t[j] - pot_s
                upd = back & (~done_s) & (nd < ds)
                ds[upd] = nd[upd]
                pred_s[upd] = j
        dmax = dt[target]
        pot_s += np.minimum(ds, dmax)
        pot_t += np.minimum(dt, dmax)
        # walk back, find the bottleneck
        path = []
        j = target
        while True:
            i = pred_t[j]
            path.append((i, j))
            if pred_s[i] < 0:
                break
            j = pred_s[i]
        start = path[-1][0]
        amt = min(sup[start], dem[target])
        # reverse arcs on the path (source i back to sink pred_s[i]) carry flow to undo
        rev = []
        j = target
        while True:
            i = pred_t[j]
            if pred_s[i] < 0:
                break
            rev.append((i, pred_s[i]))
            j = pred_s[i]
        for (i, jj) in rev:
            amt = min(amt, x[i, jj])
        j = target
        while True:
            i = pred_t[j]
            x[i, j] += amt
            if pred_s[i] < 0:
                break
            x[i, pred_s[i]] -= amt
            j = pred_s[i]
        sup[start] -= amt
        dem[target] -= amt
    assert np.all(x >= 0)
    assert np.array_equal(x.sum(1), supply.astype(np.int64))
    assert np.array_equal(x.sum(0), demand.astype(np.int64))
    return int((x * cost.astype(np.int64)).sum())


def test_min_cost_flow_checker_on_small_instance():
    t = synth.transport_lp(6, 5, seed=11)
    A = t.to_dense()
    h = linprog(t.c, A_eq=A, b_eq=t.b, bounds=(0, None), method="highs")
    exact = transport_min_cost(t.b[:6], t.b[6:], t.c.reshape(6, 5))
    assert abs(h.fun - exact) < 1e-6
    assert abs(brute_force_lp(synth.transport_lp(2, 3, seed=5).to_dense(), synth.transport_lp(2, 3, seed=5).b,
                              synth.transport_lp(2, 3, seed=5).c)
               - transport_min_cost(synth.transport_lp(2, 3, seed=5).b[:2], synth.transport_lp(2, 3, seed=5).b[2:],
                                    synth.transport_lp(2, 3, seed=5).c.reshape(2, 3))) < 1e-9


def test_ipm_config1_transport_exact_integer_optimum():
    lp = synth.config(1)
    r = oracle.ipm(lp)
    assert r["status"] == oracle.OK and r["gamma_rel"] <= 1e-8
    ns, nt = lp.meta["n_src"], lp.meta["n_snk"]
    exact = transport_min_cost(lp.b[:ns], lp.b[ns:], lp.c.reshape(ns, nt))
    assert abs(r["pobj"] - exact) <= 1e-8 * exact
    assert abs(r["dobj"] - exact) <= 1e-8 * exact


def test_ipm_basis_pursuit_closed_form():
    """Basis pursuit with a sparse +-1 signal well inside the recovery region: the LP
    optimum is ||x_true||_1 = k, attained at u = max(x_true, 0), v = max(-x_true, 0)."""
    lp = synth.basis_pursuit_lp(64, 256, 4, seed=7)
    o = oracle.ipm_opts(solver=oracle.solver_opts(order=oracle.ORDER_NATURAL))
    r = oracle.ipm(lp, o)
    assert r["status"] == oracle.OK
    k = lp.meta["k"]
    assert abs(r["pobj"] - k) <= 1e-7 * k
    xt = lp.meta["x_true"]
    N = lp.meta["N"]
    x = r["x"][:N] - r["x"][N:]
    assert np.abs(x - xt).max() < 1e-6


# ---------------------------------------------------------------- invariances
def test_row_sign_flip_is_bitwise_invariant():
    lp = synth.config(0)
    r1 = oracle.ipm(lp)
    A = lp.to_dense().copy()
    flip = [3, 77, 150]
    A[flip] *= -1
    b = lp.b.copy()
    b[flip] *= -1
    lp2 = synth.from_dense(A, b, lp.c)
    r2 = oracle.ipm(lp2)
    assert r1["iters"] == r2["iters"]
    assert np.array_equal(r1["x"], r2["x"]) and np.array_equal(r1["s"], r2["s"])
    y2 = r2["y"].copy()
    y2[flip] *= -1
    assert np.array_equal(r1["y"], y2)


def test_duplicate_rows_do_not_change_the_solution():
    """Config-0 LP with its duplicated rows vs the same LP without them."""
    lp = synth.config(0)
    A = lp.to_dense()
    mb = lp.meta["m_base"]
    red = synth.from_dense(A[:mb], lp.b[:mb], lp.c)
    r_full = oracle.ipm(lp)
    r_red = oracle.ipm(red)
    assert r_full["status"] == oracle.OK and r_red["status"] == oracle.OK
    assert abs(r_full["pobj"] - r_red["pobj"]) <= 1e-8 * abs(r_red["pobj"])
    np.testing.assert_allclose(r_full["x"], r_red["x"], atol=1e-6)
    # duals: y_i + y_i' of the duplicated pair equals y_i of the reduced LP
    y = r_full["y"][:mb].copy()
    for t, r in enumerate(lp.meta["dup_rows"]):
        y[r] += r_full["y"][mb + t]
    np.testing.assert_allclose(y, r_red["y"], atol=1e-5 * np.abs(r_red["y"]).max())


def test_column_scaling_keeps_the_objective():
    lp = synth.config(0)
    A = lp.to_dense()
    k = 10.0 ** np.random.default_rng(3).uniform(-1, 1, lp.n)
    lp2 = synth.from_dense(A * k, lp.b, lp.c * k)
    r1, r2 = oracle.ipm(lp), oracle.ipm(lp2)
    assert r1["status"] == oracle.OK and r2["status"] == oracle.OK
    assert abs(r1["pobj"] - r2["pobj"]) <= 1e-8 * abs(r1["pobj"])
    np.testing.assert_allclose(r1["x"], r2["x"] * k, atol=1e-6)


# ---------------------------------------------------------------- failure paths
def test_failed_krylov_solve_relaxes_eps_in():
    """Sec. 4.2: a solve that misses the tolerance within kmax multiplies the next step's
    eps_in by 1.5 on top of the schedule; eps_in stays in [1e-14, 1e-4]."""
    lp = synth.config(0)
    o = oracle.ipm_opts(solver=oracle.solver_opts(kmax=2), max_iter=6)
    r = oracle.ipm(lp, o)
    log = r["log"]
    assert all(L["fail_af"] or L["fail_cc"] for L in log[:r["iters"]])
    for k in range(1, r["iters"]):
        lg = np.log10(log[k]["gamma"])
        fac = 0.375 if lg <= -3 else (0.75 if lg <= 1 else 1.0)
        expect = min(max(log[k - 1]["eps_in"] * fac * 1.5, 1e-14), 1e-4)
        assert log[k]["eps_in"] == pytest.approx(expect, rel=1e-15)
    assert r["status"] == oracle.NOT_CONVERGED


def test_iteration_cap_and_infeasible_lp():
    lp = synth.config(0)
    r = oracle.ipm(lp, oracle.ipm_opts(max_iter=3))
    assert r["status"] == oracle.NOT_CONVERGED and r["iters"] == 3 and r["gamma_rel"] > 1e-8
    # x1 + x2 = 1 and x1 + x2 = 2: infeasible, so no optimum exists
    bad = synth.from_dense(np.array([[1.0, 1.0, 0.0], [1.0, 1.0, 0.0], [0.0, 1.0, 1.0]]),
                           np.array([1.0, 2.0, 1.0]), np.array([1.0, 1.0, 1.0]))
    r = oracle.ipm(bad, oracle.ipm_opts(max_iter=30))
    assert r["status"] in (oracle.NOT_CONVERGED, oracle.DIVERGED)


def test_eps_in_schedule_without_failures():
    lp = synth.config(0)
    r = oracle.ipm(lp)
    log = r["log"]
    assert log[0]["eps_in"] == 1e-6
    for k in range(1, r["iters"]):
        lg = np.log10(log[k]["gamma"])
        fac = 0.375 if lg <= -3 else (0.75 if lg <= 1 else 1.0)
        if log[k - 1]["fail_af"] or log[k - 1]["fail_cc"]:
            fac *= 1.5
        expect = min(max(log[k - 1]["eps_in"] * fac, 1e-14), 1e-4)
        assert log[k]["eps_in"] == pytest.approx(expect, rel=1e-15)
        # sigma rule of Sec. 2.1
        if log[k]["sigma"] > 0 and log[k]["gamma"] <= 1e-3:
            assert log[k]["sigma"] == pytest.approx(min(0.208, 10 * log[k]["gamma"]), rel=1e-14)

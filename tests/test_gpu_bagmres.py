"""BA-GMRES (GMRES on C A_hat A_hat^T dyh = C f_hat in m-space, eq. ba_ne, C the NE-SOR or
NE-SSOR operator) on the GPU through the C ABI, against the CPU FP64 oracle.  GPU only.

Tolerances.  At a fixed number of iterations both sides compute the same GMRES iterate in
exact arithmetic and differ by rounding (summation order, fused multiply-add, CGS2 on the
GPU against MGS in the oracle): 1e-9 relative, as for AB-GMRES.  The residual estimate
|gamma_k| is compared to 1e-8 relative.  Converged solves are compared with the min-norm
solution pinv(A D) f (dw = A_hat^T dyh lies in the range of A_hat^T, so a solution of
A_hat dw = f_hat of that form is the min-norm one): 1e-8 relative at solve tolerance
1e-12; the oracle reaches 1e-12 relative or better on these cases.  The method stops on
its own (preconditioned) residual, so the true residual is bounded more loosely: 1e-10
relative to ||f_hat||.
"""
import numpy as np
import pytest

import oracle
from _parity import assert_close, rel
import paper_1604_07491_amd as lpk
from paper_1604_07491_amd import synth

pytestmark = pytest.mark.gpu




def _case(name):
    if name == "config0":   # 200 x 500: z and rows staged in LDS (one-block sweep)
        return synth.config(0)
    if name == "ragged":
        return synth.sparse_lp(331, 777, 5, 4, seed=21)
    if name == "ldsz":      # z in LDS, rows streamed from HBM
        return synth.sparse_lp(300, 2000, 6, 2, seed=61)
    if name == "transport":
        return synth.transport_lp(31, 29, seed=8)
    if name == "transport_wide":   # z over the LDS limit: colour-by-colour sweeps
        return synth.transport_lp(130, 100, seed=8)
    raise ValueError(name)


def _dir_problem(lp, seed=0):
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.2, 2.0, lp.n)
    w = rng.standard_normal(lp.n)
    return d, oracle.csr_mv(lp, d * w)


INNER = {"nesor": oracle.NESOR, "nessor": oracle.NESSOR}
FIXED = [("config0", 1), ("config0", 4), ("config0", 13), ("ragged", 1), ("ragged", 4), ("ragged", 13),
         ("ldsz", 1), ("ldsz", 6), ("transport", 1), ("transport", 3), ("transport_wide", 1),
         ("transport_wide", 2)]


@pytest.mark.parametrize("inner", ["nesor", "nessor"])
@pytest.mark.parametrize("name,k", FIXED)
def test_bagmres_fixed_iterations(name, k, inner):
    lp = _case(name)
    d, f = _dir_problem(lp, k)
    print(f"case {name} k={k} bagmres {inner} m={lp.m} n={lp.n}", flush=True)
    with lpk.from_lp(lp, lpk.options(krylov="bagmres", inner=inner, krylov_max_iter=k)) as p:
        dw, dy, info = lpk.direction_solve(p, d, f, 0.0)
    odw, ody, oinfo = oracle.dirsolve(lp, d, f, 0.0,
                                      oracle.solver_opts(krylov=oracle.BAGMRES, inner=INNER[inner], kmax=k))
    assert info["iters"] == oinfo["iters"] == k
    assert_close(dw, odw, 1e-9)
    # dy is unique up to the null space of (A D)^T: compare (A D)^T dy
    AD = lp.to_dense() * d
    assert_close(AD.T @ np.asarray(dy), AD.T @ ody, 1e-9)
    assert abs(info["beta"] - oinfo["beta"]) <= 1e-12 * oinfo["beta"]
    assert abs(info["res_est"] - oinfo["res_est"]) <= 1e-8 * oinfo["res_est"]
    assert abs(info["res_true"] - oinfo["res_true"]) <= 1e-9 * oinfo["beta"]


@pytest.mark.parametrize("inner", ["nesor", "nessor"])
@pytest.mark.parametrize("name", ["config0", "ragged", "ldsz", "transport", "transport_wide"])
def test_bagmres_converged_is_min_norm(name, inner):
    lp = _case(name)
    d, f = _dir_problem(lp, 3)
    print(f"case {name} bagmres {inner}", flush=True)
    with lpk.from_lp(lp, lpk.options(krylov="bagmres", inner=inner)) as p:
        dw, dy, info = lpk.direction_solve(p, d, f, 1e-12)
    _, _, oinfo = oracle.dirsolve(lp, d, f, 1e-12, oracle.solver_opts(krylov=oracle.BAGMRES, inner=INNER[inner]))
    AD = lp.to_dense() * d
    ref = np.linalg.pinv(AD) @ f
    print(f"iters {info['iters']} (oracle {oinfo['iters']}) res_true/beta {info['res_true'] / info['beta']:.2e} "
          f"err {rel(dw, ref):.2e}", flush=True)
    assert not info["failed"]
    assert abs(info["iters"] - oinfo["iters"]) <= 1
    assert_close(dw, ref, 1e-8)
    assert_close(AD.T @ np.asarray(dy), ref, 1e-8)
    assert info["res_true"] <= 1e-10 * info["beta"]


def test_bagmres_zero_right_hand_side():
    lp = _case("ragged")
    d = np.ones(lp.n)
    with lpk.from_lp(lp, lpk.options(krylov="bagmres", inner="nessor")) as p:
        dw, dy, info = lpk.direction_solve(p, d, np.zeros(lp.m), 1e-10)
    assert info["iters"] == 0 and info["beta"] == 0.0 and not info["failed"]
    assert not np.any(np.asarray(dw)) and not np.any(np.asarray(dy))


def test_bagmres_solves_the_corrector_least_squares_form():
    """f = (A D) h: the solve gives dw = (A D)^T dy with dy a least-squares solution of
    min ||(A D)^T dy - h|| (eq. ba_ne), on a problem with duplicated rows."""
    lp = synth.sparse_lp(240, 900, 5, 3, seed=77)
    rng = np.random.default_rng(5)
    d = rng.uniform(0.2, 2.0, lp.n)
    h = rng.standard_normal(lp.n)
    AD = lp.to_dense() * d
    f = AD @ h
    with lpk.from_lp(lp, lpk.options(krylov="bagmres", inner="nessor")) as p:
        dw, dy, info = lpk.direction_solve(p, d, f, 1e-12)
    dy_ls = np.linalg.lstsq(AD.T, h, rcond=None)[0]
    assert not info["failed"]
    assert_close(dw, AD.T @ dy_ls, 1e-8)


def test_bagmres_batch_matches_alone():
    """A problem's interior-point iterates are bitwise the same alone and in a batch of
    problems of different shapes (LDS and streamed sweeps mixed)."""
    lps = [synth.transport_lp(20 + 3 * i, 18 + 2 * i, seed=40 + i) for i in range(4)]
    lps.append(synth.sparse_lp(300, 2000, 6, 2, seed=61))
    opt = dict(krylov="bagmres", inner="nesor")
    alone = []
    for lp in lps:
        with lpk.from_lp(lp, lpk.options(**opt)) as p:
            r = lpk.lp_solve(p)
            x, y, s, _ = lpk.lp_get_state(p)
            alone.append((r, np.asarray(x).copy()))
    probs = [lpk.from_lp(lp, lpk.options(**opt)) for lp in lps]
    try:
        res = lpk.lp_solve_batch(probs, width=8)
        for (ra, xa), rb, p in zip(alone, res, probs):
            xb, _, _, _ = lpk.lp_get_state(p)
            assert rb["status"] == ra["status"]
            assert rb["iters"] == ra["iters"] and rb["krylov_iters"] == ra["krylov_iters"]
            assert np.array_equal(np.asarray(xb), xa)
    finally:
        for p in probs:
            p.close()


@pytest.mark.parametrize("inner", ["nesor", "nessor"])
def test_bagmres_lp_solve_end_to_end(inner):
    lp = synth.transport_lp(31, 29, seed=8)
    sopts = oracle.solver_opts(krylov=oracle.BAGMRES, inner=INNER[inner])
    o = oracle.ipm(lp, oracle.ipm_opts(solver=sopts))
    print(f"oracle bagmres {inner}: status {o['status']} iters {o['iters']} pobj {o['pobj']!r}", flush=True)
    assert o["status"] == oracle.OK
    with lpk.from_lp(lp, lpk.options(krylov="bagmres", inner=inner)) as p:
        r = lpk.lp_solve(p)
    print(f"gpu iters {r['iters']} krylov {r['krylov_iters']} gamma_rel {r['gamma_rel']:.2e} pobj {r['pobj']!r}",
          flush=True)
    assert r["status"] == lpk.LP_OK
    assert r["gamma_rel"] <= 1e-8
    assert abs(r["pobj"] - o["pobj"]) <= 1e-7 * abs(o["pobj"])
    assert abs(r["dobj"] - o["pobj"]) <= 1e-7 * abs(o["pobj"])

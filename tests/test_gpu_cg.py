"""CGNE and MRNE preconditioned by inner iterations (Sec. 3.3), and NE-SSOR sweeps, on the
GPU through the C ABI, against the CPU FP64 oracle.  GPU only.

Tolerances.  At a fixed number of iterations both sides compute the same CG iterate in
exact arithmetic and differ by rounding (summation order, fused multiply-add).  CG
recurrences amplify rounding once the residual nears the rounding level, so the fixed-k
cases stop while the relative residual is still far above it (the oracle's iterate moves
by about 1e-15 relative under a 1e-15 perturbation of f at these k): 1e-9 relative.
Converged solves are compared with the min-norm solution pinv(A D) f: CG started from
zero keeps dw in the range of (A D)^T, so it converges to that solution; 1e-8 relative at
solve tolerance 1e-12 (the oracle reaches 1e-11 or better on these cases).  Mixed
precision (FP32 sweeps) perturbs the preconditioner, which CG does not absorb as the
flexible AB-GMRES does, so CGNE's mixed cases use solve tolerance 1e-10 and 1e-6; MRNE is
FP64 only (the library rejects mixed MRNE: its recurrence for q = A^T C g drifts and
diverges under a perturbed C, as an FP32 emulation of the sweeps on the CPU shows).
"""
import numpy as np
import pytest

import oracle
import paper_1604_07491_amd as lpk
from paper_1604_07491_amd import synth

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a = np.asarray(a.cpu() if hasattr(a, "cpu") else a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _case(name):
    if name == "config0":
        return synth.config(0)
    if name == "ragged":
        return synth.sparse_lp(331, 777, 5, 4, seed=21)
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


KRY = {"cgne": oracle.CGNE, "mrne": oracle.MRNE}
INNER = {"nessor": oracle.NESSOR, "nesor": oracle.NESOR, "cimmino": oracle.CIMMINO}
FIXED = [("config0", 1), ("config0", 4), ("config0", 13), ("ragged", 1), ("ragged", 4), ("ragged", 13),
         ("transport", 1), ("transport", 3), ("transport_wide", 1), ("transport_wide", 3)]


@pytest.mark.parametrize("inner", ["nessor", "nesor", "cimmino"])
@pytest.mark.parametrize("krylov", ["cgne", "mrne"])
@pytest.mark.parametrize("name,k", FIXED)
def test_cg_fixed_iterations(name, k, krylov, inner):
    lp = _case(name)
    d, f = _dir_problem(lp, 3)
    print(f"case {name} k={k} {krylov} {inner} m={lp.m} n={lp.n}", flush=True)
    with lpk.from_lp(lp, lpk.options(krylov=krylov, inner=inner, krylov_max_iter=k)) as p:
        dw, dy, info = lpk.direction_solve(p, d, f, 0.0)
    odw, ody, oinfo = oracle.dirsolve(lp, d, f, 0.0, oracle.solver_opts(krylov=KRY[krylov], inner=INNER[inner], kmax=k))
    assert info["iters"] == oinfo["iters"] == k
    assert _rel(dw, odw) <= 1e-9
    # dy is unique up to the null space of (A D)^T: compare (A D)^T dy
    AD = lp.to_dense() * d
    assert _rel(AD.T @ np.asarray(dy), AD.T @ ody) <= 1e-9
    assert abs(info["res_est"] - oinfo["res_est"]) <= 1e-9 * oinfo["beta"]
    assert abs(info["res_true"] - oinfo["res_true"]) <= 1e-9 * oinfo["beta"]


@pytest.mark.parametrize("name,k", [("config0", 1), ("config0", 4), ("config0", 13), ("ragged", 4),
                                    ("transport", 4), ("transport_wide", 3)])
def test_nessor_abgmres_fixed_iterations(name, k):
    lp = _case(name)
    d, f = _dir_problem(lp, k)
    print(f"case {name} k={k} abgmres nessor", flush=True)
    with lpk.from_lp(lp, lpk.options(inner="nessor", krylov_max_iter=k)) as p:
        dw, dy, info = lpk.direction_solve(p, d, f, 0.0)
    odw, ody, oinfo = oracle.dirsolve(lp, d, f, 0.0, oracle.solver_opts(inner=oracle.NESSOR, kmax=k, flexible=1))
    assert info["iters"] == oinfo["iters"] == k
    assert _rel(dw, odw) <= 1e-9
    AD = lp.to_dense() * d
    assert _rel(AD.T @ np.asarray(dy), AD.T @ ody) <= 1e-9


# MRNE runs in FP64 only (its q recurrence needs one fixed linear preconditioner)
CONVERGED = [(kr, pr) for kr in ("cgne", "mrne") for pr in ("fp64", "mixed") if (kr, pr) != ("mrne", "mixed")]


@pytest.mark.parametrize("inner", ["nessor", "cimmino"])
@pytest.mark.parametrize("krylov,precision", CONVERGED)
@pytest.mark.parametrize("name", ["config0", "ragged", "transport", "transport_wide"])
def test_cg_converged_is_min_norm(name, krylov, precision, inner):
    lp = _case(name)
    d, f = _dir_problem(lp, 3)
    tol, bound = (1e-12, 1e-8) if precision == "fp64" else (1e-10, 1e-6)
    print(f"case {name} {krylov} {inner} {precision}", flush=True)
    with lpk.from_lp(lp, lpk.options(krylov=krylov, inner=inner, precision=precision)) as p:
        dw, dy, info = lpk.direction_solve(p, d, f, tol)
    AD = lp.to_dense() * d
    ref = np.linalg.pinv(AD) @ f
    print(f"iters {info['iters']} res_true/beta {info['res_true'] / info['beta']:.2e} err {_rel(dw, ref):.2e}", flush=True)
    assert not info["failed"]
    assert _rel(dw, ref) <= bound
    assert _rel(AD.T @ np.asarray(dy), ref) <= bound
    assert info["res_true"] <= 10 * tol * info["beta"]


def test_cg_zero_right_hand_side():
    lp = _case("ragged")
    d = np.ones(lp.n)
    for krylov in ("cgne", "mrne"):
        with lpk.from_lp(lp, lpk.options(krylov=krylov, inner="nessor")) as p:
            dw, dy, info = lpk.direction_solve(p, d, np.zeros(lp.m), 1e-10)
        assert info["iters"] == 0 and info["beta"] == 0.0 and not info["failed"]
        assert not np.any(np.asarray(dw)) and not np.any(np.asarray(dy))


@pytest.mark.parametrize("krylov", ["cgne", "mrne"])
def test_cg_batch_matches_alone(krylov):
    """A problem's interior-point iterates are bitwise the same alone and in a batch of
    problems of different shapes."""
    lps = [synth.transport_lp(20 + 3 * i, 18 + 2 * i, seed=40 + i) for i in range(5)]
    opt = dict(krylov=krylov, inner="nessor")
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


@pytest.mark.parametrize("krylov", ["cgne", "mrne"])
def test_cg_lp_solve_end_to_end(krylov):
    lp = synth.transport_lp(31, 29, seed=8)
    sopts = oracle.solver_opts(krylov=KRY[krylov], inner=oracle.NESSOR)
    o = oracle.ipm(lp, oracle.ipm_opts(solver=sopts))
    print(f"oracle {krylov}: status {o['status']} iters {o['iters']} pobj {o['pobj']!r}", flush=True)
    assert o["status"] == oracle.OK
    with lpk.from_lp(lp, lpk.options(krylov=krylov, inner="nessor")) as p:
        r = lpk.lp_solve(p)
    print(f"gpu iters {r['iters']} krylov {r['krylov_iters']} gamma_rel {r['gamma_rel']:.2e} pobj {r['pobj']!r}",
          flush=True)
    assert r["status"] == lpk.LP_OK
    assert r["gamma_rel"] <= 1e-8
    assert abs(r["pobj"] - o["pobj"]) <= 1e-7 * abs(o["pobj"])
    assert abs(r["dobj"] - o["pobj"]) <= 1e-7 * abs(o["pobj"])

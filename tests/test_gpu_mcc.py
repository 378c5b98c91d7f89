"""Multiple centrality correctors (lp_options.max_correctors) on the GPU against the
oracle with the same number of correctors.  GPU only.

Both sides take the same steps in exact arithmetic.  A corrector is kept or dropped by a
comparison of step lengths, which rounding (fused multiply-add on the GPU, summation
order) can flip when the two sides are within rounding of the threshold, so the number of
interior-point iterations may differ by one; the optimum may not: objectives within 1e-7
relative, as in the other end-to-end tests.
"""
import numpy as np
import pytest

import oracle
import paper_1604_07491_amd as lpk
from paper_1604_07491_amd import synth

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "sparse":
        return synth.config(0)
    if name == "transport":
        return synth.transport_lp(31, 29, seed=8)
    if name == "wide":
        return synth.transport_lp(130, 100, seed=8)
    raise ValueError(name)


@pytest.mark.parametrize("K", [1, 2])
@pytest.mark.parametrize("name", ["sparse", "transport", "wide"])
def test_correctors_match_the_oracle(name, K):
    lp = _case(name)
    o = oracle.ipm(lp, oracle.ipm_opts(max_correctors=K))
    assert o["status"] == oracle.OK
    with lpk.from_lp(lp, lpk.options(max_correctors=K)) as p:
        r = lpk.lp_solve(p)
        log = lpk.lp_get_log(p)
    nc = sum(L["correctors"] for L in log)
    print(f"{name} K={K}: gpu iters {r['iters']} correctors {nc}; oracle iters {o['iters']} "
          f"correctors {sum(L['correctors'] for L in o['log'])}", flush=True)
    assert r["status"] == lpk.LP_OK and r["gamma_rel"] <= 1e-8
    assert abs(r["pobj"] - o["pobj"]) <= 1e-7 * abs(o["pobj"])
    assert abs(r["iters"] - o["iters"]) <= 1
    assert nc > 0 and all(0 <= L["correctors"] <= K for L in log)
    assert all(L["k_mcc"] > 0 for L in log if L["correctors"] > 0)


def test_zero_correctors_take_no_corrector_solve():
    lp = _case("transport")
    with lpk.from_lp(lp, lpk.options(max_correctors=0)) as p:
        r = lpk.lp_solve(p)
        log = lpk.lp_get_log(p)
    assert r["status"] == lpk.LP_OK
    assert all(L["correctors"] == 0 and L["k_mcc"] == 0 for L in log)


def test_correctors_batch_matches_alone():
    lps = [synth.transport_lp(20 + 3 * i, 18 + 2 * i, seed=40 + i) for i in range(3)]
    lps += [synth.sparse_lp(100 + 20 * i, 260 + 40 * i, 5, 1, seed=50 + i) for i in range(2)]
    opt = dict(max_correctors=2)
    alone = []
    for lp in lps:
        with lpk.from_lp(lp, lpk.options(**opt)) as p:
            r = lpk.lp_solve(p)
            x, _, _, _ = lpk.lp_get_state(p)
            alone.append((r, np.asarray(x).copy()))
    probs = [lpk.from_lp(lp, lpk.options(**opt)) for lp in lps]
    try:
        res = lpk.lp_solve_batch(probs, width=8)
        for (ra, xa), rb, p in zip(alone, res, probs):
            xb, _, _, _ = lpk.lp_get_state(p)
            assert rb["status"] == ra["status"] and rb["iters"] == ra["iters"]
            assert np.array_equal(np.asarray(xb), xa)
    finally:
        for p in probs:
            p.close()


@pytest.mark.parametrize("krylov,inner", [("cgne", "nessor"), ("mrne", "nessor"), ("bagmres", "nesor")])
def test_correctors_with_other_krylov_methods(krylov, inner):
    """The corrector solves run through whichever Krylov method the LP uses.  CGNE and MRNE
    test the residual recomputed from their iterate on both sides (not a recurrence).  The
    step counts agree to the one step a corrector decision within rounding of its threshold
    may add, or else the side that stops first does so where the other side's gamma_rel is
    within a factor 2 of eps_out = 1e-8: late solves stop at eps_in of a few 1e-8, so the
    iterates, and gamma_rel with them, are determined only to about that level, and a side
    just above the threshold may need two more steps (measured on this LP with MRNE: the
    oracle's gamma_rel is 1.10e-8 after 10 steps and 2.38e-8 after 11)."""
    lp = _case("transport")
    kry = {"cgne": oracle.CGNE, "mrne": oracle.MRNE, "bagmres": oracle.BAGMRES}[krylov]
    inn = {"nessor": oracle.NESSOR, "nesor": oracle.NESOR}[inner]
    o = oracle.ipm(lp, oracle.ipm_opts(max_correctors=2, solver=oracle.solver_opts(krylov=kry, inner=inn)))
    assert o["status"] == oracle.OK
    with lpk.from_lp(lp, lpk.options(max_correctors=2, krylov=krylov, inner=inner)) as p:
        r = lpk.lp_solve(p)
        log = lpk.lp_get_log(p)
    nc = sum(L["correctors"] for L in log)
    print(f"{krylov}: gpu iters {r['iters']} correctors {nc}; oracle iters {o['iters']} "
          f"correctors {sum(L['correctors'] for L in o['log'])}", flush=True)
    assert r["status"] == lpk.LP_OK and r["gamma_rel"] <= 1e-8
    assert abs(r["pobj"] - o["pobj"]) <= 1e-7 * abs(o["pobj"])
    assert nc > 0
    gl = [L["gamma_rel"] for L in log]
    ol = [L["gamma_rel"] for L in o["log"]]
    first, other = (gl, ol) if r["iters"] < o["iters"] else (ol, gl)
    stop = min(r["iters"], o["iters"])
    print(f"gamma_rel at step {stop}: gpu {gl[stop]:.3e} oracle {ol[stop]:.3e}", flush=True)
    assert abs(r["iters"] - o["iters"]) <= 1 or other[stop] <= 2e-8

"""Presolve of dependent rows before a GPU solve: the LP with its duplicated rows removed
(lp_presolve_rows) reaches the optimum of the full LP (the oracle on the full LP).  GPU only."""
import numpy as np
import pytest

import oracle
import paper_1604_07491_amd as lpk
from paper_1604_07491_amd import synth

pytestmark = pytest.mark.gpu


def _reduced(lp, keep):
    A = lp.to_dense()[keep]
    return synth.from_dense(A, lp.b[keep], lp.c)


@pytest.mark.parametrize("shape", [(198, 500, 6, 2, 0), (120, 300, 5, 4, 1)])
def test_presolved_lp_reaches_the_full_optimum(shape):
    mb, n, k, dup, seed = shape
    lp = synth.sparse_lp(mb, n, k, dup, seed=seed)
    keep = lpk.lp_presolve_rows(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.val, lp.b)
    assert keep.sum() == mb
    red = _reduced(lp, keep)
    o = oracle.ipm(lp)
    assert o["status"] == oracle.OK
    with lpk.from_lp(red) as p:
        r = lpk.lp_solve(p)
    with lpk.from_lp(lp) as p:
        rf = lpk.lp_solve(p)
    print(f"{lp.m}x{lp.n}: reduced iters {r['iters']} krylov {r['krylov_iters']}; "
          f"full iters {rf['iters']} krylov {rf['krylov_iters']}", flush=True)
    assert r["status"] == lpk.LP_OK and r["gamma_rel"] <= 1e-8
    assert abs(r["pobj"] - o["pobj"]) <= 1e-7 * abs(o["pobj"])


@pytest.mark.parametrize("case", ["transport", "planted"])
def test_general_presolve_then_gpu_solve(case):
    """lp_presolve_dependent_rows before a GPU solve: the transportation LP (its one
    dependency, the last demand row, dropped) and a sparse LP with rows that are
    combinations of 2-4 earlier rows.  The reduced LP's GPU optimum equals the oracle's
    optimum of the full LP."""
    if case == "transport":
        lp = synth.transport_lp(20, 16, seed=4)
    else:
        base = synth.sparse_lp(60, 150, 4, 0, seed=9)
        A = base.to_dense()
        rng = np.random.default_rng(9)
        rows, rhs = [A[i] for i in range(base.m)], list(base.b)
        for _ in range(8):
            pos = int(rng.integers(4, len(rows) + 1))
            idx = rng.choice(pos, size=int(rng.integers(2, 5)), replace=False)
            w = rng.normal(size=len(idx))
            rows.insert(pos, sum(wi * rows[i] for wi, i in zip(w, idx)))
            rhs.insert(pos, sum(wi * rhs[i] for wi, i in zip(w, idx)))
        lp = synth.from_dense(np.array(rows), np.array(rhs), base.c)
    keep = lpk.lp_presolve_dependent_rows(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.val, lp.b)
    assert keep.sum() == np.linalg.matrix_rank(lp.to_dense())
    red = _reduced(lp, keep)
    o = oracle.ipm(lp)
    assert o["status"] == oracle.OK
    with lpk.from_lp(red) as p:
        r = lpk.lp_solve(p)
    print(f"{case}: {lp.m} -> {red.m} rows; gpu iters {r['iters']} pobj {r['pobj']:.10g}; "
          f"oracle (full) {o['pobj']:.10g}", flush=True)
    assert r["status"] == lpk.LP_OK and r["gamma_rel"] <= 1e-8
    assert abs(r["pobj"] - o["pobj"]) <= 1e-7 * max(1.0, abs(o["pobj"]))

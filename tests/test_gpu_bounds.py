"""Bounded variables lo <= x <= hi on the GPU (``lp_create_bounded``, ``lp_bounded_solution``)
against the oracle's bounded solve, which is pinned against HiGHS.  GPU only.

Both sides solve the same standard form (the reductions agree exactly, checked on the
host in test_bounds_host.py), so the objectives agree to the solve tolerance: 1e-7
relative, as in the other end-to-end tests.  The recovered x must lie within its bounds
and satisfy A x = b to the stopping tolerance.
"""
import numpy as np
import pytest

import oracle
import paper_1604_07491_amd as lpk
from oracle import bounds
from paper_1604_07491_amd import synth

pytestmark = pytest.mark.gpu

SHAPES = [(28, 80, 4, 2, 0), (60, 150, 5, 0, 1), (198, 500, 6, 2, 2)]


def _check_point(lp0, lo, hi, x, obj_ref):
    x = np.asarray(x.cpu() if hasattr(x, "cpu") else x)
    A = lp0.to_dense()
    scale = 1.0 + np.abs(x).max()
    assert np.all(x >= lo - 1e-7 * scale) and np.all(x <= hi + 1e-7 * scale)
    assert np.linalg.norm(A @ x - lp0.b) <= 1e-7 * (1 + np.linalg.norm(lp0.b))
    assert abs(lp0.c @ x - obj_ref) <= 1e-7 * max(1.0, abs(obj_ref))


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("krylov", ["abgmres", "bagmres"])
def test_bounded_lp_solve_matches_oracle(shape, krylov):
    mb, n, k, dup, seed = shape
    lp0, lo, hi = synth.bounded_lp(mb, n, k, dup, seed=seed)
    print(f"bounded {mb + dup}x{n} seed {seed} {krylov} kinds {lp0.meta['kinds']}", flush=True)
    o = bounds.ipm_bounded(lp0.to_dense(), lp0.b, lp0.c, lo, hi)
    assert o["status"] == oracle.OK
    with lpk.from_bounded_lp(lp0, lo, hi, lpk.options(krylov=krylov)) as p:
        assert (p.m, p.n) == (o["lp"].m, o["lp"].n)
        r = lpk.lp_solve(p)
        x, y, obj = lpk.lp_bounded_solution(p)
    print(f"gpu status {r['status']} iters {r['iters']} obj {obj!r} oracle {o['obj']!r}", flush=True)
    assert r["status"] == lpk.LP_OK and r["gamma_rel"] <= 1e-8
    assert abs(obj - o["obj"]) <= 1e-7 * max(1.0, abs(o["obj"]))
    # the standard form's objective plus the constant is the caller's objective
    assert abs(r["pobj"] + o["bmap"].offset - obj) <= 1e-8 * max(1.0, abs(obj))
    _check_point(lp0, lo, hi, x, o["obj"])
    assert y.shape == (lp0.m,)


@pytest.mark.parametrize("seed", [6, 8, 43, 56, 60])
def test_split_free_variables_are_recentred(seed):
    """LPs whose split free variables diverge without the pair recentring (both sides
    recentre after the starting point and after every step)."""
    lp0, lo, hi = synth.bounded_lp(198, 500, 6, 2, seed=seed)
    o = bounds.ipm_bounded(lp0.to_dense(), lp0.b, lp0.c, lo, hi)
    assert o["status"] == oracle.OK
    with lpk.from_bounded_lp(lp0, lo, hi) as p:
        r = lpk.lp_solve(p)
        x, y, obj = lpk.lp_bounded_solution(p)
        xs, _, _, _ = lpk.lp_get_state(p)
    print(f"seed {seed}: gpu iters {r['iters']} oracle {o['iters']} obj {obj!r} oracle {o['obj']!r}", flush=True)
    assert r["status"] == lpk.LP_OK and r["gamma_rel"] <= 1e-8
    assert abs(obj - o["obj"]) <= 1e-7 * max(1.0, abs(o["obj"]))
    _check_point(lp0, lo, hi, x, o["obj"])
    pr = bounds.free_pairs(o["bmap"])
    a, b = np.asarray(xs)[pr[:, 0]], np.asarray(xs)[pr[:, 1]]
    assert np.all(np.minimum(a, b) <= 0.5 * (1 + np.abs(a - b)) * (1 + 1e-12))


def test_bounded_device_arrays():
    lp0, lo, hi = synth.bounded_lp(60, 150, 5, 0, seed=1)
    o = bounds.ipm_bounded(lp0.to_dense(), lp0.b, lp0.c, lo, hi)
    with lpk.from_bounded_lp(lp0, lo, hi, device=True) as p:
        r = lpk.lp_solve(p)
        x, y, obj = lpk.lp_bounded_solution(p)
        assert x.is_cuda and y.is_cuda
    assert r["status"] == lpk.LP_OK
    assert abs(obj - o["obj"]) <= 1e-7 * max(1.0, abs(o["obj"]))
    _check_point(lp0, lo, hi, x, o["obj"])


def test_bounded_batch_matches_alone():
    cases = [synth.bounded_lp(40 + 10 * i, 120 + 20 * i, 4, 1, seed=30 + i) for i in range(4)]
    alone = []
    for lp0, lo, hi in cases:
        with lpk.from_bounded_lp(lp0, lo, hi) as p:
            r = lpk.lp_solve(p)
            alone.append((r, np.asarray(lpk.lp_bounded_solution(p)[0]).copy()))
    probs = [lpk.from_bounded_lp(lp0, lo, hi) for lp0, lo, hi in cases]
    try:
        res = lpk.lp_solve_batch(probs, width=4)
        for (ra, xa), rb, p in zip(alone, res, probs):
            assert rb["status"] == ra["status"] and rb["iters"] == ra["iters"]
            assert np.array_equal(np.asarray(lpk.lp_bounded_solution(p)[0]), xa)
    finally:
        for p in probs:
            p.close()


def test_solution_of_an_unbounded_problem_is_refused():
    lp = synth.config(0)
    with lpk.from_lp(lp) as p:
        with pytest.raises(lpk.LpError) as e:
            lpk.lp_bounded_solution(p)
    assert e.value.status == lpk.LP_EINVAL

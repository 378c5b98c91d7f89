"""Parity at the workloads' full sizes, on outputs the oracle computes quickly: direction
solves stopped after a fixed number of Krylov iterations (the oracle needs about a second
for one at 120,000 x 434,580).  GPU only.

Tolerances as in the smaller parity tests: FP64 paths 1e-9 relative (rounding order only);
FP32 sweeps (mixed precision) against the FP64 oracle 1e-4 relative, since the FP32
preconditioner perturbs every basis vector by about 1e-7 relative and the fixed-k iterate
amplifies that by the conditioning of the small Krylov problem.
"""
import functools

import numpy as np
import pytest

import oracle
from _parity import assert_close, rel, to_np
import paper_1604_07491_amd as lpk
from paper_1604_07491_amd import synth

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def _lp(name):
    if name == "config3":
        return synth.config(3)
    if name == "config1":
        return synth.config(1)
    if name == "serving_largest":
        # the largest member of the serving mix (m drawn first from each member's seed)
        ms = [int(np.random.default_rng(1000 + i).integers(200, 20_001)) for i in range(256)]
        i = int(np.argmax(ms))
        rng = np.random.default_rng(1000 + i)
        m = int(rng.integers(200, 20_001))
        n = int(round(m * rng.uniform(2.0, 4.0)))
        k = int(rng.integers(4, 11))
        return synth.sparse_lp(m - 2, n, k, 2, seed=1000 + i, name=f"serve_{i}_{m}x{n}")
    raise ValueError(name)


def _dir_problem(lp, seed):
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.2, 2.0, lp.n)
    w = rng.standard_normal(lp.n)
    return d, oracle.csr_mv(lp, d * w)


KRY = {"abgmres": oracle.ABGMRES, "cgne": oracle.CGNE, "mrne": oracle.MRNE, "bagmres": oracle.BAGMRES}
CASES = [("config3", "abgmres", "fp64", 1), ("config3", "abgmres", "fp64", 3), ("config3", "abgmres", "mixed", 3),
         ("config3", "cgne", "fp64", 2), ("config3", "bagmres", "fp64", 2),
         ("config1", "cgne", "fp64", 3), ("config1", "mrne", "fp64", 3), ("config1", "bagmres", "fp64", 3),
         ("serving_largest", "abgmres", "fp64", 3), ("serving_largest", "abgmres", "mixed", 3)]


@pytest.mark.parametrize("name,krylov,precision,k", CASES)
def test_fixed_iteration_direction_at_full_size(name, krylov, precision, k):
    lp = _lp(name)
    d, f = _dir_problem(lp, k)
    inner = "nessor" if krylov in ("cgne", "mrne") else "nesor"
    print(f"{name} {lp.m}x{lp.n} nnz {lp.nnz} {krylov} {inner} {precision} k={k}", flush=True)
    with lpk.from_lp(lp, lpk.options(krylov=krylov, inner=inner, precision=precision, krylov_max_iter=k)) as p:
        dw, dy, info = lpk.direction_solve(p, d, f, 0.0)
    so = oracle.solver_opts(krylov=KRY[krylov], inner=oracle.NESSOR if inner == "nessor" else oracle.NESOR,
                            kmax=k, flexible=1 if krylov == "abgmres" else 0)
    odw, ody, oinfo = oracle.dirsolve(lp, d, f, 0.0, so)
    tol = 1e-9 if precision == "fp64" else 1e-4
    # dy is unique up to the null space of (A D)^T: compare (A D)^T dy = d o (A^T dy)
    gdy = d * oracle.csr_tmv(lp, to_np(dy))
    ody_w = d * oracle.csr_tmv(lp, ody)
    print(f"iters {info['iters']} dw err {rel(dw, odw):.2e} (A D)^T dy err {rel(gdy, ody_w):.2e}", flush=True)
    assert info["iters"] == oinfo["iters"] == k
    assert_close(dw, odw, tol)
    assert_close(gdy, ody_w, tol)
    assert abs(info["res_true"] - oinfo["res_true"]) <= tol * oinfo["beta"]

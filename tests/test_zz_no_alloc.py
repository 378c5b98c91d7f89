"""direction_solve_noalloc (no device allocation in the call; per-call storage in the
library's fixed device array) against direction_solve on the same inputs.  GPU only.

Both launch the same kernels in the same order on the same data (direction_solve replays
them as a captured graph, the variant launches them one by one), so the results agree to
rounding, here checked at 1e-12 element by element.  Two calls in a row through the
variant, the second on a smaller LP, show that the array's leftover contents from the
first call do not leak into the second.
"""
import numpy as np
import pytest

import oracle
from _parity import assert_close, to_np
import paper_1604_07491_amd as lpk
from paper_1604_07491_amd import synth

pytestmark = pytest.mark.gpu


def _dir_problem(lp, seed):
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.2, 2.0, lp.n)
    return d, oracle.csr_mv(lp, d * rng.standard_normal(lp.n))


@pytest.mark.parametrize("krylov,inner", [("abgmres", "nesor"), ("cgne", "nessor")])
def test_noalloc_matches_direction_solve_on_two_calls(krylov, inner):
    import torch
    torch.cuda.set_device(0)
    big = synth.transport_lp(130, 100, seed=8)        # 230 x 13000: per-colour sweeps
    small = synth.config(0)                           # 200 x 500: one-block LDS sweeps
    for lp, tol in ((big, 1e-10), (small, 1e-10)):
        d, f = _dir_problem(lp, lp.m)
        print(f"{krylov} {lp.m}x{lp.n}", flush=True)
        with lpk.from_lp(lp, lpk.options(krylov=krylov, inner=inner)) as p:
            rdw, rdy, rinfo = lpk.direction_solve(p, d, f, tol)
        with lpk.from_lp(lp, lpk.options(krylov=krylov, inner=inner)) as p:
            dt = torch.tensor(d, dtype=torch.float64, device="cuda")
            ft = torch.tensor(f, dtype=torch.float64, device="cuda")
            dw = torch.full((lp.n,), float("nan"), dtype=torch.float64, device="cuda")
            dy = torch.full((lp.m,), float("nan"), dtype=torch.float64, device="cuda")
            info = lpk.direction_solve_noalloc(p, dt, ft, tol, dw, dy)
        print(f"iters {info['iters']} (direction_solve {rinfo['iters']}) res_true {info['res_true']:.3e}", flush=True)
        assert info["iters"] == rinfo["iters"] and info["failed"] == rinfo["failed"] == 0
        assert_close(to_np(dw), rdw, 1e-12)
        assert_close(to_np(dy), rdy, 1e-12)
        assert abs(info["res_true"] - rinfo["res_true"]) <= 1e-12 * rinfo["beta"]


def test_noalloc_rejects_a_workspace_beyond_its_array():
    import torch
    lp = synth.sparse_lp(2998, 7000, 5, 2, seed=3)     # AB-GMRES with kmax = m: about 144 MB
    d, f = _dir_problem(lp, 1)
    with lpk.from_lp(lp) as p:
        dt = torch.tensor(d, dtype=torch.float64, device="cuda")
        ft = torch.tensor(f, dtype=torch.float64, device="cuda")
        dw = torch.zeros(lp.n, dtype=torch.float64, device="cuda")
        with pytest.raises(lpk.LpError) as e:
            lpk.direction_solve_noalloc(p, dt, ft, 1e-8, dw)
        assert e.value.status == lpk.LP_ETOOBIG
        assert "scratch" in lpk.lib().lp_last_error().decode()
    # the same LP with a Krylov limit that fits solves
    with lpk.from_lp(lp, lpk.options(krylov_max_iter=200)) as p:
        info = lpk.direction_solve_noalloc(p, dt, ft, 1e-8, dw)
        assert info["iters"] >= 1 and np.isfinite(to_np(dw)).all()

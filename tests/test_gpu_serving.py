"""Lockstep batches and the request server (GPU).

Every reduction of an LP is partitioned by that LP's own sizes, so a result must be
bitwise identical alone (a batch of one) and inside any batch, including when LPs leave
and others join mid-way.  Admission must keep the summed
footprint of running requests within the budget, reject requests that can never fit, and
still complete every accepted request."""
import numpy as np
import pytest

import oracle
import paper_1604_07491_amd as lpk
from paper_1604_07491_amd import synth

pytestmark = pytest.mark.gpu


def _mix(count, seed0=50):
    lps = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        mb = int(rng.integers(60, 240))
        lps.append(synth.sparse_lp(mb, int(mb * rng.uniform(2.0, 3.0)), int(rng.integers(4, 8)), 2, seed=seed0 + i))
    return lps


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_results_identical_alone_and_in_mix(precision):
    lps = _mix(6)
    alone = []
    for lp in lps:
        with lpk.from_lp(lp, lpk.options(precision=precision)) as p:
            r = lpk.lp_solve(p)
            alone.append((r, lpk.lp_get_state(p)[:3]))
    probs = [lpk.from_lp(lp, lpk.options(precision=precision)) for lp in lps]
    res = lpk.lp_solve_batch(probs, width=3)
    for i, p in enumerate(probs):
        x, y, s, _ = lpk.lp_get_state(p)
        r0, (x0, y0, s0) = alone[i]
        assert res[i]["status"] == lpk.LP_OK and res[i]["iters"] == r0["iters"]
        assert res[i]["krylov_iters"] == r0["krylov_iters"]
        assert np.array_equal(x, x0) and np.array_equal(y, y0) and np.array_equal(s, s0)
        p.close()
    # and each agrees with the oracle's optimum
    for lp, (r0, _) in zip(lps[:3], alone[:3]):
        o = oracle.ipm(lp)
        assert abs(r0["pobj"] - o["pobj"]) <= 1e-7 * abs(o["pobj"])


def test_batch_mixed_groups_and_dense():
    """fp64 and mixed problems in one call form two groups; small dense (basis pursuit)
    problems run the Gram-matrix path in lockstep."""
    sp = _mix(3, seed0=20)
    bp = [synth.basis_pursuit_lp(64, 160, 6, seed=s) for s in (3, 4, 5)]
    mk = [
        lambda: lpk.from_lp(sp[0]),
        lambda: lpk.from_lp(sp[1], lpk.options(precision="mixed")),
        lambda: lpk.from_lp(sp[2]),
    ] + [(lambda lp=lp: lpk.lp_create_dense(lp.dense, lp.b, lp.c)) for lp in bp]
    alone = []
    for f in mk:
        with f() as q:
            r = lpk.lp_solve(q)
            alone.append((r, lpk.lp_get_state(q)[0]))
    made = [f() for f in mk]
    res = lpk.lp_solve_batch(made, width=2)
    for i, p in enumerate(made):
        assert res[i]["status"] == lpk.LP_OK
        assert res[i]["iters"] == alone[i][0]["iters"]
        assert np.array_equal(lpk.lp_get_state(p)[0], alone[i][1])
        p.close()


def test_batch_timing_replay():
    lps = _mix(4, seed0=30)
    probs = [lpk.from_lp(lp) for lp in lps]
    lpk.lp_solve_batch(probs, width=4)
    one = lpk.lp_time_kernel(probs[0], lpk.LP_K_SWEEP, reps=20)
    allb = lpk.lp_time_batch_kernel(probs, lpk.LP_K_SWEEP, reps=20)
    assert allb["us_per_launch"] > 0 and one["us_per_launch"] > 0
    # bytes are summed over the batch
    per = []
    for p in probs:
        t = lpk.lp_time_kernel(p, lpk.LP_K_SWEEP, reps=2)
        per.append(t["bytes_per_launch"] * t["launches_per_group"])
    assert abs(allb["bytes_per_launch"] * allb["launches_per_group"] - sum(per)) <= 1e-9 * sum(per)
    for p in probs:
        p.close()


def test_server_admission_and_results():
    lps = _mix(10, seed0=80)
    alone = {}
    for i, lp in enumerate(lps[:4]):
        with lpk.from_lp(lp) as p:
            lpk.lp_solve(p)
            alone[i] = lpk.lp_get_state(p)[0]
    fps = [lpk.lp_footprint_bytes(lp.m, lp.n, lp.nnz) for lp in lps]
    budget = int(2.5 * max(fps))          # at most two or three resident at once
    big = synth.sparse_lp(1500, 3500, 6, 2, seed=7)   # never fits this budget
    assert lpk.lp_footprint_bytes(big.m, big.n, big.nnz) > budget
    with lpk.Server(slots=4, max_skip=2, hbm_budget=budget) as srv:
        tickets = [srv.submit(lp) for lp in lps]
        tbig = srv.submit(big)
        bad = lps[0]
        with pytest.raises(lpk.LpError):
            rp = bad.row_ptr.copy(); rp[3] = rp[2]
            srv.submit(synth.LP(bad.m, bad.n, rp, bad.col_idx, bad.val, bad.b, bad.c))
        assert srv.wait(len(tickets) + 1, 300.0)
        done = {c["ticket"]: c for c in srv.poll()}
        assert set(done) == set(tickets) | {tbig}
        assert done[tbig]["status"] == lpk.LP_ETOOBIG
        for t in tickets:
            assert done[t]["status"] == lpk.LP_OK and done[t]["gamma_rel"] <= 1e-8
        # the running set never exceeded the budget
        ev = sorted([(done[t]["t_start"], done[t]["footprint"]) for t in tickets] +
                    [(done[t]["t_done"], -done[t]["footprint"]) for t in tickets], key=lambda e: (e[0], e[1]))
        cur = peak = 0
        for _, f in ev:
            cur += f
            peak = max(peak, cur)
        assert peak <= budget
        for i in range(4):
            x, y, s = srv.result(tickets[i])
            assert np.array_equal(x, alone[i])
        with pytest.raises(lpk.LpError):
            srv.result(tickets[0])      # released after the first fetch


def test_server_lanes_keep_results_bitwise():
    """The slots split into lanes (lockstep batches on streams of their own, rounds queued
    from one thread): every LP's solution is bitwise the same with 1, 2 and 3 lanes (3: an
    uneven split of 8 slots), and the same as alone."""
    lps = _mix(12, seed0=300)
    alone = []
    for lp in lps[:3]:
        with lpk.from_lp(lp) as p:
            lpk.lp_solve(p)
            alone.append(lpk.lp_get_state(p)[0])
    got = {}
    for lanes in (1, 2, 3):
        print(f"lanes {lanes}", flush=True)
        with lpk.Server(slots=8, lanes=lanes) as srv:
            tickets = [srv.submit(lp) for lp in lps]
            assert srv.wait(len(tickets), 300.0)
            done = {c["ticket"]: c for c in srv.poll()}
            assert set(done) == set(tickets)
            res = []
            for t in tickets:
                assert done[t]["status"] == lpk.LP_OK and done[t]["gamma_rel"] <= 1e-8
                res.append((done[t]["iters"], done[t]["krylov_iters"], srv.result(t)[0]))
            got[lanes] = res
    for lanes in (2, 3):
        for a, b in zip(got[1], got[lanes]):
            assert a[0] == b[0] and a[1] == b[1]
            assert np.array_equal(a[2], b[2])
    for i in range(3):
        assert np.array_equal(got[2][i][2], alone[i])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_mixes_lds_and_per_colour_sweeps(precision):
    """FP64: small LPs sweep in one block from LDS alone (row data staged); a 302 x 2000 LP
    keeps z in LDS and reads its rows from memory; a transportation LP with
    n = 8000 (each colour over 4 rounds of a block) sweeps colour by colour.  Mixed: the
    transportation LP, whose FP64 sweep cannot run from LDS, sweeps in FP32 (staged in LDS,
    where FP32 fits) while the others stay in FP64, in one batch whose launches each serve
    the LPs of their precision.  Each LP's result is bitwise as alone, and the optimum
    matches the oracle's."""
    lps = [synth.transport_lp(100, 80, seed=3)] + _mix(3, seed0=60) + [synth.sparse_lp(300, 2000, 6, 2, seed=61)]
    opts = lambda: lpk.options(precision=precision)
    alone = []
    for lp in lps:
        with lpk.from_lp(lp, opts()) as p:
            r = lpk.lp_solve(p)
            alone.append((r, lpk.lp_get_state(p)[0]))
    probs = [lpk.from_lp(lp, opts()) for lp in lps]
    res = lpk.lp_solve_batch(probs, width=len(lps))
    for i, p in enumerate(probs):
        assert res[i]["status"] == lpk.LP_OK
        assert res[i]["krylov_iters"] == alone[i][0]["krylov_iters"]
        assert np.array_equal(lpk.lp_get_state(p)[0], alone[i][1])
        p.close()
    o = oracle.ipm(lps[0])
    assert abs(alone[0][0]["pobj"] - o["pobj"]) <= 1e-7 * abs(o["pobj"])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_mixes_sliced_and_csr_colours(precision):
    """A transportation LP whose sink rows are stored in row slices (150 x 100), one whose
    sinks stay in CSR form (100 x 90: slices would pad by more than a quarter) and a small
    sparse LP in one batch: colour 1 then runs both the sliced and the CSR sweep launch, each
    skipping the other kind's LPs.  Every LP's result is bitwise as alone, and the sliced
    LP's optimum matches the oracle's."""
    lps = [synth.transport_lp(150, 100, seed=9), synth.transport_lp(100, 90, seed=3)] + _mix(1, seed0=70)
    opts = lambda: lpk.options(precision=precision)
    alone = []
    for lp in lps:
        with lpk.from_lp(lp, opts()) as p:
            r = lpk.lp_solve(p)
            alone.append((r, lpk.lp_get_state(p)[0]))
    print(f"{precision}: alone iterations", [a[0]["iters"] for a in alone], flush=True)
    probs = [lpk.from_lp(lp, opts()) for lp in lps]
    res = lpk.lp_solve_batch(probs, width=len(lps))
    for i, p in enumerate(probs):
        assert res[i]["status"] == lpk.LP_OK
        assert res[i]["krylov_iters"] == alone[i][0]["krylov_iters"]
        assert np.array_equal(lpk.lp_get_state(p)[0], alone[i][1])
        p.close()
    o = oracle.ipm(lps[0])
    assert abs(alone[0][0]["pobj"] - o["pobj"]) <= 1e-7 * abs(o["pobj"])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_narrow_graphs_keep_results_bitwise(precision):
    """Sixteen transportation LPs of one shape wait for each other's solves; while fewer
    than half of them still iterate, the engine launches narrower captures of the Krylov
    iterations (widths 8 here) over only those LPs.  Every LP's iterate is bitwise as alone
    and its Krylov count the same."""
    lps = [synth.transport_lp(30, 20, seed=100 + i) for i in range(16)]
    opts = lambda: lpk.options(precision=precision)
    alone = []
    for lp in lps:
        with lpk.from_lp(lp, opts()) as p:
            r = lpk.lp_solve(p)
            alone.append((r, lpk.lp_get_state(p)[0]))
    probs = [lpk.from_lp(lp, opts()) for lp in lps]
    res = lpk.lp_solve_batch(probs, width=16)
    ks = sorted(r["krylov_iters"] for r, _ in alone)
    print(f"{precision}: Krylov iterations alone {ks[0]}..{ks[-1]}", flush=True)
    for i, p in enumerate(probs):
        assert res[i]["status"] == lpk.LP_OK
        assert res[i]["krylov_iters"] == alone[i][0]["krylov_iters"]
        assert np.array_equal(lpk.lp_get_state(p)[0], alone[i][1])
        p.close()


def test_dots_task_width_keeps_results_bitwise():
    """The Gram-Schmidt dots reduce one, two or four basis columns per task, chosen by the
    launch width times the basis size; every column's dot takes the same reduction tree
    either way.  An LP whose late solves pass 254 iterations is solved alone (one column a
    task) and as 64 copies in one batch (four columns a task once k >= 254, two from 126):
    every copy's iterate is bitwise the alone one, with the same Krylov count."""
    lp = synth.sparse_lp(598, 1800, 6, 2, seed=7)
    with lpk.from_lp(lp) as p:
        ks = []
        for _ in range(99):
            info = lpk.ipm_step(p)
            ks += [info["k_af"], info["k_cc"]]
            if info["converged"]:
                break
    print(f"largest solve {max(ks)} iterations", flush=True)
    assert max(ks) >= 254
    with lpk.from_lp(lp) as p:
        r0 = lpk.lp_solve(p)
        x0 = lpk.lp_get_state(p)[0]
    probs = [lpk.from_lp(lp) for _ in range(64)]
    res = lpk.lp_solve_batch(probs, width=64)
    for i, p in enumerate(probs):
        assert res[i]["status"] == lpk.LP_OK
        assert res[i]["krylov_iters"] == r0["krylov_iters"]
        assert np.array_equal(lpk.lp_get_state(p)[0], x0)
        p.close()

"""Benchmark: interior-point LP solves per second on one MI355X.

Default workload: the serving mix.  256 sparse LPs (m ~ U{200..m_hi}, n = m U(2, 4), 4-10
nonzeros per column, seeds 1000 + i) go to the library's server, which keeps up to W of
them at once, split into L lockstep batches (lanes, each on its own stream, default 4),
admits new ones by HBM footprint and overlaps their work.
The K timed steps are closed-loop runs (every LP submitted at t = 0); a warm-up run comes
first.  Then an open-loop run offers 0.8 x that capacity as a seeded Poisson trace, for the
latencies, and both runs repeat in the other precision.  Prints one JSON line:

  value         converged LPs (status OK, gamma_rel <= 1e-8) per second, closed loop
  p50_ms/p99_ms latency from submission to completion in the open-loop run
  roofline      the kernel class with the most time per Krylov iteration in the mix's
                batch, timed by replaying its launches for W LPs back-to-back between two
                HIP events on the library's stream (lp_time_batch_kernel); achieved =
                algorithmic bytes per launch (summed over the LPs) / mean launch duration
  cpu_baseline  the CPU FP64 oracle on a seeded sample of the mix (about 20 s, one core)

The stated mix goes to m = 20,000; its whole-run cost is beyond any single-GPU run (the
design notes give the oracle's Krylov counts), so m_hi is 1000 unless --m-hi says otherwise.

Other workloads (--workload): transport_300x300 (64 transportation LPs per step, 64 in
lockstep), sparse_200x500, bounded_200x500 (general bounds, reduced to the standard form by
lp_create_bounded), basis_pursuit_1024x16384, sparse_120000x434580 (with --ipm-steps),
streaming_1199000x4345800 (kernel bandwidth outside the Infinity Cache), copy_probe
(counter calibration).  Method flags: --krylov (abgmres, cgne, mrne, bagmres), --inner
(nesor, nessor, cimmino), --precision (fp64, mixed), --correctors K.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6


def kernels_digest(files=("sweep.hip", "kernels.h")):
    """sha256 of the sweep kernels' source and of the header that sizes their launches, which
    the committed counter runs were taken on (the one-block sweep: sweep_lds.hip)."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_1604_07491_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def counter_traffic(args, kernel, width, precision=None, files=("sweep.hip", "kernels.h")):
    """HBM bytes per launch of `kernel` from the committed counter runs, if they were taken
    for this workload and batch width on the kernels as they are now (else None)."""
    if not args.traffic or not os.path.exists(args.traffic):
        return None
    key = f"{args.workload}/{precision or args.precision}/w{width}/{kernel}"
    if args.inner != "nesor" or args.krylov != "abgmres":
        key += f"/{args.inner}/{args.krylov}"
    rec = json.load(open(args.traffic)).get(key)
    if not rec or rec.get("kernels_sha256") != kernels_digest(files):
        return None
    return rec["bytes_per_launch"]


def make_lps(workload, count):
    from paper_1604_07491_amd import synth
    if workload == "transport_300x300":
        return [synth.transport_lp(300, 300, seed=1 + i) for i in range(count)]
    if workload == "sparse_200x500":
        return [synth.sparse_lp(198, 500, 6, 2, seed=i, name="sparse_200x500") for i in range(count)]
    if workload == "basis_pursuit_1024x16384":
        return [synth.basis_pursuit_lp(1024, 8192, 64, seed=2 + i) for i in range(count)]
    if workload == "sparse_120000x434580":
        return [synth.config(3)]
    if workload == "bounded_200x500":
        # general bounds (lower, box, upper-only, free, fixed), reduced to the standard form
        # by the library; lo and hi ride along on the generator's LP
        out = []
        for i in range(count):
            lp, lo, hi = synth.bounded_lp(198, 500, 6, 2, seed=i)
            lp.lo, lp.hi = lo, hi
            out.append(lp)
        return out
    raise ValueError(workload)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (serving mix: closed-loop runs of the whole mix) [3]")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="serving_mix",
                    choices=["transport_300x300", "sparse_200x500", "basis_pursuit_1024x16384",
                             "sparse_120000x434580", "serving_mix", "streaming_1199000x4345800",
                             "bounded_200x500", "copy_probe"])
    ap.add_argument("--ipm-steps", type=int, default=0,
                    help="time this many interior-point steps of the first LP instead of whole solves")
    ap.add_argument("--krylov-cap", type=int, default=1500,
                    help="serving_mix: Krylov basis cap per solve (stated cap of the mix)")
    ap.add_argument("--m-hi", type=int, default=1000,
                    help="serving_mix: largest m of the mix (the stated mix goes to 20000; see the design notes)")
    ap.add_argument("--precision-mix", default="mixed", choices=["fp64", "mixed"],
                    help="serving_mix: the precision the value is quoted for (the other is run for comparison)")
    ap.add_argument("--load", type=float, default=0.8,
                    help="serving_mix: offered load as a fraction of the closed-loop mixed throughput")
    ap.add_argument("--batch", type=int, default=None, help="LPs per step [serving mix 256; others 64]")
    ap.add_argument("--width", type=int, default=None, help="LPs in lockstep [serving mix 256; others 64]")
    ap.add_argument("--lanes", type=int, default=4,
                    help="serving mix: lockstep batches the width is split into, each on its own stream [4]")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--inner", default="nesor", choices=["nesor", "nessor", "cimmino"])
    ap.add_argument("--schedule", type=int, default=0, choices=[0, 1, 2],
                    help="batch phases: 0 auto, 1 together, 2 each LP alone")
    ap.add_argument("--krylov", default="abgmres", choices=["abgmres", "cgne", "mrne", "bagmres"],
                    help="outer iteration: AB-GMRES (Sec. 3.2), CGNE / MRNE (Sec. 3.3) or BA-GMRES (eq. ba_ne)")
    ap.add_argument("--correctors", type=int, default=0,
                    help="multiple centrality correctors per interior-point step (0: Mehrotra's method)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--replay-only", action="store_true",
                    help="serving mix: only the kernel-class replay of the roofline (for counter runs)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "counters.json"),
                    help="counter-derived HBM bytes per launch (FETCH_SIZE/WRITE_SIZE runs)")
    args = ap.parse_args()
    serving = args.workload == "serving_mix"
    if args.steps is None:
        args.steps = 3
    if args.batch is None:
        args.batch = 256 if serving else 64
    if args.width is None:
        args.width = 256 if serving else 64
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (independent LPs would shard "
                                   "across GPUs with no exchange; that path is not built)"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1604_07491_amd as lpk

    torch.cuda.set_device(0)
    if args.workload == "serving_mix":
        return serve_main(args)
    if args.workload == "streaming_1199000x4345800":
        return streaming_main(args)
    if args.workload == "copy_probe":
        # a plain device copy of known size: the reference that scales the HBM byte
        # counters (FETCH_SIZE, WRITE_SIZE) read for the library's kernels
        nbytes = 1 << 30
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(5):
            dst.copy_(src)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / 5
        print(json.dumps({"metric": "device copy", "bytes_read_per_copy": nbytes, "bytes_written_per_copy": nbytes,
                          "copies": 5, "ms_per_copy": ms, "gbs": 2 * nbytes / (ms * 1e-3) / 1e9}), flush=True)
        return
    if args.ipm_steps > 0:
        return steps_main(args)
    lps = make_lps(args.workload, args.batch)
    dev = lambda a: torch.as_tensor(np.asarray(a)).cuda()
    opts = lpk.options(precision=args.precision, inner=args.inner, krylov=args.krylov, schedule=args.schedule,
                       max_correctors=args.correctors)
    probs = []
    for lp in lps:
        if lp.dense is not None:
            probs.append(lpk.lp_create_dense(dev(lp.dense), dev(lp.b), dev(lp.c), opts))
        elif hasattr(lp, "lo"):
            probs.append(lpk.lp_create_bounded(lp.m, lp.n, dev(lp.row_ptr), dev(lp.col_idx), dev(lp.val),
                                               dev(lp.b), dev(lp.c), dev(lp.lo), dev(lp.hi), opts))
        else:
            probs.append(lpk.lp_create(lp.m, lp.n, dev(lp.row_ptr), dev(lp.col_idx), dev(lp.val), dev(lp.b),
                                       dev(lp.c), opts))
    torch.cuda.synchronize()
    print(f"created {len(probs)} LPs of {args.workload}", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        lpk.lp_solve_batch(probs, args.width)
    torch.cuda.synchronize()
    lat, res = [], []
    t0 = time.perf_counter()
    for step in range(args.steps):
        out = lpk.lp_solve_batch(probs, args.width)
        res += out
        lat += [r["seconds"] for r in out]
        print(f"step {step} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    n_ok = sum(1 for r in res if r["status"] == lpk.LP_OK and r["gamma_rel"] <= 1e-8)
    ok = n_ok == len(res)

    # one LP alone: its latency, and a profiled solve to find the dominant kernel class
    p0 = probs[0]
    alone = []
    for _ in range(2):
        alone.append(lpk.lp_solve(p0)["seconds"])
    lpk.lp_profile(p0, (1 << lpk.LP_K_COUNT) - 1)
    r0 = lpk.lp_solve(p0)
    stats = lpk.lp_profile_read(p0)
    lpk.lp_profile(p0, 0)
    cls_id = {"sweep": lpk.LP_K_SWEEP, "spmv_csr": lpk.LP_K_SPMV_CSR, "spmv_csc": lpk.LP_K_SPMV_CSC,
              "gs_dots": lpk.LP_K_GS_DOTS, "gs_update": lpk.LP_K_GS_UPDATE, "gram": lpk.LP_K_GRAM}
    timed = {k: v for k, v in stats.items() if k in cls_id and v["launches"] > 0}
    dom = max(timed, key=lambda k: timed[k]["ms_total"])
    # the dominant class for the batch as it runs in the timed steps
    width = min(args.width, len(probs))
    tk = lpk.lp_time_batch_kernel(probs[:width], cls_id[dom], reps=200 if dom != "gram" else 5)
    achieved = tk["bytes_per_launch"] / (tk["us_per_launch"] * 1e-6) / 1e9
    t1 = lpk.lp_time_kernel(p0, cls_id[dom], reps=200 if dom != "gram" else 5)
    if dom == "gram":
        # the dense path's build is a contraction: FP64 matrix cores
        achieved = tk["flops_per_launch"] / (tk["us_per_launch"] * 1e-6) / 1e12
    traffic = counter_traffic(args, dom, width)
    bound, peak, unit = ("mfma", FP64_MFMA_PEAK_TFLOPS, "TFLOP/s") if dom == "gram" else ("hbm", HBM_PEAK_GBS, "GB/s")
    roofline = {"bound": bound, "kernel": dom, "achieved": achieved, "peak": peak, "unit": unit,
                "frac": achieved / peak, "traffic": traffic, "us_per_launch": tk["us_per_launch"],
                "bytes_per_launch": tk["bytes_per_launch"], "launches_per_group": tk["launches_per_group"],
                "lps_per_launch": width,
                "timing": "lp_time_batch_kernel replay, 200 x group, HIP events on the library stream",
                "single_lp": {"us_per_launch": t1["us_per_launch"], "bytes_per_launch": t1["bytes_per_launch"],
                              "achieved": t1["bytes_per_launch"] / (t1["us_per_launch"] * 1e-6) / 1e9}}
    extra = {"batch_kernels": {}}
    for name in ("sweep", "spmv_csr", "spmv_csc", "gs_dots", "gs_update"):
        if name not in timed:
            continue
        tb = lpk.lp_time_batch_kernel(probs[:width], cls_id[name], reps=200)
        gbs = tb["bytes_per_launch"] / (tb["us_per_launch"] * 1e-6) / 1e9
        extra["batch_kernels"][name] = {"us_per_launch": tb["us_per_launch"], "gbs": gbs,
                                        "frac": gbs / HBM_PEAK_GBS, "launches_per_group": tb["launches_per_group"]}
    if "gram" in timed:
        tg = lpk.lp_time_kernel(p0, lpk.LP_K_GRAM, reps=5)
        extra["dense_build"] = {"bound": "mfma", "ms": tg["us_per_launch"] / 1e3,
                                "achieved_tflops": tg["flops_per_launch"] / (tg["us_per_launch"] * 1e-6) / 1e12,
                                "peak_tflops": FP64_MFMA_PEAK_TFLOPS}
        extra["dense_build"]["frac"] = extra["dense_build"]["achieved_tflops"] / FP64_MFMA_PEAK_TFLOPS

    cpu = None
    if not args.no_cpu_baseline and lps[0].dense is None and lps[0].n <= 200000:
        import oracle
        tc = time.perf_counter()
        so = oracle.solver_opts(krylov={"abgmres": oracle.ABGMRES, "cgne": oracle.CGNE, "mrne": oracle.MRNE,
                                          "bagmres": oracle.BAGMRES}[args.krylov],
                                inner={"nesor": oracle.NESOR, "nessor": oracle.NESSOR, "cimmino": oracle.CIMMINO}[args.inner])
        io = oracle.ipm_opts(solver=so, max_correctors=args.correctors)
        if hasattr(lps[0], "lo"):
            from oracle import bounds
            o = bounds.ipm_bounded(lps[0].to_dense(), lps[0].b, lps[0].c, lps[0].lo, lps[0].hi, io)
        else:
            o = oracle.ipm(lps[0], io)
        tcpu = time.perf_counter() - tc
        cpu = {"value": 1.0 / tcpu, "unit": "LPs/s", "cores": 1, "kind": "oracle",
               "sample": f"1 full solve of the {args.workload} LP ({o['iters']} IPM iterations, {tcpu:.2f} s)",
               "objective_rel_err_gpu_vs_oracle": abs(r0["pobj"] - o["pobj"]) / abs(o["pobj"])}

    lat_ms = np.array(lat) * 1e3
    line = {
        "metric": "LPs solved/s at rel. gap 1e-8 (p50/p99 latency; Krylov+NE-SOR kernel HBM GB/s)",
        "value": n_ok / total,
        "unit": "LPs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total / args.steps * 1e3,
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "latency_alone_ms": float(np.median(alone) * 1e3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 sweeps + f64",
        "data": "synthetic",
        "all_converged": ok,
        "ipm_iters": r0["iters"],
        "krylov_iters": r0["krylov_iters"],
        "gamma_rel": r0["gamma_rel"],
        "config": {"workload": args.workload, "m": lps[0].m, "n": lps[0].n, "nnz": lps[0].nnz,
                   **({"standard_form": {"m": p0.m, "n": p0.n}} if hasattr(lps[0], "lo") else {}),
                   "lps_per_step": len(probs), "lps_in_lockstep": args.width,
                   "precision": args.precision, "inner": args.inner,
                   "krylov": {"abgmres": "AB-GMRES", "cgne": "CGNE", "mrne": "MRNE", "bagmres": "BA-GMRES"}[args.krylov],
                   "inner_sweeps": 2, "omega": 1.0, "schedule": args.schedule,
                   "max_correctors": args.correctors},
        "roofline": roofline,
        "kernel_classes": {k: {"launches": v["launches"], "ms_total": v["ms_total"],
                               "us_per_launch_event_bracketed": v["ms_total"] * 1e3 / max(v["launches"], 1)}
                           for k, v in stats.items() if v["launches"] > 0},
        "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)
    for p in probs:
        p.close()


def kernel_roofline(p, classes, reps=20):
    """lp_time_kernel for each class: mean launch duration, algorithmic bytes per launch,
    GB/s and the fraction of the 8 TB/s HBM peak; 'group' is one preconditioner
    application (all colours and sweeps) for the sweep class."""
    import paper_1604_07491_amd as lpk
    out = {}
    for name, cls in classes.items():
        t = lpk.lp_time_kernel(p, cls, reps=reps)
        gbs = t["bytes_per_launch"] / (t["us_per_launch"] * 1e-6) / 1e9
        out[name] = {"us_per_launch": t["us_per_launch"], "bytes_per_launch": t["bytes_per_launch"],
                     "launches_per_group": t["launches_per_group"],
                     "us_per_group": t["us_per_launch"] * t["launches_per_group"],
                     "achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS}
        print(f"  {name}: {out[name]}", file=sys.stderr, flush=True)
    return out


def streaming_main(args):
    """Kernel bandwidth on an instance larger than the Infinity Cache: the config-3
    generator at 10x (m = 1.2M, n = 4.35M, 34.8M nonzeros; A_hat in CSR and CSC is 0.84 GB
    in FP64).  One direction solve at D = I builds A_hat; then the sweep and the two
    products of the Krylov loop are timed by replay."""
    import numpy as np
    import paper_1604_07491_amd as lpk
    from paper_1604_07491_amd import synth
    t0 = time.perf_counter()
    lp = synth.streaming_lp(10)
    print(f"generated {lp.m}x{lp.n}, nnz {lp.nnz} in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    res = {}
    for prec in ("mixed", "fp64"):
        t0 = time.perf_counter()
        p = lpk.from_lp(lp, lpk.options(precision=prec, krylov_max_iter=8))
        tc = time.perf_counter() - t0
        ncol = len(p.colouring())
        print(f"{prec}: created in {tc:.1f} s", file=sys.stderr, flush=True)
        dw, dy, info = lpk.direction_solve(p, np.ones(lp.n), lp.b, 1e-12)
        res[prec] = kernel_roofline(p, {"sweep": lpk.LP_K_SWEEP, "spmv_csr": lpk.LP_K_SPMV_CSR,
                                        "spmv_csc": lpk.LP_K_SPMV_CSC}, reps=args.steps if args.steps > 3 else 10)
        res[prec]["create_s"] = tc
        res[prec]["colours"] = ncol
        p.close()
    sw = res["mixed"]["sweep"]
    line = {"metric": "inner-iteration sweep HBM GB/s (instance larger than the Infinity Cache)",
            "value": sw["achieved_gbs"], "unit": "GB/s", "n_gpus": 1, "higher_is_better": True,
            "dtype": "f32 sweeps + f64", "data": "synthetic",
            "config": {"workload": "streaming_1199000x4345800", "m": lp.m, "n": lp.n, "nnz": lp.nnz},
            "kernels": res}
    print(json.dumps(line), flush=True)


def steps_main(args):
    """Time `ipm_steps` interior-point steps of the workload LP (the starting point is the
    first call's); for LPs whose whole solve takes hours."""
    import paper_1604_07491_amd as lpk
    lp = make_lps(args.workload, 1)[0]
    t0 = time.perf_counter()
    p = lpk.from_lp(lp, lpk.options(precision=args.precision, inner=args.inner))
    tc = time.perf_counter() - t0
    print(f"created {lp.m}x{lp.n} nnz {lp.nnz} in {tc:.1f} s", file=sys.stderr, flush=True)
    steps = []
    for k in range(args.ipm_steps):
        ts = time.perf_counter()
        info = lpk.ipm_step(p)
        dt = time.perf_counter() - ts
        steps.append({"s": dt, "k_af": info["k_af"], "k_cc": info["k_cc"], "gamma_rel": info["gamma_rel"],
                      "fail_af": info["fail_af"], "fail_cc": info["fail_cc"], "eps_in": info["eps_in"]})
        print(f"step {k}: {steps[-1]}", file=sys.stderr, flush=True)
        if info["converged"]:
            break
    kr = kernel_roofline(p, {"sweep": lpk.LP_K_SWEEP, "spmv_csr": lpk.LP_K_SPMV_CSR,
                             "spmv_csc": lpk.LP_K_SPMV_CSC})
    line = {"metric": "interior-point steps (time per step, Krylov iterations)", "value":
            len(steps) / sum(s["s"] for s in steps), "unit": "IPM steps/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f64" if args.precision == "fp64" else "f32 sweeps + f64",
            "data": "synthetic", "config": {"workload": args.workload, "m": lp.m, "n": lp.n, "nnz": lp.nnz,
                                            "precision": args.precision, "create_s": tc},
            "steps": steps, "kernels": kr}
    print(json.dumps(line), flush=True)
    p.close()


def _serve_run(lps, arrivals, precision, width, cap, lanes=1):
    """Submit every LP at its arrival time (seconds from the first) to a server; return the
    completions and the wall time from the first arrival to the last completion."""
    import paper_1604_07491_amd as lpk
    solver = lpk.options(precision=precision, krylov_max_iter=cap)
    with lpk.Server(slots=width, solver=solver, lanes=lanes) as srv:
        t0 = time.perf_counter()
        tickets = {}
        for i, (lp, ta) in enumerate(zip(lps, arrivals)):
            delay = ta - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets[srv.submit(lp)] = i
        done = []
        while len(done) < len(lps):
            srv.wait(len(lps) - len(done), 30.0)
            got = srv.poll()
            done += got
            print(f"  completed {len(done)} / {len(lps)}", file=sys.stderr, flush=True)
        wall = max(c["t_done"] for c in done) - min(c["t_submit"] for c in done)
    return done, wall


def _converged(done):
    import paper_1604_07491_amd as lpk
    return [c for c in done if c["status"] == lpk.LP_OK and c["gamma_rel"] <= 1e-8]


def _mix_roofline(lps, precision, width, args=None):
    """The kernel classes of the serving mix timed as the batch runs them: every LP of the
    mix created on the device, scaled by one short direction solve, then each class's
    launches for `width` LPs replayed back-to-back between two HIP events on the library's
    stream (lp_time_batch_kernel).  The dominant class is the one with the most time per
    Krylov iteration (launches per iteration x duration)."""
    import numpy as np
    import torch
    import paper_1604_07491_amd as lpk
    dev = lambda a: torch.as_tensor(np.asarray(a)).cuda()
    probs = []
    for lp in lps[:width]:
        p = lpk.lp_create(lp.m, lp.n, dev(lp.row_ptr), dev(lp.col_idx), dev(lp.val), dev(lp.b), dev(lp.c),
                          lpk.options(precision=precision))
        lpk.direction_solve(p, dev(np.ones(lp.n)), dev(lp.b), 0.5)   # one scaling (D = I)
        probs.append(p)
    torch.cuda.synchronize()
    layouts = [p.sweep_layout() for p in probs]
    per_iter = {"sweep": lpk.LP_K_SWEEP, "spmv_csr": lpk.LP_K_SPMV_CSR, "gs_dots": lpk.LP_K_GS_DOTS,
                "gs_update": lpk.LP_K_GS_UPDATE}
    if any(f for f, _ in layouts):
        per_iter["spmv_csc"] = lpk.LP_K_SPMV_CSC
    classes = {}
    for name, cls in per_iter.items():
        t = lpk.lp_time_batch_kernel(probs, cls, reps=20)
        k = t["launches_per_group"]   # the class's launches in one Krylov iteration
        if k == 0:
            # the product u = A_hat z_k of LPs whose one-block sweep forms it: no launch
            print(f"  {name}: no launches (formed inside the sweep)", file=sys.stderr, flush=True)
            continue
        gbs = t["bytes_per_launch"] / (t["us_per_launch"] * 1e-6) / 1e9
        classes[name] = {"us_per_launch": t["us_per_launch"], "bytes_per_launch": t["bytes_per_launch"],
                         "launches_per_iteration": k, "us_per_iteration": k * t["us_per_launch"], "gbs": gbs,
                         "frac": gbs / HBM_PEAK_GBS}
        print(f"  {name}: {classes[name]}", file=sys.stderr, flush=True)
    for p in probs:
        p.close()
    dom = max(classes, key=lambda k: classes[k]["us_per_iteration"])
    c = classes[dom]
    # HBM bytes per launch from the committed counter runs of this replay (FETCH_SIZE and
    # WRITE_SIZE, scaled by a plain copy's), while the sweep kernels are unchanged
    files = ("sweep_lds.hip", "kernels.h") if all(kk != 0 for _, kk in layouts) else ("sweep.hip", "sweep_lds.hip", "kernels.h")
    traffic = counter_traffic(args, dom, len(probs), precision, files) if args is not None else None
    roofline = {"bound": "hbm", "kernel": dom, "achieved": c["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": c["frac"], "traffic": traffic, "us_per_launch": c["us_per_launch"],
                "bytes_per_launch": c["bytes_per_launch"], "lps_per_launch": len(probs),
                "timing": "lp_time_batch_kernel replay, 20 x group, HIP events on the library stream"}
    if dom == "sweep":
        roofline["note"] = ("one workgroup per LP sweeps every colour with block barriers between them (a "
                            "chain of 2 x colours dependent steps of 1-2 us, bound by latency, not bandwidth), "
                            "then forms u = A_hat z_k from its z for AB-GMRES")
    kinds = {k: sum(1 for _, kk in layouts if kk == k) for k in (0, 1, 2)}
    return roofline, classes, {"fp32_sweeps": sum(f for f, _ in layouts), "staged_in_lds": kinds[2],
                               "z_in_lds_rows_from_memory": kinds[1], "colour_by_colour": kinds[0]}


def serve_main(args):
    """Serving mix: LPs of different sizes arrive; the server keeps up to `width` of them in
    one lockstep batch, admits new ones by HBM footprint as others finish, and overlaps
    their work.  value: closed-loop capacity (every LP submitted at t = 0), converged LPs
    per second over the timed runs.  Latency: an open-loop run offering `load` times that
    capacity as a seeded Poisson trace, p50 / p99 from submission to completion.  Both
    precisions run the same LPs and the same trace."""
    import numpy as np
    import paper_1604_07491_amd as lpk
    from paper_1604_07491_amd import synth
    count = args.batch
    width = min(args.width, count)
    lps, unit = synth.serving_mix(count=count, m_hi=args.m_hi, rate=1.0)
    print(f"generated {count} LPs (m {min(l.m for l in lps)}..{max(l.m for l in lps)})", file=sys.stderr,
          flush=True)
    prec = args.precision_mix
    if args.replay_only:
        roofline, classes, layout = _mix_roofline(sorted(lps, key=lambda l: -l.m), prec, width, args)
        print(json.dumps({"roofline": roofline, "batch_kernels": classes, "sweep_layout": layout}), flush=True)
        return
    for _ in range(args.warmup):
        done, wall = _serve_run(lps, np.zeros(count), prec, width, args.krylov_cap, args.lanes)
        print(f"warm-up closed loop {prec}: {len(_converged(done)) / wall:.2f} LPs/s", file=sys.stderr, flush=True)
    closed = {}
    walls, conv = [], []
    for step in range(args.steps):
        done, wall = _serve_run(lps, np.zeros(count), prec, width, args.krylov_cap, args.lanes)
        walls.append(wall)
        conv.append(len(_converged(done)))
        print(f"step {step}: closed loop {prec} {conv[-1] / wall:.2f} LPs/s", file=sys.stderr, flush=True)
    closed[prec] = {"lps_per_s": sum(conv) / sum(walls), "wall_s": sum(walls) / len(walls),
                    "converged": min(conv), "lps": count,
                    "krylov_iters_total": int(sum(c["krylov_iters"] for c in done))}
    other = "fp64" if prec == "mixed" else "mixed"
    done, wall = _serve_run(lps, np.zeros(count), other, width, args.krylov_cap, args.lanes)
    closed[other] = {"lps_per_s": len(_converged(done)) / wall, "wall_s": wall, "converged": len(_converged(done)),
                     "lps": count, "krylov_iters_total": int(sum(c["krylov_iters"] for c in done))}
    print(f"closed loop {other}: {closed[other]}", file=sys.stderr, flush=True)
    rate = args.load * closed[prec]["lps_per_s"]
    arrivals = unit / rate          # unit-rate Poisson trace scaled to the offered rate
    out = {}
    for pr in (prec, other):
        done, wall = _serve_run(lps, arrivals, pr, width, args.krylov_cap, args.lanes)
        lat = np.array([c["t_done"] - c["t_submit"] for c in done]) * 1e3
        ok = _converged(done)
        out[pr] = {"lps_per_s": len(ok) / wall, "wall_s": wall, "p50_ms": float(np.percentile(lat, 50)),
                   "p99_ms": float(np.percentile(lat, 99)), "converged": len(ok),
                   "max_gamma_rel": max(c["gamma_rel"] for c in done),
                   "krylov_iters_total": int(sum(c["krylov_iters"] for c in done)),
                   "ipm_iters_total": int(sum(c["iters"] for c in done))}
        print(f"open loop {pr}: {out[pr]}", file=sys.stderr, flush=True)
    roofline, classes, layout = _mix_roofline(sorted(lps, key=lambda l: -l.m), prec, width, args)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        # LPs of the mix in a seeded random order until about 20 s of CPU work
        order = np.random.default_rng(7).permutation(count)
        tc = time.perf_counter()
        done_cpu = 0
        for i in order:
            oracle.ipm(lps[int(i)])
            done_cpu += 1
            if time.perf_counter() - tc > 20.0:
                break
        tcpu = time.perf_counter() - tc
        cpu = {"value": done_cpu / tcpu, "unit": "LPs/s", "cores": 1, "kind": "oracle",
               "sample": f"{done_cpu} LPs of the mix in seeded random order, one core, {tcpu:.1f} s"}
    c = closed[prec]
    o = out[prec]
    line = {
        "metric": "LPs solved/s at rel. gap 1e-8 (p50/p99 latency), serving mix",
        "value": c["lps_per_s"], "unit": "LPs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": c["wall_s"] * 1e3, "p50_ms": o["p50_ms"], "p99_ms": o["p99_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if layout["fp32_sweeps"] == 0 else "f32 sweeps + f64", "data": "synthetic",
        "all_converged": c["converged"] == count and o["converged"] == count,
        "config": {"workload": "serving_mix", "lps": count, "m_range": [200, args.m_hi],
                   "stated_m_range": [200, 20000], "n": "m x U(2, 4)", "nnz_per_column": "U{4..10}",
                   "seeds": "1000 + i", "arrival": "Poisson, seed 4242", "offered_load": args.load,
                   "rate_per_s": rate, "lps_in_lockstep": width, "lanes": args.lanes, "precision": prec, "krylov": "AB-GMRES",
                   "inner": "NE-SOR", "inner_sweeps": 2, "omega": 1.0, "krylov_cap": args.krylov_cap,
                   "sweep_layout": layout},
        "closed_loop": closed, "open_loop": out,
        "mixed_over_fp64": closed["mixed"]["lps_per_s"] / closed["fp64"]["lps_per_s"],
        "roofline": roofline, "batch_kernels": classes,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

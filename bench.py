"""Benchmark: interior-point LP solves per second on one MI355X.

One step solves B LPs of the workload's shape (distinct seeds; the first is the workload
LP itself) to a relative duality gap of 1e-8, up to W of them in lockstep (lp_solve_batch:
each phase of an interior-point iteration is one launch for the whole batch; a finished
LP leaves and a waiting one joins).  Inputs are created on the device before the timed
region (torch tensors handed to lp_create), so `value` excludes host-to-device copies.
Prints one JSON line:

  value         LPs solved per second over the K timed steps (all B x K solves)
  p50_ms/p99_ms per-LP latency inside the timed steps (joining the batch to leaving it)
  roofline      the dominant kernel class of a profiled solve, timed for the batch as it
                runs (lp_time_batch_kernel: one launch covers all W LPs) by replaying its
                launches back-to-back between two HIP events on the library's stream;
                achieved = algorithmic bytes per launch (summed over the W LPs) / mean
                launch duration
  cpu_baseline  the CPU FP64 oracle on the workload LP (one full solve, one core)
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
    raise ValueError(workload)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="transport_300x300",
                    choices=["transport_300x300", "sparse_200x500", "basis_pursuit_1024x16384",
                             "sparse_120000x434580"])
    ap.add_argument("--batch", type=int, default=64, help="LPs per step")
    ap.add_argument("--width", type=int, default=64, help="LPs in lockstep")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--inner", default="nesor", choices=["nesor", "cimmino"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic", default=None, help="JSON file: counter-derived bytes per launch by kernel class")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1604_07491_amd as lpk

    torch.cuda.set_device(0)
    lps = make_lps(args.workload, args.batch)
    dev = lambda a: torch.as_tensor(np.asarray(a)).cuda()
    opts = lpk.options(precision=args.precision, inner=args.inner)
    probs = []
    for lp in lps:
        if lp.dense is not None:
            probs.append(lpk.lp_create_dense(dev(lp.dense), dev(lp.b), dev(lp.c), opts))
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
    ok = all(r["status"] == lpk.LP_OK and r["gamma_rel"] <= 1e-8 for r in res)

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
              "gram": lpk.LP_K_GRAM}
    timed = {k: v for k, v in stats.items() if k in cls_id and v["launches"] > 0}
    dom = max(timed, key=lambda k: timed[k]["ms_total"])
    # the dominant class for the batch as it runs in the timed steps
    width = min(args.width, len(probs))
    tk = lpk.lp_time_batch_kernel(probs[:width], cls_id[dom], reps=200 if dom != "gram" else 5)
    achieved = tk["bytes_per_launch"] / (tk["us_per_launch"] * 1e-6) / 1e9
    t1 = lpk.lp_time_kernel(p0, cls_id[dom], reps=200 if dom != "gram" else 5)
    traffic = None
    if args.traffic and os.path.exists(args.traffic):
        traffic = json.load(open(args.traffic)).get(args.workload, {}).get(dom)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "us_per_launch": tk["us_per_launch"],
                "bytes_per_launch": tk["bytes_per_launch"], "launches_per_group": tk["launches_per_group"],
                "lps_per_launch": width,
                "timing": "lp_time_batch_kernel replay, 200 x group, HIP events on the library stream",
                "single_lp": {"us_per_launch": t1["us_per_launch"], "bytes_per_launch": t1["bytes_per_launch"],
                              "achieved": t1["bytes_per_launch"] / (t1["us_per_launch"] * 1e-6) / 1e9}}
    extra = {}
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
        o = oracle.ipm(lps[0])
        tcpu = time.perf_counter() - tc
        cpu = {"value": 1.0 / tcpu, "unit": "LPs/s", "cores": 1, "kind": "oracle",
               "sample": f"1 full solve of the {args.workload} LP ({o['iters']} IPM iterations, {tcpu:.2f} s)",
               "objective_rel_err_gpu_vs_oracle": abs(r0["pobj"] - o["pobj"]) / abs(o["pobj"])}

    lat_ms = np.array(lat) * 1e3
    line = {
        "metric": "LPs solved/s at rel. gap 1e-8 (p50/p99 latency; Krylov+NE-SOR kernel HBM GB/s)",
        "value": len(res) / total,
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
                   "lps_per_step": len(probs), "lps_in_lockstep": args.width,
                   "precision": args.precision, "inner": args.inner, "krylov": "AB-GMRES",
                   "inner_sweeps": 2, "omega": 1.0},
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


if __name__ == "__main__":
    main()

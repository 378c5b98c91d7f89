"""Benchmark: interior-point LP solves per second on one MI355X.

One step = one whole lp_solve (starting point, every interior-point iteration with its
predictor and corrector direction solves) of the workload LP, inputs resident in HBM
(created once from torch device tensors).  Prints one JSON line:

  value        LPs solved per second over the K timed steps (rel. gap <= 1e-8 each)
  p50/p99      per-solve latency (ms); p99 of K samples is their maximum for K < 100
  roofline     the dominant kernel class of the solve (largest total time in a profiled
               solve run after the timed steps), HIP-event timed per launch on the
               library's stream: algorithmic bytes per launch / mean launch duration
  cpu_baseline the CPU FP64 oracle on the same LP (one full solve, one core)
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="transport_300x300",
                    choices=["transport_300x300", "sparse_200x500", "basis_pursuit_1024x16384"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--inner", default="nesor", choices=["nesor", "cimmino"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic", default=None, help="JSON file with counter-derived bytes per launch")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1604_07491_amd as lpk
    from paper_1604_07491_amd import synth

    lp = {"transport_300x300": lambda: synth.config(1), "sparse_200x500": lambda: synth.config(0),
          "basis_pursuit_1024x16384": lambda: synth.config(2)}[args.workload]()
    torch.cuda.set_device(0)
    dev = lambda a: torch.as_tensor(np.asarray(a)).cuda()
    opts = lpk.options(precision=args.precision, inner=args.inner)
    if lp.dense is not None:
        p = lpk.lp_create_dense(dev(lp.dense), dev(lp.b), dev(lp.c), opts)
    else:
        p = lpk.lp_create(lp.m, lp.n, dev(lp.row_ptr), dev(lp.col_idx), dev(lp.val), dev(lp.b), dev(lp.c), opts)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        r = lpk.lp_solve(p)
    torch.cuda.synchronize()
    lat = []
    res = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        t = time.perf_counter()
        r = lpk.lp_solve(p)
        lat.append(time.perf_counter() - t)
        res.append(r)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ok = all(r["status"] == lpk.LP_OK and r["gamma_rel"] <= 1e-8 for r in res)

    # profiled solve (not timed): per-launch HIP events of every kernel class
    lpk.lp_profile(p, (1 << lpk.LP_K_COUNT) - 1)
    lpk.lp_solve(p)
    stats = lpk.lp_profile_read(p)
    lpk.lp_profile(p, 0)
    dom = max(stats, key=lambda k: stats[k]["ms_total"])
    st = stats[dom]
    per_launch_s = st["ms_total"] / 1e3 / max(st["launches"], 1)
    bytes_launch = st["bytes_total"] / max(st["launches"], 1)
    achieved = bytes_launch / per_launch_s / 1e9 if per_launch_s > 0 else 0.0
    traffic = None
    if args.traffic and os.path.exists(args.traffic):
        tr = json.load(open(args.traffic))
        traffic = tr.get(dom)

    cpu = None
    if not args.no_cpu_baseline and lp.dense is None:
        import oracle
        tc = time.perf_counter()
        o = oracle.ipm(lp)
        tcpu = time.perf_counter() - tc
        cpu = {"value": 1.0 / tcpu, "unit": "LPs/s", "cores": 1, "kind": "oracle",
               "sample": f"1 full solve of {args.workload} ({o['iters']} IPM iterations, {tcpu:.2f} s)",
               "objective_rel_err_gpu_vs_oracle": abs(res[-1]["pobj"] - o["pobj"]) / abs(o["pobj"])}

    lat_ms = np.array(lat) * 1e3
    line = {
        "metric": "LPs solved/s at rel. gap 1e-8 (p50/p99 latency; Krylov+NE-SOR kernel HBM GB/s)",
        "value": args.steps / total,
        "unit": "LPs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total / args.steps * 1e3,
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 sweeps + f64",
        "data": "synthetic",
        "all_converged": ok,
        "ipm_iters": res[-1]["iters"],
        "krylov_iters": res[-1]["krylov_iters"],
        "gamma_rel": res[-1]["gamma_rel"],
        "config": {"workload": args.workload, "m": lp.m, "n": lp.n, "nnz": lp.nnz,
                   "precision": args.precision, "inner": args.inner, "krylov": "AB-GMRES",
                   "inner_sweeps": 2, "omega": 1.0, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "launches": st["launches"], "us_per_launch": per_launch_s * 1e6,
                     "bytes_per_launch": bytes_launch},
        "kernel_classes": {k: {"launches": v["launches"], "ms_total": v["ms_total"],
                               "us_per_launch": v["ms_total"] * 1e3 / max(v["launches"], 1),
                               "GBps": (v["bytes_total"] / (v["ms_total"] / 1e3) / 1e9) if v["ms_total"] > 0 else 0,
                               "TFLOPs": (v["flops_total"] / (v["ms_total"] / 1e3) / 1e12) if v["ms_total"] > 0 else 0}
                           for k, v in stats.items() if v["launches"] > 0},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    p.close()


if __name__ == "__main__":
    main()

"""Reduce rocprofv3 CSV output to the short summaries kept under profiles/.

    python -m paper_1604_07491_amd.profsum trace <rocprof output dir> <out.json>
    python -m paper_1604_07491_amd.profsum pmc   <rocprof output dir> <out.json>
    python -m paper_1604_07491_amd.profsum window <rocprof output dir> <out.json> <kernel> <grid y> <count>
    python -m paper_1604_07491_amd.profsum pmcwindow <rocprof output dir> <out.json> <kernel> <grid threads> <count>

trace: per (kernel, grid) launch counts and mean durations from the kernel trace, and for
each batch width the mean duration of the NE-SOR sweep launches of the timing replay (the
sweep launches after the last back-substitution of that width: bench.py replays the
dominant kernel last).  pmc: per (kernel, grid) mean counter value, and the mean over the
last 800 batched sweep dispatches (the replay window of bench.py's kernel table).  window:
the mean duration of the last <count> launches of the kernel whose name contains <kernel>
with grid y = <grid y> (bench.py replays its dominant kernel for the serving mix's batch
last of all its launches of that grid), with the per-kernel table of the whole trace.
pmcwindow: the mean counter value over the last <count> dispatches of the kernel whose name
contains <kernel> with <grid threads> threads in all (a counter run of that replay).
"""
import collections
import csv
import glob
import json
import os
import sys


def _one(d, pattern):
    fs = glob.glob(os.path.join(d, "**", pattern), recursive=True)
    if not fs:
        raise SystemExit(f"no {pattern} under {d}")
    return fs[0]


def trace_summary(d):
    rows = list(csv.DictReader(open(_one(d, "*kernel_trace.csv"))))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    agg = collections.defaultdict(lambda: [0, 0.0])
    for r in rows:
        key = (r["Kernel_Name"].split("(")[0][:48], int(r["Grid_Size_X"]), int(r["Grid_Size_Y"]))
        agg[key][0] += 1
        agg[key][1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
    res = {"kernels": [[k[0], k[1], k[2], n, us / 1e3, us / n]
                       for k, (n, us) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:40]]}
    res["replay"] = {}
    for y in sorted({int(r["Grid_Size_Y"]) for r in rows if "k_nesor" in r["Kernel_Name"]}):
        bs = [i for i, r in enumerate(rows) if "k_backsolve" in r["Kernel_Name"] and int(r["Grid_Size_Y"]) == y]
        if not bs:
            continue
        rep = [r for r in rows[bs[-1]:] if "k_nesor" in r["Kernel_Name"] and int(r["Grid_Size_Y"]) == y]
        us = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rep]
        if us:
            res["replay"][y] = {"n": len(us), "avg_us": sum(us) / len(us)}
    sf = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    if sf:
        res["stats_head"] = open(sf[0]).read().splitlines()[:25]
    return res


def pmc_summary(d):
    rows = list(csv.DictReader(open(_one(d, "*counter_collection.csv"))))
    agg = collections.defaultdict(lambda: [0, 0.0])
    seq = []
    for r in rows:
        key = (r["Kernel_Name"].split("(")[0][:48], r["Grid_Size"], r["Counter_Name"])
        v = float(r["Counter_Value"])
        agg[key][0] += 1
        agg[key][1] += v
        seq.append((int(r["Dispatch_Id"]), key, v))
    res = {"n": len(rows), "by_kernel": [[k[0], k[1], k[2], n, s / n]
                                         for k, (n, s) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:20]]}
    seq.sort()
    # the batched sweep launches (grids above 100k threads), last 800: the final replay of
    # the sweep group in bench.py (every colour kind of the group in its proportion)
    tail = [v for _, k, v in seq if "k_nesor" in k[0] and int(k[1]) > 100000][-800:]
    if tail:
        res.update(nesor_batch_tail_n=len(tail), nesor_batch_tail_avg=sum(tail) / len(tail))
    return res


def window_summary(d, kernel, grid_y, count):
    rows = list(csv.DictReader(open(_one(d, "*kernel_trace.csv"))))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    sel = [r for r in rows if kernel in r["Kernel_Name"] and int(r["Grid_Size_Y"]) == grid_y][-count:]
    us = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in sel]
    res = {"kernel": kernel, "grid_y": grid_y, "n": len(us), "avg_us": sum(us) / max(1, len(us)),
           "min_us": min(us) if us else None, "max_us": max(us) if us else None}
    agg = collections.defaultdict(lambda: [0, 0.0])
    for r in rows:
        key = r["Kernel_Name"].split("(")[0][:48]
        agg[key][0] += 1
        agg[key][1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
    total = sum(v[1] for v in agg.values())
    res["kernels"] = [[k, n, us / 1e3, us / n, us / total]
                      for k, (n, us) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:15]]
    return res


def pmc_window(d, kernel, grid_threads, count):
    rows = list(csv.DictReader(open(_one(d, "*counter_collection.csv"))))
    sel = [r for r in rows if kernel in r["Kernel_Name"] and int(r["Grid_Size"]) == grid_threads]
    sel.sort(key=lambda r: int(r["Dispatch_Id"]))
    out = {}
    for name in sorted({r["Counter_Name"] for r in sel}):
        v = [float(r["Counter_Value"]) for r in sel if r["Counter_Name"] == name][-count:]
        out[name] = {"n": len(v), "mean": sum(v) / max(1, len(v)), "min": min(v) if v else None,
                     "max": max(v) if v else None}
    return {"kernel": kernel, "grid_threads": grid_threads, "counters": out}


if __name__ == "__main__":
    kind, d, out = sys.argv[1:4]
    if kind == "pmcwindow":
        res = pmc_window(d, sys.argv[4], int(sys.argv[5]), int(sys.argv[6]))
    elif kind == "window":
        res = window_summary(d, sys.argv[4], int(sys.argv[5]), int(sys.argv[6]))
    else:
        res = trace_summary(d) if kind == "trace" else pmc_summary(d)
    json.dump(res, open(out, "w"), indent=1)

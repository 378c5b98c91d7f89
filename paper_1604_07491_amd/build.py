"""Build the HIP library ``liblpk.so`` in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblpk.so")
SOURCES = ["kernels.hip", "sweep.hip", "sweep_lds.hip", "engine.hip", "capi.hip", "profile.hip", "dense.hip", "server.hip", "noalloc.hip", "colour.cpp", "bounds.cpp", "presolve.cpp"]
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         # no packed FP32 instructions are generated
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result"]


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        lang = [] if src.endswith(".hip") else ["-x", "c++"]
        cmd = ["hipcc", *FLAGS, *lang, "-c", os.path.join(SRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-c", os.path.join(SRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = False
    for src, pr in procs:
        out = pr.communicate()[0].decode()
        lines = [l for l in out.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if pr.returncode != 0 or (verbose and lines):
            sys.stderr.write(f"--- {src}\n" + "\n".join(lines) + "\n")
        failed |= pr.returncode != 0
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

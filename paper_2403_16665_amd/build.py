"""Build the HIP library libdensedft.so for gfx950 (in-tree).

Every .hip source and dd_api.cpp is compiled by hipcc to an object file in
parallel, then linked into ``paper_2403_16665_amd/libdensedft.so``.  All
device code is built with packed FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdensedft.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def sources():
    return [f for f in sorted(os.listdir(CSRC)) if f.endswith((".hip", ".cpp"))]


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    procs, objs = [], []
    pending = list(sources())
    failed = []
    while pending or procs:
        while pending and len(procs) < jobs:
            src = pending.pop(0)
            obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
            objs.append(obj)
            lang = ["-x", "hip"] if src.endswith(".cpp") else []
            cmd = [HIPCC] + FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                stderr=subprocess.STDOUT, text=True)))
        src, pr = procs.pop(0)
        out, _ = pr.communicate()
        msgs = [l for l in out.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if pr.returncode != 0:
            failed.append(src)
            print("\n".join(msgs), file=sys.stderr)
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    tmp = LIB + ".tmp"
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs,
                   check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

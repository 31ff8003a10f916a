"""Build the HIP library (libnullspace.so) for gfx950 with hipcc, in-tree.

Usage: python -m paper_2407_04634_amd.build [-v]
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libnullspace.so")
SOURCES = ["capi.hip", "kernels_sparse.hip", "kernels_dense.hip", "eig.hip", "solver.hip", "noalloc.hip",
           "precond_ic.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-variable",
    "-Wno-unused-but-set-variable",
    # packed FP32 instructions stay disabled in every GPU build
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast",
    "-munsafe-fp-atomics",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Compile every source for gfx950 and link libnullspace.so (always rebuilds)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objdir = tempfile.mkdtemp(prefix="nsp_build_")
    objs = []
    procs = []
    try:
        for s in srcs:
            o = os.path.join(objdir, os.path.basename(s) + ".o")
            cmd = [hipcc(), *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", s, "-o", o]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            objs.append(o)
            while len([p for _, p in procs if p.poll() is None]) >= jobs:
                procs[0][1].wait() if procs[0][1].poll() is None else None
                for _, p in procs:
                    if p.poll() is None:
                        p.wait()
                        break
        for s, p in procs:
            out, _ = p.communicate()
            text = out.decode(errors="replace")
            if p.returncode != 0:
                raise RuntimeError(f"hipcc failed on {os.path.basename(s)}:\n{text}")
            if verbose and text.strip():
                print(text)
        tmp = LIB + ".tmp"
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp,
               "-L/opt/rocm/lib", "-lrocblas", "-lrocsolver"]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(objdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

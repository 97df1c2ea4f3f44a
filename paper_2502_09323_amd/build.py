"""Compile the HIP sources of libpb for gfx950 into ``paper_2502_09323_amd/libpb.so``."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = ["pb_api.hip", "pb_build.hip", "pb_solve.hip", "pb_energy.hip", "pb_server.hip", "pb_refine.hip", "pb_mg.hip",
       "pb_noalloc.hip"]
LIB = os.path.join(HERE, "libpb.so")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def build(verbose: bool = False, extra=None) -> str:
    """Always recompiles; returns the path of the shared library."""
    out = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    cmd += list(extra or [])
    cmd += [os.path.join(HERE, "csrc", s) for s in SRC] + ["-o", out]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])

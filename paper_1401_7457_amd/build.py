"""Compile the HIP library libcxbwt.so in-tree for gfx950 with hipcc, and
libcxbwt_ceilings.so (the measurement kernel of bench.py --mode ceilings)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", "cxbwt.hip")]
OUT = os.path.join(HERE, "libcxbwt.so")
CEILINGS_SOURCES = [os.path.join(HERE, "csrc", "ceilings.hip")]
CEILINGS_OUT = os.path.join(HERE, "libcxbwt_ceilings.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # keep hipcc from forming packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _hipcc(sources, out, verbose: bool) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), *sources, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    errs = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{errs}")
    if verbose and errs.strip():
        print(errs, file=sys.stderr)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    _hipcc(CEILINGS_SOURCES, CEILINGS_OUT, verbose)
    return _hipcc(SOURCES, OUT, verbose)


if __name__ == "__main__":
    print(build(verbose=True))

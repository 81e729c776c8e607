"""Build the HIP libraries for gfx950 with hipcc (in-tree, next to this file):
liblrdmc.so (the projection library behind include/lrdmc.h) and
libmfma_probe.so (the measurement prototype of the table's contraction)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "lrdmc.hip")
OUT = os.path.join(HERE, "liblrdmc.so")
PROBE_SRC = os.path.join(HERE, "csrc", "mfma_probe.hip")
PROBE_OUT = os.path.join(HERE, "libmfma_probe.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17",
    # packed FP32 instructions stay off in every HIP object of this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no loop-invariant hoisting of machine instructions: hoisted 64-bit
    # constants of exp/log stay live across the whole move loop and spill
    "-mllvm", "-disable-machine-licm",
    "-Wall", "-Wno-unused-function",
]


def _build_one(src: str, out: str, verbose: bool) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           src, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed to build {os.path.basename(out)}")
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    _build_one(PROBE_SRC, PROBE_OUT, verbose)
    return _build_one(SRC, OUT, verbose)


if __name__ == "__main__":
    print(build(verbose=True))

"""Build libkbnb.so (HIP for gfx950) in-tree with hipcc.

Every HIP source is compiled with packed-FP32 instructions disabled
(``-Xclang -target-feature -Xclang -packed-fp32-ops``); the host pass warns
that it does not know the feature, which is harmless.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkbnb.so")
SOURCES = ["kbnb_kernels.hip", "kbnb_engine.hip", "kbnb_bnb.cpp", "kbnb_tune.cpp",
           "kbnb_pool.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False) -> str:
    """Compile every source and link libkbnb.so (always recompiles)."""
    out = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(HERE, "..", "include"), "-o", out,
           *[os.path.join(CSRC, s) for s in SOURCES], "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libkbnb.so")
    os.replace(out, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

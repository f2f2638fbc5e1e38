"""Compile libtril.so (HIP, gfx950) in-tree with hipcc.

Flags:
  --offload-arch=gfx950        MI355X only
  -O3 -std=c++17 -fPIC -shared
  -ffp-contract=off            no fused multiply-adds: FP64 narrow-phase arithmetic
                               keeps its written evaluation order
  -Xclang -target-feature -Xclang -packed-fp32-ops
                               no packed FP32 instructions
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libtril.so")

SOURCES = ["abi.hip", "radix_sort.hip", "lbvh.hip", "traverse.hip", "narrow.hip", "stats.hip",
           "st.hip", "mlp.hip", "annihilate.hip", "kinematics.hip",
           "grid.hip", "noalloc.hip", "audit.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libtril.so")
    warn = [l for l in (r.stdout + r.stderr).splitlines()
            if "warning" in l and "packed-fp32-ops" not in l and "not a recognized feature" not in l]
    if verbose and warn:
        print("\n".join(warn))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Build libpfk.so (the HIP library behind include/pfk.h) for gfx950.

Run ``python -m paper_1511_07226_amd.build`` or call ``build()``.  The
library is written next to this file so it travels with the source tree.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpfk.so")
SOURCES = [os.path.join(HERE, "csrc", "pfk_api.hip")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds are fused only inside a source expression (a*b + c), never
    # across statements after inlining: every kernel that shares a device body
    # (single, batched, persistent) then rounds identically
    "-ffp-contract=on",
    "-I" + os.path.join(ROOT, "include"),
    "-Wall",
    "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libpfk.so; returns the library path."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libpfk.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

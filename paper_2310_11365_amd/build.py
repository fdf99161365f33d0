"""Build of the HIP library libmcpr.so (gfx950) from csrc/.

The library is the product: every step of the hot path runs in its kernels.
It is built in-tree (next to this file) so that it travels with the source
tree; nothing is installed.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmcpr.so")
SOURCES = ["kernels.hip", "cdf.hip", "api.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # every fused multiply-add in the kernels is written out explicitly
    "-ffp-contract=off",
    # no packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-mcode-object-version=5",
    "-Wall",
]


def build_command(out: str = LIB):
    return [HIPCC, *FLAGS, "-I", CSRC, "-I", INCLUDE, *[os.path.join(CSRC, s) for s in SOURCES], "-o", out]


def build(out: str = LIB, verbose: bool = False) -> str:
    """Compile libmcpr.so for gfx950 (cross-compiles without a GPU)."""
    tmp = out + ".tmp"
    cmd = build_command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))

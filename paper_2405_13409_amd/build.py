"""Build libspoly.so (gfx950) in-tree with hipcc.

Two sources are generated on every build: the elimination phase of the
one-vertex kernels (csrc/gen_laplace.py -> csrc/laplace_gen.inc) and the
square-root approximation table (sqrtfit.py -> csrc/sqrt_table.inc).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libspoly.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _write_if_changed(path: str, data: bytes) -> None:
    old = open(path, "rb").read() if os.path.exists(path) else b""
    if old != data:
        with open(path, "wb") as f:
            f.write(data)


def generate() -> None:
    out = subprocess.check_output([sys.executable, os.path.join(CSRC, "gen_laplace.py")])
    _write_if_changed(os.path.join(CSRC, "laplace_gen.inc"), out)
    out = subprocess.check_output([sys.executable, os.path.join(HERE, "sqrtfit.py")])
    _write_if_changed(os.path.join(CSRC, "sqrt_table.inc"), out)


def sources():
    """The unity translation unit; it includes every module under csrc/."""
    return [os.path.join(CSRC, "libspoly.hip")]


def build(verbose: bool = False) -> str:
    generate()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *HIP_FLAGS, "-o", tmp, *sources()]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

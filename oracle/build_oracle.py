"""Compile the C++ oracle (oracle/wfq_oracle.cpp) into oracle/libwfq_oracle.so with g++ and OpenMP.

Test infrastructure: building the checker is not using it. Every call recompiles.
Usage: python -m oracle.build_oracle
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wfq_oracle.cpp")
LIB = os.path.join(HERE, "libwfq_oracle.so")


def build(verbose: bool = False) -> str:
    gxx = shutil.which("g++") or shutil.which("c++")
    if gxx is None:
        raise RuntimeError("no C++ compiler (g++) for the oracle")
    tmp = LIB + ".tmp"
    # plain IEEE FP64: no fast-math, no contraction of a*b+c into fused operations
    cmd = [gxx, "-std=c++17", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-Wall", SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling the C++ oracle failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(verbose=True)

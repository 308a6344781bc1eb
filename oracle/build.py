"""Compile the CPU oracle library (test infrastructure; see oracle/__init__.py)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "jz_oracle.c")
LIB = os.path.join(HERE, "libjz_oracle.so")

# -ffp-contract=off: every product and sum rounds separately (no FMA), which is
# the fixed arithmetic both sides of the parity check use. No -ffast-math, so
# subnormals are kept and no reassociation happens.
CFLAGS = ["-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared", "-fvisibility=hidden", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

"""Build the gfx950 HIP library ``libjz.so`` in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libjz.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["api.hip", "build.hip", "knn.hip", "fof.hip", "serve.hip", "tune.hip", "noalloc.hip", "catalogue.hip"]

# -ffp-contract=off: no FMA contraction, so distances use the fixed float32
# expression. Packed FP32 instructions are disabled. Subnormals are kept
# (the HIP default for f32 on gfx950).
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
            "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


# knn.hip orders top-k keys as doubles with v_min_f64 / v_max_f64, and both
# leaf stages reduce boxes with min / max; no value in these files is ever
# NaN (coordinates are finite, fillers sit at +-inf and never meet inf - inf),
# so NaN handling (and the IEEE-mode canonicalizations it needs around every
# min / max) is switched off for them. Rounding and subnormal handling are
# unaffected.
EXTRA = {"knn.hip": ["-fno-honor-nans", "-mno-amdgpu-ieee"],
         "fof.hip": ["-fno-honor-nans", "-mno-amdgpu-ieee"]}


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *HIPFLAGS, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, out))
    if out.strip() and verbose:
        print(out, flush=True)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)

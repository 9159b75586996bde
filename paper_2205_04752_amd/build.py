"""Build libhmat.so (HIP kernels + host planner + C ABI) for gfx950 in-tree.

Every source is compiled by hipcc; objects go to ``_build/`` next to this file
and the shared library to ``libhmat.so`` in the package directory.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhmat.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
# Keep the compiler from forming packed FP32 instructions.
NO_PK = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

SOURCES = [
    # (file, extra flags)
    ("kernels.hip", ["-x", "hip", f"--offload-arch={ARCH}", *NO_PK, "-munsafe-fp-atomics"]),
    ("product.hip", ["-x", "hip", f"--offload-arch={ARCH}", *NO_PK]),
    ("amvm.hip", ["-x", "hip", f"--offload-arch={ARCH}", *NO_PK]),
    # the planner's geometry and admissibility tests must not be contracted
    ("planner.cpp", ["-ffp-contract=off"]),
    ("api.cpp", []),
    ("server.cpp", []),
]


def _compile(src: str, extra: list[str]) -> str:
    obj = os.path.join(OUT, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda se: _compile(*se), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

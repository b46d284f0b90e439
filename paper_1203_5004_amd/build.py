"""Build the HIP library (gfx950) in-tree: paper_1203_5004_amd/_lib/libwagener_hull.so.

hipcc cross-compiles for gfx950 without a GPU, so this runs anywhere the
ROCm toolchain is installed.  Usage: ``python -m paper_1203_5004_amd.build``.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "wagener_hull.hip")
SOURCES = [SRC, os.path.join(HERE, "csrc", "read_reference.hip"),
           os.path.join(HERE, "csrc", "radix_sort.hip")]
DEPS = [*SOURCES, os.path.join(HERE, "csrc", "uh_device.hpp"),
        os.path.join(HERE, "csrc", "radix_sort.hpp"),
        os.path.join(ROOT, "include", "wagener_hull.h")]
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libwagener_hull.so")
ARCH = os.environ.get("UH_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",                       # the predicate's error bound
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(HERE, "csrc"), *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

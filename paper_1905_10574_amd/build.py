"""Build libtrsyl.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1905_10574_amd.build   (or call build())
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtrsyl.so")
ARCH = os.environ.get("TRSYL_ARCH", "gfx950")

HIP_SOURCES = ["solver.hip", "extras.hip", "noalloc.hip"]
HOST_SOURCES = ["capi.cpp", "capi_extras.cpp"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function"]
# packed FP32 VALU forms are disabled for all device code
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          ]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = True, defines: tuple = ()) -> str:
    """Compile every source and link libtrsyl.so.  `defines` adds -D options (e.g. the optional
    TRSYL_PHASE_STAMPS timing hooks)."""
    extra = [f"-D{d}" for d in defines]
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = []
    for src in HIP_SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(bdir, src + ".o")
        _run(["hipcc", "-c", path, "-o", obj] + COMMON + DEVICE + extra)
        objs.append(obj)
    for src in HOST_SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(bdir, src + ".o")
        _run(["hipcc", "-c", path, "-o", obj] + COMMON)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run(["hipcc", "-shared", "-o", tmp] + objs + [f"--offload-arch={ARCH}"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(defines=tuple(a[2:] for a in sys.argv[1:] if a.startswith("-D")))
    sys.exit(0)

"""Build librcpsp.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "librcpsp.so")
OBJ = os.path.join(ROOT, "_build")
SOURCES = [os.path.join(CSRC, f) for f in ("rcpsp_host.cpp", "rcpsp_serve.cpp", "rcpsp_kernels.hip",
                                           "rcpsp_k_search.hip", "rcpsp_k_count.hip", "rcpsp_k_batch.hip",
                                           "rcpsp_k_serve.hip", "rcpsp_noalloc.hip")]
HEADERS = [os.path.join(ROOT, "include", "rcpsp.h"), os.path.join(CSRC, "rcpsp_internal.h"),
           os.path.join(CSRC, "rcpsp_launch.h"), os.path.join(CSRC, "rcpsp_runtime.h"),
           os.path.join(CSRC, "rcpsp_device.h")]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-pthread",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def build(verbose: bool = False) -> str:
    """Compile every HIP source for gfx950 (one object per source, side by
    side) and link paper_1711_04556_amd/librcpsp.so."""
    os.makedirs(OBJ, exist_ok=True)
    objs = [os.path.join(OBJ, os.path.basename(s) + ".o") for s in SOURCES]

    def compile_one(k):
        cmd = [hipcc()] + FLAGS + ["-c", SOURCES[k], "-o", objs[k]]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    with ThreadPoolExecutor(min(len(SOURCES), 8)) as ex:
        list(ex.map(compile_one, range(len(SOURCES))))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Build libpffrg.so (HIP for gfx950) in the package directory.

Each source is compiled to an object in parallel (hipcc -c), then the objects
are linked into the shared library.
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(HERE, "csrc", f)
        for f in ("pffrg.hip", "pffrg_batch.hip", "pffrg_peaks.hip", "pffrg_noalloc.hip")]
LIB = os.path.join(HERE, "libpffrg.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    tag = f".tmp{os.getpid()}"
    objs = [os.path.join(HERE, "csrc", os.path.basename(s) + tag + ".o") for s in SRCS]
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]

    def compile_one(i):
        cmd = [HIPCC, *FLAGS, *inc, "-c", "-o", objs[i], SRCS[i]]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)

    try:
        with ThreadPoolExecutor(max_workers=min(len(SRCS), os.cpu_count() or 1)) as ex:
            list(ex.map(compile_one, range(len(SRCS))))
        tmp = LIB + tag
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)

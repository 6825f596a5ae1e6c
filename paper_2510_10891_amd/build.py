"""Build the gfx950 solver library (libhprlp.so) in-tree with hipcc.

Usage: python -m paper_2510_10891_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhprlp.so")
# the matrix-product instantiations first: they take the longest to compile
SOURCES = ["kernels_check_cols64.hip", "kernels_check_cols32.hip", "kernels_check_colsmixed.hip",
           "kernels_primal32.hip", "kernels_primal64.hip", "kernels_dual32.hip", "kernels_dual64.hip",
           "kernels_spmv.hip", "kernels_check_rows.hip", "kernels.hip", "setup.hip", "solver.hip", "mlp.hip",
           "probe.hip"]
HEADERS = ["internal.h", "csr.h"]

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source (in parallel, one hipcc per translation unit) and link the shared
    library; always rebuilds."""
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    cmds = []
    for src in SOURCES:
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        cmds.append((obj, [hipcc(), *FLAGS, "-I", os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, src),
                           "-o", obj]))
    if verbose:
        for _, cmd in cmds:
            print(" ".join(cmd), flush=True)
    jobs = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(subprocess.check_call, cmd) for _, cmd in cmds]:
            f.result()
    objs = [obj for obj, _ in cmds]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Build the HIP sweep library (libvefsweep.so) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libvefsweep.so")
SOURCES = ["plan.cpp", "kernels.hip", "sweep_p1.hip", "sweep_p2.hip", "sweep_p3.hip", "sweep_p4.hip", "probe.hip", "emat.hip",
           "hrt.hip", "lambda.hip", "api.cpp"]
ARCH = os.environ.get("VEF_OFFLOAD_ARCH", "gfx950")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

# -packed-fp32-ops: keep the compiler from emitting packed FP32 VALU forms.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Per-source flags: the HRT elimination is a fully unrolled loop over the
# 56 rows of the p = 3 block matrix, above the default limit on the size of a
# pragma-requested unroll (a rolled loop indexes the row array at run time,
# which puts it in scratch memory).
SOURCE_FLAGS = {"hrt.hip": ["-mllvm", "-pragma-unroll-threshold=1000000"]}


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    return "hipcc"


def _compile(src, verbose):
    obj = os.path.join(HERE, "_build", os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-c",
           "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-command-line-argument"]
    cmd += DEVICE_FLAGS + SOURCE_FLAGS.get(src, [])
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    cmd += [os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return obj


def build(verbose: bool = False, out: str = LIB, jobs: int = 0) -> str:
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, min(os.cpu_count() or 1, 8)))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = out + ".tmp"
    # rocSOLVER (sparse re-factorisation of the reduced VEF system) and the
    # rocBLAS handle it runs on
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + [
        "-L" + os.path.join(ROCM, "lib"), "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lrocsolver", "-lrocblas"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)

"""Compile the HIP library ``libchs.so`` for gfx950 with hipcc.

Flags that matter for the results: no FMA contraction (the squared distance
is the unfused FP32 sum), no fast-math, FP32 denormals kept, and packed FP32
instructions disabled (their results have been unreliable on some parts).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["prims.hip", "build.hip", "search.hip", "radius.hip", "knn.hip", "agg.hip", "noalloc.hip"]
LIB = os.path.join(HERE, "libchs.so")
ARCH = os.environ.get("CHS_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-ffp-contract=off",
    "-fno-fast-math",
    "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-result",
    f"-I{os.path.join(ROOT, 'include')}",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose=False, extra=()):
    """Always recompiles (one hipcc process per source, in parallel, then one
    link); writes libchs.so next to this file."""
    tmp = LIB + ".tmp"
    objs, procs = [], []
    for src in sources():
        obj = os.path.join(CSRC, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [HIPCC, *[f for f in FLAGS if f != "-shared"], *extra, "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
    failed = [cmd for cmd, pr in procs if pr.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    link = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    for obj in objs:
        os.remove(obj)
    os.replace(tmp, LIB)
    return LIB


def asm(source, out):
    """AMD assembly of one source (device side), for inspecting codegen."""
    cmd = [HIPCC, *[f for f in FLAGS if f not in ("-shared",)], "--cuda-device-only", "-S",
           "-o", out, os.path.join(CSRC, source)]
    subprocess.check_call(cmd)
    return out


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)

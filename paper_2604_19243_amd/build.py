"""Build libkifmm_mi355x.so in-tree with hipcc for gfx950.

Every source is compiled on each call (the build is a few seconds per file and
the library is small).  HIP sources get the gfx950 offload target and packed
FP32 instructions disabled; host sources are compiled as plain C++ with FP
contraction off, so the double-precision leaf assignment is reproducible.
"""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libkifmm_mi355x.so")
BUILD = os.path.join(ROOT, "_build")

HIP_SOURCES = ["gemm.hip", "m2l.hip", "leaf.hip", "plan.hip"]
CPP_SOURCES = ["capi.cpp", "tree.cpp", "ops.cpp", "linalg.cpp"]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(args):
    cmd, src = args
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return src


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    common = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", os.path.join(ROOT, "include"), "-I", SRC]
    jobs = []
    objs = []
    for s in HIP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        objs.append(o)
        jobs.append(([cc, "-x", "hip", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                      "-packed-fp32-ops", "-munsafe-fp-atomics", *common, "-c", os.path.join(SRC, s), "-o", o], s))
    for s in CPP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        objs.append(o)
        jobs.append(([cc, "-x", "c++", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", *common, "-c",
                      os.path.join(SRC, s), "-o", o], s))
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", "8"))))
    with ThreadPoolExecutor(workers) as ex:
        for s in ex.map(_compile, jobs):
            if verbose:
                print("compiled", s, flush=True)
    tmp = OUT + ".tmp"
    link = [cc, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{' '.join(link)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Build libesp.so (HIP for gfx950) in-tree.

Every HIP source is compiled with hipcc for gfx950 only; packed FP32
instructions are disabled in device code (-target-feature -packed-fp32-ops)
and hardware float atomics are enabled (-munsafe-fp-atomics; all buffers are
coarse-grained device memory). The host-only parameter code is compiled with
g++.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT_DIR = os.path.join(HERE, "_obj")
LIB = os.path.join(HERE, "libesp.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-I", INCLUDE, "-I", CSRC]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    jobs = [
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "kernels.hip"), "-o", os.path.join(OUT_DIR, "kernels.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "fft.hip"), "-o", os.path.join(OUT_DIR, "fft.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "local.hip"), "-o", os.path.join(OUT_DIR, "local.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "runtime.cpp"), "-o", os.path.join(OUT_DIR, "runtime.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "assembly.cpp"), "-o", os.path.join(OUT_DIR, "assembly.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "server.cpp"), "-o", os.path.join(OUT_DIR, "server.o")],
        ["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, "plan.cpp"), "-o", os.path.join(OUT_DIR, "plan.o")],
    ]
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout + r.stderr, file=sys.stderr)
    objs = [j[-1] for j in jobs]
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

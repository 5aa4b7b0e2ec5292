"""Build libjf.so in-tree: host C++ with g++, HIP sources with hipcc for gfx950.

    python -m paper_2103_11595_amd.build        (or build() from Python)

Every HIP translation unit is compiled with packed FP32 instructions disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libjf.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HOST_SOURCES = ["api.cpp", "circuit.cpp", "network.cpp", "planner.cpp", "emulate.cpp"]
HIP_SOURCES = ["kernels.hip", "executor.hip"]
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return cmd[-1]


def build(verbose: bool = False, host_cxx: str | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    cxx = host_cxx or shutil.which("g++") or "g++"
    jobs = []
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        jobs.append([cxx, "-O2", "-g", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
                     "-I" + os.path.join(ROCM, "include"), "-D__HIP_PLATFORM_AMD__",
                     "-c", os.path.join(CSRC, src), "-o", obj])
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        jobs.append([hipcc] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for out in ex.map(_run, jobs):
            if verbose:
                print("built", out)
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950"] + objs + ["-o", tmp])
    os.replace(tmp, LIB)
    if verbose:
        print("linked", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

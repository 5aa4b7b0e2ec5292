"""Build libjf.so in-tree: host C++ with g++, HIP sources with hipcc for gfx950.

    python -m paper_2103_11595_amd.build             (or build() from Python)
    python -m paper_2103_11595_amd.build --sanitize  (a separate _build/libjf_asan.so)

Every HIP translation unit is compiled with packed FP32 instructions disabled.  The sanitizer build
instruments the host sources compiled by g++ (the planner, network builder, ingest, emulation and
the C ABI: the 64-bit offset arithmetic over caller-sized tables) with AddressSanitizer and
UndefinedBehaviorSanitizer; the HIP sources are built as usual.  Run the host test suite against
it (no GPU needed; libstdc++ is preloaded after the sanitizer runtime so that its exception
interceptors resolve in a Python process):

    LD_PRELOAD="$(g++ -print-file-name=libasan.so) $(g++ -print-file-name=libstdc++.so)" \
    ASAN_OPTIONS=detect_leaks=0 UBSAN_OPTIONS=halt_on_error=1:print_stacktrace=1 \
    JF_LIB=paper_2103_11595_amd/_build/libjf_asan.so python -m pytest tests/test_host.py
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


SANITIZE = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]


def build(verbose: bool = False, host_cxx: str | None = None, sanitize: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    cxx = host_cxx or shutil.which("g++") or "g++"
    jobs = []
    objs = []
    tag = ".asan" if sanitize else ""
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + tag + ".o")
        objs.append(obj)
        jobs.append([cxx, "-O1" if sanitize else "-O2", "-g", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function"]
                    + (SANITIZE if sanitize else [])
                    + ["-I" + os.path.join(ROCM, "include"), "-D__HIP_PLATFORM_AMD__",
                       "-c", os.path.join(CSRC, src), "-o", obj])
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        jobs.append([hipcc] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for out in ex.map(_run, jobs):
            if verbose:
                print("built", out)
    lib = os.path.join(BUILD, "libjf_asan.so") if sanitize else LIB
    tmp = lib + ".tmp"
    extra = ["-lasan", "-lubsan"] if sanitize else []
    _run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950"] + objs + extra + ["-o", tmp])
    os.replace(tmp, lib)
    if verbose:
        print("linked", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv[1:])
    sys.exit(0)

"""Build libgigaqbx.so for gfx950 in-tree (host planner with g++, kernels with hipcc)."""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgigaqbx.so")
ARCH = os.environ.get("GQ_OFFLOAD_ARCH", "gfx950")

HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall"]
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]
# roctx stage ranges (rocprofiler-sdk's marker library, part of ROCm)
LINK_FLAGS = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout)
        raise RuntimeError("compile failed: " + " ".join(cmd[:3]))
    return r.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for f in ("planner.cpp", "translations.cpp"):
        jobs.append(["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, f),
                     "-o", os.path.join(BUILD, f + ".o")])
    hip_sources = ("kernels.hip", "kernels_p2x.hip", "kernels_pt.hip", "kernels_rot.hip",
                   "oversample.hip", "associate.hip", "executor.hip", "noalloc.hip")
    for f in hip_sources:
        jobs.append(["hipcc", *HIP_FLAGS, "-c", os.path.join(CSRC, f),
                     "-o", os.path.join(BUILD, f + ".o")])
    with ThreadPoolExecutor(max_workers=6) as ex:
        for out in ex.map(_run, jobs):
            if verbose and out:
                print(out)
    objs = [os.path.join(BUILD, f + ".o") for f in ("planner.cpp", "translations.cpp", *hip_sources)]
    tmp = LIB + ".tmp%d" % os.getpid()
    _run(["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs, *LINK_FLAGS])
    os.replace(tmp, LIB)
    return LIB


SAN_LIB = os.path.join(HERE, "libgigaqbx_san.so")
SAN_BUILD = os.path.join(HERE, "_build_san")


def build_sanitized(verbose: bool = False) -> str:
    """A host-sanitized copy of the library (AddressSanitizer and UndefinedBehaviorSanitizer
    on the host code only; device code is built as usual), for CPU runs of the host-side
    tests with host-only plans.  Load it in a process started with clang's ASan runtime
    preloaded and GQ_LIBRARY pointing at it."""
    os.makedirs(SAN_BUILD, exist_ok=True)
    san = ["-fno-omit-frame-pointer", "-g"]
    jobs = []
    for f in ("planner.cpp", "translations.cpp"):
        jobs.append(["/opt/rocm/llvm/bin/clang++", "-O1", "-std=c++17", "-fPIC",
                     "-ffp-contract=off", "-fsanitize=address,undefined", *san, "-c",
                     os.path.join(CSRC, f), "-o", os.path.join(SAN_BUILD, f + ".o")])
    hip_sources = ("kernels.hip", "kernels_p2x.hip", "kernels_pt.hip", "kernels_rot.hip",
                   "oversample.hip", "associate.hip", "executor.hip", "noalloc.hip")
    for f in hip_sources:
        jobs.append(["hipcc", *HIP_FLAGS, "-Xarch_host", "-fsanitize=address,undefined", *san,
                     "-c", os.path.join(CSRC, f), "-o", os.path.join(SAN_BUILD, f + ".o")])
    with ThreadPoolExecutor(max_workers=6) as ex:
        for out in ex.map(_run, jobs):
            if verbose and out:
                print(out)
    objs = [os.path.join(SAN_BUILD, f + ".o") for f in ("planner.cpp", "translations.cpp",
                                                         *hip_sources)]
    tmp = SAN_LIB + ".tmp%d" % os.getpid()
    _run(["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-shared-libsan",
          "-Xarch_host", "-fsanitize=address,undefined", "-o", tmp, *objs, *LINK_FLAGS])
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--sanitize":
        print(build_sanitized(verbose=True))
    else:
        print(build(verbose=True))

"""Build the gfx950 shared library (in-tree) with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_NAME = "libfdtdrom.so"
LIB_PATH = os.path.join(HERE, LIB_NAME)
# device code: compiled for gfx950 by hipcc
HIP_SOURCES = ["csrc/kernels.hip", "csrc/adjoint.hip"]
# host code (runtime, C ABI, model builder): plain C++ against the HIP host
# API, compiled by the host compiler
CPP_SOURCES = ["csrc/runtime.cpp", "csrc/adjoint_rt.cpp", "csrc/batch_rt.cpp", "csrc/romgen.cpp"]
SOURCES = HIP_SOURCES + CPP_SOURCES

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    "--offload-arch=gfx950",
    # keep the compiler from emitting packed FP32 VALU ops
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # IEEE-rounded FP32 division: the FP32 coefficient model depends on it
    "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-Wno-unused-command-line-argument",
]
CXX_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-D__HIP_PLATFORM_AMD__"]


def rocm_path() -> str:
    return os.environ.get("ROCM_PATH", "/opt/rocm")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), os.path.join(rocm_path(), "bin", "hipcc"), "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def cxx() -> str:
    cand = os.path.join(rocm_path(), "llvm", "bin", "clang++")
    return cand if os.path.exists(cand) else "clang++"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("build of " + LIB_NAME + " failed: " + " ".join(cmd[:2]) + " ...")


def build(verbose: bool = False) -> str:
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(rocm_path(), "include")]
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    cmds, objs = [], []
    for src in HIP_SOURCES:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmds.append([hipcc(), *HIPCC_FLAGS, *inc, "-c", os.path.join(HERE, src), "-o", obj])
        objs.append(obj)
    for src in CPP_SOURCES:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmds.append([cxx(), *CXX_FLAGS, *inc, "-c", os.path.join(HERE, src), "-o", obj])
        objs.append(obj)
    # one compiler process per source file, side by side
    from concurrent.futures import ThreadPoolExecutor
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = LIB_PATH + ".tmp"
    _run([hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))

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


# AddressSanitizer + UndefinedBehaviorSanitizer for the host sources only
# (compiled and linked by the host compiler; the device objects are the
# normal build's)
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined"]


def sanitizer_runtime() -> str:
    """Path of the AddressSanitizer runtime to preload into the interpreter."""
    return subprocess.run([cxx(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                          text=True, check=True).stdout.strip()


def build_sanitized(outdir: str, verbose: bool = False) -> str:
    """The library with the host code (runtime, C ABI, model builder) built
    with the sanitizers, into outdir; load it with FDTD_ROM_LIB pointing at
    it and the sanitizer runtime preloaded.  Uses the device objects of the
    normal build (built first if missing)."""
    objdir = os.path.join(HERE, "_build")
    dev = [os.path.join(objdir, os.path.basename(s) + ".o") for s in HIP_SOURCES]
    if not all(os.path.exists(o) for o in dev):
        build(verbose)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(rocm_path(), "include")]
    os.makedirs(outdir, exist_ok=True)
    cmds, objs = [], []
    for src in CPP_SOURCES:
        obj = os.path.join(outdir, os.path.basename(src) + ".san.o")
        cmds.append([cxx(), *SAN_FLAGS, "-std=c++17", "-fPIC", "-D__HIP_PLATFORM_AMD__", *inc, "-c",
                     os.path.join(HERE, src), "-o", obj])
        objs.append(obj)
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(len(cmds)) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    out = os.path.join(outdir, "libfdtdrom_san.so")
    lib_dir = os.path.join(rocm_path(), "lib")
    _run([cxx(), "-shared", *SAN_FLAGS, "-shared-libasan", *objs, *dev, "-L", lib_dir, "-lamdhip64",
          "-Wl,-rpath," + lib_dir, "-o", out], verbose)
    return out


if __name__ == "__main__":
    print(build(verbose=True))

"""Builds libdaqisland.so (the HIP library behind include/daq.h) in-tree.

hipcc for gfx950 only; packed-FP32 instruction selection is disabled for all
device code. The library is rebuilt on every call.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdaqisland.so")
SOURCES = [os.path.join(HERE, "csrc", "chop_kernels.hip"),
           os.path.join(HERE, "csrc", "daq_runtime.hip"),
           os.path.join(HERE, "csrc", "daq_server.hip"),
           os.path.join(HERE, "csrc", "compress_kernels.hip"),
           os.path.join(HERE, "csrc", "ceiling.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Wall", "-Wno-unused-result",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]


# profiler ranges of the serving loop (roctx, part of ROCm)
LIBS = ["-lrocprofiler-sdk-roctx"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + SOURCES + LIBS + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 feature: drop that note
    noise = "not a recognized feature for this target"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l and "ignoring feature" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + err)
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


C_CLIENT_SRC = os.path.join(ROOT, "tests", "native", "c_client.c")
C_CLIENT = os.path.join(ROOT, "tests", "native", "c_client")


def build_c_client(verbose: bool = False) -> str:
    """The plain C client of include/daq.h used by the tests (gcc, C11, HIP's C
    runtime API), linked against the library built above."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"),
           "-I", os.path.join(ROOT, "include"), C_CLIENT_SRC, "-L", HERE, "-ldaqisland",
           "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath,$ORIGIN/../../paper_1611_04959_amd",
           "-Wl,-rpath," + os.path.join(rocm, "lib"), "-o", C_CLIENT]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("gcc failed:\n" + r.stderr)
    return C_CLIENT


SAN_DIR = os.path.join(ROOT, "tests", "native", "sanitized")
SAN_LIB = os.path.join(SAN_DIR, "libdaqisland.so")
SAN_STRESS_SRC = os.path.join(ROOT, "tests", "native", "server_stress.cpp")
SAN_STRESS = os.path.join(SAN_DIR, "server_stress")
# host code only: each sanitizer flag applies to the host compilation (the
# device code of the library is built as usual)
HOST_SANITIZERS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                   "-Xarch_host", "-fno-omit-frame-pointer"]


def build_sanitized(verbose: bool = False) -> str:
    """The library with AddressSanitizer and UndefinedBehaviorSanitizer on its
    host code, and the serving-loop stress program linked against it (both
    under tests/native/sanitized, used by tests/test_gpu_server_sanitized.py)."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    os.makedirs(SAN_DIR, exist_ok=True)
    cmd = [HIPCC] + FLAGS + HOST_SANITIZERS + SOURCES + LIBS + ["-o", SAN_LIB]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc (sanitized) failed:\n" + r.stderr)
    clang = os.path.join(rocm, "llvm", "bin", "clang++")
    cmd = [clang, "-O1", "-g", "-std=c++17", "-Wall", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"), "-I", os.path.join(ROOT, "include"),
           SAN_STRESS_SRC, "-L", SAN_DIR, "-ldaqisland", "-L", os.path.join(rocm, "lib"), "-lamdhip64",
           "-lpthread", "-Wl,-rpath,$ORIGIN", "-Wl,-rpath," + os.path.join(rocm, "lib"), "-o", SAN_STRESS]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("clang++ (sanitized stress) failed:\n" + r.stderr)
    return SAN_STRESS


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_c_client(verbose=True))
    print(build_sanitized(verbose=True))

"""Build libkgf.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1109_1205_amd.build          # compile every source
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libkgf.so")
SOURCES = ["api.hip", "basis.hip", "hamiltonian.hip", "krylov.hip", "greens.hip", "adjoint.hip", "spectral.hip", "driven.hip", "necpt.hip"]
ARCH = os.environ.get("KGF_OFFLOAD_ARCH", "gfx950")

# Packed-FP32 instructions stay disabled in all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Wno-unused-command-line-argument", "-Wno-unknown-warning-option"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libkgf)")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *COMMON, *DEVICE_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer for the C ABI
# check (tests/abi_check.cpp); device code is compiled as usual.
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
SAN_LINK = ["-fsanitize=address,undefined"]
ABI_CHECK_SRC = os.path.join(ROOT, "tests", "abi_check.cpp")
ABI_CHECK_BIN = os.path.join(ROOT, "tests", "abi_check_asan")


def clangxx() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    for cand in (os.path.join(rocm, "llvm", "bin", "clang++"), shutil.which("clang++")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("clang++ not found (ROCm's LLVM is required for the sanitizer build)")


def _compile_san(src: str) -> str:
    d = os.path.join(BUILD, "san")
    obj = os.path.join(d, os.path.splitext(os.path.basename(src))[0] + ".o")
    cmd = [hipcc(), *COMMON, *DEVICE_FLAGS, "-O1", "-g", *SAN_HOST, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"sanitizer build failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build_abi_check(verbose: bool = True) -> str:
    """The C ABI check program linked against a host-sanitized copy of the
    library objects (tests/abi_check_asan)."""
    os.makedirs(os.path.join(BUILD, "san"), exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES] + [ABI_CHECK_SRC]
    with ThreadPoolExecutor(max_workers=min(len(srcs), 8)) as ex:
        objs = list(ex.map(_compile_san, srcs))
    rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    tmp = ABI_CHECK_BIN + ".tmp"
    cmd = [clangxx(), *SAN_LINK, "-o", tmp, *objs, "-L", rocm_lib, "-lamdhip64", "-lrocprofiler-sdk-roctx",
           f"-Wl,-rpath,{rocm_lib}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"sanitizer link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, ABI_CHECK_BIN)
    if verbose:
        print(f"built {ABI_CHECK_BIN}")
    return ABI_CHECK_BIN


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs,
           "-L", rocm_lib, "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{rocm_lib}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    try:
        build()
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)

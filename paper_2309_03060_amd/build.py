"""Compile libcola.so (HIP for gfx950) in-tree.

Every .hip source under csrc/ is compiled with hipcc for gfx950 into
_build/, then linked into paper_2309_03060_amd/libcola.so.  Packed-FP32
instruction selection is disabled for device code (the host pass of hipcc
warns that it does not know the feature; that warning is harmless).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(os.path.dirname(PKG), "_build")
LIB = os.path.join(PKG, "libcola.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src).replace(".hip", ".o"))
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link libcola.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    workers = min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, "-L/opt/rocm/lib",
           "-lrocprofiler-sdk-roctx"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


# Host-sanitizer build: the same sources with the host code (only) instrumented by
# AddressSanitizer and UndefinedBehaviorSanitizer, and the C driver tests/native/abi_sanitize.cpp
# that exercises every entry point through the C ABI.  The device code is compiled as usual.
ASAN_DIR = os.path.join(os.path.dirname(PKG), "tests", "native", "_asan")
CLANG = os.environ.get("COLA_CLANG", "/opt/rocm/llvm/bin/clang++")


def _compile_asan(src: str) -> str:
    obj = os.path.join(BUILD, "asan", os.path.basename(src).replace(".hip", ".o"))
    cmd = [HIPCC, *FLAGS, "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g", "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc (host sanitizer build) failed for {src}:\n{res.stdout}\n{res.stderr}")
    return obj


def build_host_sanitizer(verbose: bool = False) -> str:
    """libcola_asan.so and the driver abi_sanitize under tests/native/_asan; returns the driver."""
    os.makedirs(os.path.join(BUILD, "asan"), exist_ok=True)
    os.makedirs(ASAN_DIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    workers = min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile_asan, srcs))
    lib = os.path.join(ASAN_DIR, "libcola_asan.so")
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib, *objs, "-L/opt/rocm/lib",
           "-lrocprofiler-sdk-roctx"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link (host sanitizer build) failed:\n{res.stdout}\n{res.stderr}")
    drv = os.path.join(ASAN_DIR, "abi_sanitize")
    src = os.path.join(os.path.dirname(PKG), "tests", "native", "abi_sanitize.cpp")
    san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    cmd = [CLANG, "-std=c++17", "-O1", "-g", *san, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", src,
           "-L" + ASAN_DIR, "-lcola_asan", "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath," + ASAN_DIR,
           "-Wl,-rpath,$ORIGIN", "-Wl,-rpath,/opt/rocm/lib", "-o", drv]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"driver build failed:\n{res.stdout}\n{res.stderr}")
    if verbose:
        print("built", drv)
    return drv


if __name__ == "__main__":
    build(verbose=True)

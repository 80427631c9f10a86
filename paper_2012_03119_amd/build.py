"""Builds libgss.so (the HIP library) for gfx950 with hipcc, in-tree.

    python -m paper_2012_03119_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libgss.so")
BUILD_DIR = os.path.join(ROOT, "_build")
SOURCES = ["context.hip", "store.hip", "planes.hip", "test.hip", "batch.hip", "serve.hip", "simulate.hip", "mlp.hip", "priority.hip", "sort.hip", "rank.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
    # no packed FP32 instructions anywhere in the library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def _hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = os.path.join(rocm, "bin", "hipcc")
    return cand if os.path.exists(cand) else "hipcc"


def build(verbose: bool = False, extra_flags=()) -> str:
    """Compiles every source (always) and links libgss.so next to this file."""
    return _build_library(OUT, BUILD_DIR, HIPCC_FLAGS + list(extra_flags), verbose)


# The host sanitizer run (tests/test_gpu_host_sanitized.py): the library with its
# host code under AddressSanitizer and UndefinedBehaviorSanitizer (each option
# applies to the host pass only; the device code is built as usual), and a driver
# built with the same sanitizers that exercises it through the C ABI.
SAN_DIR = os.path.join(ROOT, "tests", "sanitize")
SAN_LIB = os.path.join(SAN_DIR, "libgss_host_san.so")
SAN_DRIVER = os.path.join(SAN_DIR, "host_driver")
HOST_SANITIZERS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                   "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
DRIVER_SANITIZERS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def build_sanitized(verbose: bool = False) -> str:
    """Builds the sanitized library and its driver into tests/sanitize."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    clang = os.path.join(rocm, "lib", "llvm", "bin", "clang")
    obj_dir = os.path.join(BUILD_DIR, "host_san")
    _build_library(SAN_LIB, obj_dir, HIPCC_FLAGS + ["-g"] + HOST_SANITIZERS, verbose)
    oracle_obj = os.path.join(obj_dir, "oracle.o")
    steps = [
        [clang, "-O1", "-g", *DRIVER_SANITIZERS, "-c", os.path.join(ROOT, "oracle", "oracle.c"), "-o", oracle_obj],
        [clang + "++", "-O1", "-g", "-std=c++17", *DRIVER_SANITIZERS, "-D__HIP_PLATFORM_AMD__",
         "-I", os.path.join(ROOT, "include"), "-I", os.path.join(rocm, "include"),
         os.path.join(SAN_DIR, "host_driver.cpp"), oracle_obj, "-o", SAN_DRIVER + ".tmp",
         "-L", SAN_DIR, "-lgss_host_san", "-Wl,-rpath,$ORIGIN",
         "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(rocm, "lib")],
    ]
    for cmd in steps:
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"sanitized driver build failed:\n{r.stdout}\n{r.stderr}")
    os.replace(SAN_DRIVER + ".tmp", SAN_DRIVER)
    return SAN_DRIVER


def _build_library(out: str, obj_dir: str, flags, verbose: bool) -> str:
    os.makedirs(obj_dir, exist_ok=True)
    hipcc = _hipcc()

    def compile_one(src):
        obj = os.path.join(obj_dir, src.replace(".hip", ".o"))
        cmd = [hipcc, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = out + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))

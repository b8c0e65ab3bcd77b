"""Compile the HIP/C++ sources into the in-tree shared library ``libplanb.so``.

Every HIP source is built for gfx950 only, with packed-FP32 instruction
selection disabled.  The library links only the HIP runtime.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libplanb.so")
OBJDIR = os.path.join(PKG, "_build")

HIP_SOURCES = ["lookup.hip", "learned.hip", "batches.hip", "multi.hip", "build_device.hip"]
CXX_SOURCES = ["api.cpp", "builder.cpp", "server.cpp", "cpu_btree.cpp", "lifetime.cpp"]
# plain host C++ that uses no HIP at all (x86 vector intrinsics chosen at run time): the host compiler
HOST_SOURCES = ["cpu_paper_tree.cpp"]
CXX = os.environ.get("CXX", "g++")
# host code of the CPU baseline: AVX2 vector compares (any x86-64 server since 2015)
EXTRA_FLAGS = {"cpu_btree.cpp": ["-mavx2"],
               # matrix-core results straight into VGPRs (no accumulation-register
               # copies before the vector instructions that read them)
               "learned.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]
HIP_ONLY = ["--offload-arch=gfx950", "-mcode-object-version=5", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJDIR, src + ".o")
    if src.endswith(".hip"):
        cmd = [HIPCC, *HIP_ONLY, *COMMON, *EXTRA_FLAGS.get(src, []), "-c", path, "-o", obj]
    elif src in HOST_SOURCES:
        cmd = [CXX, *COMMON, "-c", path, "-o", obj]
    else:  # host C++ that calls the HIP runtime: compiled as host-only HIP code
        cmd = [HIPCC, *COMMON, *EXTRA_FLAGS.get(src, []), "-D__HIP_PLATFORM_AMD__", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    """Compile every source (always) and link libplanb.so; returns its path."""
    os.makedirs(OBJDIR, exist_ok=True)
    sources = [s for s in HIP_SOURCES + CXX_SOURCES + HOST_SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = min(len(sources), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, sources))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    shutil.rmtree(OBJDIR, ignore_errors=True)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()

"""Builds the HIP library ``libaesgpu.so`` in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libaesgpu.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["aes_host.cpp", "aes_kernels.hip", "aes_batch.hip", "aes_server.cpp", "aes_pipeline.cpp"]

# Packed FP32 instructions are turned off for all device code.
HIP_FLAGS = ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def objects(build_dir: str) -> list[str]:
    return [os.path.join(build_dir, os.path.splitext(s)[0] + ".o") for s in SOURCES]


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Compiles every source (always) and links ``libaesgpu.so``."""
    build_dir = os.path.join(PKG, "_build")
    os.makedirs(build_dir, exist_ok=True)
    procs = []
    for src, obj in zip(SOURCES, objects(build_dir)):
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [HIPCC, *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC, *lang, "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        while sum(p.poll() is None for _, p in procs) >= jobs:
            procs[0][1].wait()
    for cmd, p in procs:
        if p.wait() != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}")
    tmp = LIB + f".tmp{os.getpid()}"
    link = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objects(build_dir), "-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)

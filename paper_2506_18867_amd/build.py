"""Builds libbsc.so (the HIP library behind include/bsc.h) for gfx950 with hipcc.

Every HIP source is compiled with the device target feature ``-packed-fp32-ops``, so the
compiler does not pair float operations into packed-FP32 instructions, and the objects are
linked into ``paper_2506_18867_amd/libbsc.so``. hipcc passes the feature to both of its
passes: the host pass does not know it and prints "not a recognized feature ... ignoring",
which is harmless; the gfx950 device pass applies it (a float2 multiply-add compiles to one
packed FMA without the feature and to two scalar FMAs with it). Run
``python -m paper_2506_18867_amd.build``."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbsc.so")
SOURCES = ["host.cpp", "eval.hip", "solve.hip", "net.hip", "contact.hip", "mg.hip", "partial.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-ffp-contract=fast", "-munsafe-fp-atomics"]


def _compile(src: str) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        cmd = [HIPCC, "-x", "hip"] + DEVICE + COMMON + ["-c", path, "-o", obj]
    else:
        cmd = [HIPCC, "-D__HIP_PLATFORM_AMD__"] + COMMON + ["-c", path, "-o", obj]
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False) -> str:
    with cf.ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

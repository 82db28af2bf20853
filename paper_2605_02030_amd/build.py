"""Compile libuhnsw.so for gfx950 with hipcc (in-tree, next to this file)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libuhnsw.so")
ARCH = os.environ.get("UHNSW_OFFLOAD_ARCH", "gfx950")

# -ffp-contract=off: every multiply-add in the kernels is an explicit fma, so
# the base distances follow one rounding order. Packed FP32 instructions are
# disabled for all device code.
DEVICE_FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-ffp-contract=off",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-I", INCLUDE, "-I", CSRC]
HOST_FLAGS = ["-O2", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC]


def build(verbose: bool = False) -> str:
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    jobs = []
    for src, flags, lang in (("uhnsw_kernels.hip", DEVICE_FLAGS, ["-x", "hip"]),
                             ("uhnsw_probe.hip", DEVICE_FLAGS, ["-x", "hip"]),
                             ("uhnsw_host.cpp", HOST_FLAGS, ["-D__HIP_PLATFORM_AMD__"]),
                             ("uhnsw_serve.cpp", HOST_FLAGS, ["-D__HIP_PLATFORM_AMD__", "-pthread"])):
        obj = os.path.join(bdir, src + ".o")
        cmd = ["hipcc", *lang, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append(subprocess.Popen(cmd))
        objs.append(obj)
    for j in jobs:
        if j.wait() != 0:
            raise RuntimeError("hipcc failed")
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)

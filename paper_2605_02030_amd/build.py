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


def _units():
    """(source, object name, flags) of every translation unit. The walk,
    fused and descent kernels are compiled once per walk storage (FP32, BF16,
    FP16) and index variant (standard, extended) from one source, so the
    instantiations build in parallel."""
    hip = ["-x", "hip"]
    units = [("uhnsw_kernels.hip", "uhnsw_kernels", hip + DEVICE_FLAGS),
             ("uhnsw_probe.hip", "uhnsw_probe", hip + DEVICE_FLAGS),
             ("uhnsw_build.hip", "uhnsw_build", hip + DEVICE_FLAGS)]
    for s in range(3):
        for e in range(2):
            units.append(("uhnsw_walk_part.hip", f"uhnsw_walk_part_{s}_{e}",
                          hip + DEVICE_FLAGS + [f"-DUHNSW_PART_S={s}", f"-DUHNSW_PART_E={e}"]))
    units += [("uhnsw_host.cpp", "uhnsw_host", ["-D__HIP_PLATFORM_AMD__"] + HOST_FLAGS),
              ("uhnsw_serve.cpp", "uhnsw_serve", ["-D__HIP_PLATFORM_AMD__", "-pthread"] + HOST_FLAGS)]
    return units


def build(verbose: bool = False) -> str:
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    jobs_max = max(1, min(int(os.environ.get("MAX_JOBS") or 0) or os.cpu_count() or 1, 16))
    running = []

    def reap(block):
        while running and (block or len(running) >= jobs_max):
            j = running.pop(0)
            if j.wait() != 0:
                raise RuntimeError("hipcc failed")
            block = False if len(running) < jobs_max else block

    for src, name, flags in _units():
        obj = os.path.join(bdir, name + ".o")
        cmd = ["hipcc", *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        reap(False)
        running.append(subprocess.Popen(cmd))
        objs.append(obj)
    for j in running:
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

"""Build libhair.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2405_10565_amd.build          # or build() from Python

The library is written for MI355X only (--offload-arch=gfx950).  Flags:
  -ffp-contract=off        the integer-deciding float32 steps must not be fused
  -packed-fp32-ops off     no packed FP32 instructions in any kernel
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhair.so")
SOURCES = ["hair_api.hip", "hair_kernels.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm toolchain required to build libhair.so)")


def flags() -> list[str]:
    return ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unused-result"]


def build(verbose: bool = False, out: str = LIB, defines: tuple = ()) -> str:
    """Compile every HIP source for gfx950 and link libhair.so (default: next to this file).

    defines: extra preprocessor symbols, e.g. ("HAIR_PHASE_STATS",) for per-phase cycle
    counters printed after each frame (an instrumented build written to `out`)."""
    objs = []
    build_dir = os.path.join(os.path.dirname(os.path.abspath(out)), "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), *flags(), *[f"-D{d}" for d in defines], "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

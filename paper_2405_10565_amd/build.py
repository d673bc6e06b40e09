"""Build libhair.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2405_10565_amd.build          # or build() from Python

The library is written for MI355X only (--offload-arch=gfx950).  Flags:
  -ffp-contract=off        the integer-deciding float32 steps must not be fused
  -packed-fp32-ops off     no packed FP32 instructions in any kernel

build_checks() also builds the C-ABI checker (csrc/abi_check.cpp) twice, into bin/:
  abi_check        against libhair.so
  abi_check_asan   against libhair_asan.so, the host layer (hair_api) compiled with
                   AddressSanitizer and UndefinedBehaviorSanitizer for its host code only (the
                   sanitizers are host-side: each -fsanitize flag goes to the host compilation)
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
BIN = os.path.join(HERE, "bin")
LIB_ASAN = os.path.join(HERE, "libhair_asan.so")
# host-side sanitizers (device code is built as usual)
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                 "-Xarch_host", "-g"]
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


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build_checks(verbose: bool = False) -> list[str]:
    """bin/abi_check (linked with libhair.so) and bin/abi_check_asan (linked with
    libhair_asan.so: hair_api.hip with host-side ASan + UBSan, hair_kernels.hip's object from
    build()).  Run build() first."""
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    os.makedirs(BIN, exist_ok=True)
    kobj = os.path.join(build_dir, "hair_kernels.o")
    if not os.path.exists(kobj):
        raise RuntimeError("hair_kernels.o is missing: run build() first")
    aobj = os.path.join(build_dir, "hair_api_asan.o")
    _run([hipcc(), *flags(), *HOST_SANITIZE, "-c", os.path.join(CSRC, "hair_api.hip"), "-o", aobj], verbose)
    _run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", aobj, kobj, "-o", LIB_ASAN + ".tmp"], verbose)
    os.replace(LIB_ASAN + ".tmp", LIB_ASAN)
    src = os.path.join(CSRC, "abi_check.cpp")
    outs = []
    for name, lib, extra in (("abi_check", "libhair.so", []), ("abi_check_asan", "libhair_asan.so", HOST_SANITIZE)):
        obj = os.path.join(build_dir, name + ".o")
        exe = os.path.join(BIN, name)
        _run([hipcc(), "-O1", "-std=c++17", f"--offload-arch={ARCH}", *extra, "-c", src, "-o", obj], verbose)
        _run([hipcc(), f"--offload-arch={ARCH}", *extra, obj, f"-L{HERE}", f"-l:{lib}",
              "-Wl,-rpath,$ORIGIN/..", "-o", exe], verbose)
        outs.append(exe)
    return outs


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
    print(build_checks(verbose="-v" in sys.argv))

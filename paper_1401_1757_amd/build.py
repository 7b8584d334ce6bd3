"""Build librr.so (the C-ABI library with its gfx950 HIP kernels) in-tree.

Usage: python -m paper_1401_1757_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "librr.so")
OBJDIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Packed FP32 instructions are left to the compiler's discretion nowhere: the
# feature is switched off for every device compile.
DEVICE_FLAGS = ["-x", "hip", f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function"]
HOST_FLAGS = ["-x", "c++", "-O2", "-fPIC", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-Wall"]

DEVICE_SOURCES = ["rr_kernels.hip", "rr_kernels_pat.hip", "rr_kernels_ring.hip", "rr_mlp.hip",
                  "rr_scen.hip"]
HOST_SOURCES = ["rr_host.cpp", "rr_surrogate.cpp"]


def _sources():
    dev = [s for s in DEVICE_SOURCES if os.path.exists(os.path.join(CSRC, s))]
    host = [s for s in HOST_SOURCES if os.path.exists(os.path.join(CSRC, s))]
    return dev, host


def _stale(obj: str, src: str) -> bool:
    """The object is missing or older than its source or any header."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    headers = [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    headers += [os.path.join(INCLUDE, h) for h in os.listdir(INCLUDE) if h.endswith(".h")]
    return any(os.path.getmtime(f) > t for f in [src, *headers])


def build(verbose: bool = False, jobs: int = 4, incremental: bool = False) -> str:
    """Compile every source and link librr.so.  Recompiles everything unless
    incremental, which keeps objects newer than their source and every header."""
    os.makedirs(OBJDIR, exist_ok=True)
    dev, host = _sources()
    inc = ["-I", INCLUDE, "-I", CSRC, "-I", "/opt/rocm/include"]
    cmds, objs = [], []
    for s in dev:
        o = os.path.join(OBJDIR, s + ".o")
        src = os.path.join(CSRC, s)
        if not incremental or _stale(o, src):
            cmds.append([HIPCC, *DEVICE_FLAGS, *inc, "-c", src, "-o", o])
        objs.append(o)
    for s in host:
        o = os.path.join(OBJDIR, s + ".o")
        src = os.path.join(CSRC, s)
        if not incremental or _stale(o, src):
            cmds.append([HIPCC, *HOST_FLAGS, *inc, "-c", src, "-o", o])
        objs.append(o)
    from concurrent.futures import ThreadPoolExecutor

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.call(cmd)

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        rcs = list(ex.map(run, cmds))
    if any(rcs):
        raise RuntimeError("librr build failed")
    tmp = LIB + ".tmp"
    link = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs,
            "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv)
    print(LIB)

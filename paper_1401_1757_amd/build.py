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
                  "rr_scen.hip", "rr_noalloc.hip"]
HOST_SOURCES = ["rr_host.cpp", "rr_surrogate.cpp"]


def _sources():
    dev = [s for s in DEVICE_SOURCES if os.path.exists(os.path.join(CSRC, s))]
    host = [s for s in HOST_SOURCES if os.path.exists(os.path.join(CSRC, s))]
    return dev, host


def _includes(path: str, seen: set) -> set:
    """The project headers a source includes, directly or through other headers."""
    import re
    with open(path) as f:
        names = re.findall(r'^\s*#\s*include\s+"([^"]+)"', f.read(), re.M)
    for n in names:
        for d in (os.path.dirname(path), CSRC, INCLUDE):
            h = os.path.join(d, n)
            if os.path.exists(h):
                if h not in seen:
                    seen.add(h)
                    _includes(h, seen)
                break
    return seen


def _stale(obj: str, src: str) -> bool:
    """The object is missing or older than its source or a header it includes."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(f) > t for f in [src, *_includes(src, set())])


def build(verbose: bool = False, jobs: int = 4, incremental: bool = False) -> str:
    """Compile every source and link librr.so.  Recompiles everything unless
    incremental, which keeps objects newer than their source and its headers."""
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


SAN_LIB = os.path.join(OBJDIR, "librr_hostsan.so")


def build_host_sanitized(verbose: bool = False) -> str:
    """A CPU-only checking build: the host runtime (validation, planning,
    the ABI) compiled with AddressSanitizer and UndefinedBehaviorSanitizer,
    linked with the device objects of the last build(), as _build/librr_hostsan.so.
    Load it with the clang ASan runtime preloaded; it is never the product
    library."""
    dev, host = _sources()
    inc = ["-I", INCLUDE, "-I", CSRC, "-I", "/opt/rocm/include"]
    objs = []
    for s in dev:
        o = os.path.join(OBJDIR, s + ".o")
        if not os.path.exists(o):
            raise RuntimeError(f"{o} is missing: run build() first")
        objs.append(o)
    san = ["-g", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-fno-sanitize-recover=undefined"]
    for s in host:
        o = os.path.join(OBJDIR, s + ".san.o")
        cmd = [HIPCC, *HOST_FLAGS, *san, *inc, "-c", os.path.join(CSRC, s), "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(o)
    link = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-Xarch_host", "-fsanitize=address",
            "-Xarch_host", "-fsanitize=undefined", "-shared-libasan", "-o", SAN_LIB, *objs,
            "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    return SAN_LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv)
    print(LIB)

"""The host-side ABI checks (library load and exports, input validation of
bases and portfolios, clean failure without a GPU) against a build of the
host runtime with AddressSanitizer and UndefinedBehaviorSanitizer (CPU only;
the device objects are those of the normal build).  Runs in a child process
with the clang ASan runtime preloaded."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_host_checks_under_address_and_ub_sanitizers():
    from paper_1401_1757_amd import build
    rt = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("no clang AddressSanitizer runtime")
    if not all(os.path.exists(os.path.join(build.OBJDIR, s + ".o")) for s in build.DEVICE_SOURCES):
        pytest.skip("no device objects: run the normal build first")
    lib = build.build_host_sanitized()
    env = dict(os.environ)
    env.update(RR_LIB=lib, LD_PRELOAD=rt[-1], ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    code = ("import paper_1401_1757_amd as rr; rr.load_library(); "
            "print(open('/proc/self/maps').read().count('librr_hostsan'))")
    res = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                         text=True, timeout=600)
    assert res.returncode == 0 and int(res.stdout.strip().splitlines()[-1]) > 0, res.stderr[-2000:]
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "tests/test_abi_host.py"]
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (res.stdout + res.stderr)[-3000:]
    assert res.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in res.stderr and "runtime error:" not in res.stderr, tail
    assert " passed" in res.stdout, tail

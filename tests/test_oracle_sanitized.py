"""The CPU pins again, against the oracle built with AddressSanitizer and
UndefinedBehaviorSanitizer (out-of-bounds reads and writes, use after free,
signed overflow, misaligned or invalid loads in the C oracle abort the run).
The pins run in a child process with the sanitizer runtime preloaded; the
timing pin is left out (instrumented code is several times slower)."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_pins_under_address_and_ub_sanitizers():
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no AddressSanitizer runtime for gcc on this host")
    lib = oracle.build(sanitize=True)
    env = dict(os.environ)
    env.update(ORACLE_LIB=lib, LD_PRELOAD=asan, ORACLE_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
           "tests/test_oracle_pins.py", "tests/test_oracle_scenarios.py",
           "-k", "not complexity"]
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)
    tail = (res.stdout + res.stderr)[-3000:]
    assert res.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in res.stderr and "runtime error:" not in res.stderr, tail
    assert " passed" in res.stdout, tail

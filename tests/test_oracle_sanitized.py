"""The oracle's pins run once more against a build of the oracle
instrumented with the address and undefined-behaviour sanitizers (any
out-of-bounds access, use after free, signed overflow or misaligned access
in the C code aborts the run).  CPU only."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    out = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


def test_pins_under_sanitizers(orc):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc has no address-sanitizer runtime here")
    orc.build(sanitize=True)
    env = dict(os.environ)
    env[orc.SANITIZE_ENV] = "1"
    env["LD_PRELOAD"] = asan
    # the interpreter itself is not instrumented: its own allocations at exit
    # are not the oracle's leaks
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "4"
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-s", "-p", "no:cacheprovider",
           os.path.join(ROOT, "tests", "test_oracle_pins.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout[-3000:] + "\n" + r.stderr[-3000:])
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "failed" not in r.stdout, tail
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, tail

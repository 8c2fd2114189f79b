"""The CPU oracle and the synthetic-input generator built with
AddressSanitizer and UndefinedBehaviorSanitizer (gcc), running the oracle's
own pins and the generator round trips in a child process with the sanitizer
runtimes preloaded: any out-of-bounds access, use after free, signed
overflow, misaligned or out-of-range shift fails the test."""
import os
import subprocess
import sys

import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.slow
def test_oracle_and_synth_under_asan_ubsan():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    oracle.build(force=True, sanitized=True)
    synth.build(force=True, sanitized=True)
    env = dict(os.environ)
    env.update(PGSGD_SANITIZED="1", LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=97",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=98")
    # the oracle's pins, minus the long statistical runs; every oracle entry point is exercised
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu and not slow",
           "tests/test_oracle.py", "tests/test_batch_resolution.py"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out
    assert r.returncode == 0, out
    assert " passed" in r.stdout, out

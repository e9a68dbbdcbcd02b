"""The host code (planner and C ABI) under AddressSanitizer and UBSan.

The host checks of test_library_host.py (exports, synchronous argument
errors, plan creation failing on a machine without a GPU and freeing what it
had built, the ADI parameters of every wavenumber against the oracle) run
again in a child process against a build whose host sources are compiled with
-fsanitize=address,undefined; any report fails the child.  Device code is not
instrumented.
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_code_under_asan_and_ubsan():
    from paper_2206_04827_amd import build_sanitized as bs
    if not os.path.exists(os.path.join(bs.BUILD, "adi.o")):
        pytest.skip("the regular build's objects are missing (run __graft_entry__.build() first)")
    lib = bs.build()
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": bs.runtime_preload(),
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=99",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1:exitcode=98",
        "CYLSPEC_LIBRARY": lib,
        "PYTHONDONTWRITEBYTECODE": "1",
    })
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
           os.path.join(ROOT, "tests", "test_library_host.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert r.returncode == 0, out[-3000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out
    assert " passed" in out

"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer: the
library's host preprocessing and boundary code (libdgswe_asan.so, device code
built as usual) and the oracle (liboracle_asan.so, one thread) are rebuilt
with the sanitizers, then the rest of the CPU test suite runs against them
in a child process with clang's ASan runtime preloaded; any report ends that
process with an error."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_cpu_suite_clean_under_asan_and_ubsan():
    from oracle.oracle import build_oracle
    from paper_2508_21208_amd.build import asan_runtime, build
    rt = asan_runtime()
    if not rt:
        pytest.skip("clang's shared ASan runtime is not installed")
    lib = build(verbose=False, sanitize=True)
    olib = build_oracle(sanitize=True)
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", DGSWE_LIB=lib, DGSWE_ORACLE_LIB=olib)
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-m", "not gpu", "-x", "-q",
                        "-p", "no:cacheprovider", "--ignore", os.path.join(ROOT, "tests", "test_sanitizers.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    assert " passed" in r.stdout, tail

"""The host side of the library under AddressSanitizer and
UndefinedBehaviorSanitizer: the C-ABI host tests run again, in a child
interpreter, against the host-sanitized build (``python -m
paper_2605_10128_amd.build --sanitize``), with the ASan runtime preloaded.
Skipped when that build or the runtime is absent; a report from either
sanitizer fails the test."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_LIB = os.path.join(ROOT, "paper_2605_10128_amd", "_build", "libtto_san.so")


def _asan_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def test_host_abi_tests_clean_under_asan_and_ubsan():
    rt = _asan_runtime()
    if not os.path.exists(SAN_LIB) or rt is None:
        pytest.skip("host-sanitized library or ASan runtime not present")
    env = dict(os.environ, TTO_LIBRARY=SAN_LIB, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_host.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out

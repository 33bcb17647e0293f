"""The host C++ (plan builder, C ABI, solver host code) under AddressSanitizer
and UndefinedBehaviorSanitizer.

Builds the sanitizer variant of the library (host objects only; the device
code is the product's) and runs the host-side ABI tests against it in a
child process with the sanitizer runtimes preloaded. Any sanitizer report
aborts that process, so this test fails on it. No GPU is used.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    try:
        path = subprocess.run(["g++", f"-print-file-name={name}"], check=True,
                              capture_output=True, text=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_host_abi_tests_clean_under_asan_ubsan():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("g++ sanitizer runtimes not installed")
    from paper_2501_04684_amd import build as B
    lib = B.build(sanitize=True)
    env = dict(os.environ)
    env.update(UBF_LIBRARY=lib, LD_PRELOAD=f"{asan} {ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "tests/test_capi_host.py", "tests/test_training_host.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    report = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "runtime error" not in report and "AddressSanitizer" not in report, report

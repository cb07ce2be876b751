"""The runtime's host code under AddressSanitizer and UndefinedBehavior-
Sanitizer on the GPU: the driver (tests/native/api_sanitize.cpp, built by
paper_1411_3133_amd.build.build_sanitized next to the library) exercises
descriptor validation, single instances, checkpoints, batches with
retirement, views, graph and eager windows and the warm-start network
through the C ABI; any invalid host access or undefined behaviour in the
runtime aborts it. Leak checking is off: the HIP runtime keeps allocations
until the process ends."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "paper_1411_3133_amd", "api_sanitize")


def test_runtime_host_code_under_sanitizers(tmp_path):
    assert os.path.exists(DRIVER), "build the sanitizer driver first (paper_1411_3133_amd.build.build_sanitized)"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([DRIVER, str(tmp_path)], capture_output=True, text=True, env=env, timeout=240)
    print(r.stdout[-3000:], r.stderr[-3000:])
    assert r.returncode == 0
    assert "api_sanitize: 0 failure(s)" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr

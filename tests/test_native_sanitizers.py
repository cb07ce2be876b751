"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc) and driven through every geometry kind and wall type by a small C
program: no invalid access, leak or undefined behaviour may be reported."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-o", exe, os.path.join(ROOT, "tests", "native", "oracle_sanitize.c"),
           os.path.join(ROOT, "oracle", "mlbm_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert r.stdout.count(" ok") == 6


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
def test_streaming_fold_host_code_under_sanitizers(tmp_path):
    """The kernels' streaming fold, compiled for the host with AddressSanitizer
    and UndefinedBehaviorSanitizer (sanitizers on the host pass only): every
    source inside the grid, and a permutation for the bounce-back walls, on
    276 small grids."""
    exe = str(tmp_path / "fold_sanitize")
    src = os.path.join(ROOT, "tests", "native", "fold_sanitize.cpp")
    cmd = ["/opt/rocm/bin/hipcc", "-std=c++17", "-O1", "-g", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"), src, "-o", exe]  # noqa: E501
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "276 grids ok" in r.stdout

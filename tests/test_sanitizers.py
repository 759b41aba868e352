"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code (no GPU):
the C oracle driven through every entry point, and the library's host half
(validation, layout, masks, unequal windows) driven through its pure-host calls.
Sanitizers are applied to host code only."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, timeout=600, env=ENV)
    assert r.returncode == 0, (cmd, r.stdout[-3000:], r.stderr[-3000:])
    return r


def test_oracle_under_asan_ubsan():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_san")
        _run(["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=undefined", "-fopenmp", os.path.join(SAN, "oracle_driver.c"),
              os.path.join(ROOT, "oracle", "rewl_oracle.c"), "-o", exe, "-lquadmath", "-lm"], d)
        r = _run([exe], d)
        assert r.stdout.count("rc=0") == 4


@pytest.mark.skipif(not (shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc")),
                    reason="hipcc not installed")
def test_library_host_code_under_asan_ubsan():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    with tempfile.TemporaryDirectory() as d:
        lib = os.path.join(d, "librewl_san.so")
        # the sanitizer flags apply to the host compilation only (-Xarch_host before each)
        _run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-shared", "-fPIC", "-ffp-contract=off",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-omit-frame-pointer",
              os.path.join(ROOT, "paper_1407_5140_amd", "csrc", "rewl_api.hip"), "-o", lib], d)
        exe = os.path.join(d, "host_san")
        # the driver links with the same compiler's sanitizer runtime as the library
        clang = os.path.join(os.path.dirname(os.path.realpath(hipcc)), "..", "llvm", "bin", "clang++")
        clang = clang if os.path.exists(clang) else "/opt/rocm/llvm/bin/clang++"
        _run([clang, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
              os.path.join(SAN, "host_driver.cpp"), lib, "-o", exe, "-Wl,-rpath," + d], d)
        r = _run([exe], d)
        assert "0 failures" in r.stdout

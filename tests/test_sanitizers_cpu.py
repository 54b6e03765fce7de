"""The host code (the oracle and the library's host construction) built with
AddressSanitizer and UBSan and run on the CPU: no memory error, no undefined
behaviour, and every build a bijection (harnesses in tests/sanitize/)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]


def _compile(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    if r.returncode != 0 and "asan" in (r.stderr + r.stdout).lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-2000:]


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "0 failures" in r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_harness")
    _compile(["gcc", "-std=c11", *SAN, "-I", os.path.join(ROOT, "oracle"),
              os.path.join(ROOT, "tests", "sanitize", "oracle_harness.c"),
              os.path.join(ROOT, "oracle", "ptrhash_oracle.c"), "-o", exe, "-lm"])
    _run(exe)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_host_builder_under_sanitizers(tmp_path):
    exe = str(tmp_path / "builder_harness")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2502_15539_amd", "csrc"),
           "-I", "/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]
    _compile(["g++", "-std=c++17", *SAN, *inc, os.path.join(ROOT, "tests", "sanitize", "builder_harness.cpp"),
              os.path.join(ROOT, "paper_2502_15539_amd", "csrc", "builder.cpp"), "-o", exe, "-lpthread"])
    _run(exe)

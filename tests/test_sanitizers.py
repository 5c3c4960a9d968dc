"""The oracle and the library's host-only code built with AddressSanitizer
and UndefinedBehaviorSanitizer (host compilers only, no device code), run on
small instances of every mode; any finding aborts the run (CPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HELPERS = os.path.join(ROOT, "tests", "helpers")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")

pytestmark = pytest.mark.slow


def _compile(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _compile(["gcc", "-std=gnu11", "-ffp-contract=off", "-fopenmp", *SAN,
              os.path.join(ROOT, "oracle", "pamc_oracle.c"), os.path.join(ROOT, "oracle", "enumerate.c"),
              os.path.join(HELPERS, "oracle_sanitize.c"), "-o", exe, "-lm"])
    assert "oracle sanitizer run ok" in _run(exe)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_library_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "host_san")
    _compile(["g++", "-std=c++17", *SAN, os.path.join(ROOT, "paper_1710_09025_amd", "csrc", "instances.cpp"),
              os.path.join(HELPERS, "host_sanitize.cpp"), "-o", exe])
    assert "host sanitizer run ok" in _run(exe)

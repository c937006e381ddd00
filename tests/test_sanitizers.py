"""Host code under the address and undefined-behaviour sanitizers (CPU).

The library's host-only logic (csrc/host.cpp: offset validation, the spatial
ordering of segments, buffer layouts, the autotuner's cache format, the
radius-model checkpoint header) and the C oracle are built with g++ / gcc
and -fsanitize=address,undefined, then exercised by the self-test programs in
tests/native/.  A sanitizer report aborts the program, failing the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]


def _run(cmd, exe, want, tmp_path):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and want in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_library_host_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_selftest")
    cmd = ["g++", "-std=c++17", "-Wall", "-Wextra", *SAN,
           os.path.join(NATIVE, "host_selftest.cpp"),
           os.path.join(ROOT, "paper_2112_10408_amd", "csrc", "host.cpp"), "-o", exe]
    _run(cmd, exe, "host ok", tmp_path)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_selftest")
    cmd = ["gcc", "-std=c11", "-Wall", "-Wno-unknown-pragmas", "-ffp-contract=off", *SAN,
           os.path.join(NATIVE, "oracle_selftest.c"), os.path.join(ROOT, "oracle", "tnn_oracle.c"),
           "-o", exe, "-lm"]
    _run(cmd, exe, "oracle ok", tmp_path)

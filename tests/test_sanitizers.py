"""Host code under the address and undefined-behaviour sanitizers (CPU).

The library's host-only logic (csrc/host.cpp: offset validation, the spatial
ordering of segments, buffer layouts, the autotuner's cache format, the
radius-model checkpoint header) and the C oracle are built with g++ / gcc
and -fsanitize=address,undefined, then exercised by the self-test programs in
tests/native/ (and the host kd order against its numpy rendering).  A
sanitizer report aborts the program, failing the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]


def _san_env():
    # the environment is passed on as it is; a library preloaded ahead of the
    # sanitizer runtime is tolerated rather than removed
    return dict(os.environ,
                ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
                UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, exe, want, tmp_path):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = _san_env()
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


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_kd_order_references_agree(tmp_path):
    """The library's host reference of the kd order (built under the
    sanitizers) and the numpy rendering the GPU test compares the device
    order with give the same order: random keys, tied keys, -0 and +0,
    a flat axis, sizes around the block and up to several levels."""
    import numpy as np
    from kd_reference import kd_reference

    exe = str(tmp_path / "kd_order")
    cmd = ["g++", "-std=c++17", "-Wall", "-Wextra", *SAN,
           os.path.join(NATIVE, "kd_order_main.cpp"),
           os.path.join(ROOT, "paper_2112_10408_amd", "csrc", "host.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = _san_env()
    rng = np.random.default_rng(3)
    for n in (1, 2, 63, 64, 65, 129, 1000, 5000, 20000):
        k = rng.normal(0.0, 100.0, (n, 4)).astype(np.float32)
        k[:, 2] *= np.float32(0.01)
        if n > 10:
            k[5] = k[3]
            k[7, 0], k[8, 0] = np.float32(-0.0), np.float32(0.0)
        if n == 5000:
            k[:, 1] = np.float32(7.0)
        kin, kout = tmp_path / "keys.bin", tmp_path / "order.bin"
        kin.write_bytes(np.int64(n).tobytes() + k.tobytes())
        r = subprocess.run([exe, str(kin), str(kout)], capture_output=True, text=True, env=env,
                           timeout=120)
        assert r.returncode == 0, r.stderr[-3000:]
        host = np.frombuffer(kout.read_bytes(), dtype=np.int32)
        assert np.array_equal(host, kd_reference(k)), n

"""The host-only planning logic (csrc/ibp_host.cpp: FFT factorisation and
Bluestein tables, line LU tables, line-solve shapes, the dimension check,
the tuning-cache parser and writer, the persistent batch schedule's queue
assignment and stage order) built on its own with AddressSanitizer and
UndefinedBehaviorSanitizer and run through tests/host_selftest.cpp.  The
self-test checks invariants over sweeps of inputs (malformed cache lines
included) and prints its dimension checks, which must agree with the HIP
library's ibp_check_dims.  CPU only."""

import os
import shutil
import subprocess

import pytest

from paper_2609_19130_amd import ibpoisson as ibp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2609_19130_amd", "csrc")


@pytest.fixture(scope="module")
def selftest(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    out = tmp_path_factory.mktemp("host_selftest")
    exe = str(out / "host_selftest")
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-Wall", "-I", CSRC, os.path.join(ROOT, "tests", "host_selftest.cpp"),
           os.path.join(CSRC, "ibp_host.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(out)], capture_output=True, text=True, env=env, timeout=300)
    return r


def test_selftest_clean_under_sanitizers(selftest):
    assert selftest.returncode == 0, selftest.stderr[-4000:]
    assert "0 failures" in selftest.stderr
    assert "runtime error" not in selftest.stderr and "AddressSanitizer" not in selftest.stderr


def test_dimension_checks_match_library(selftest):
    rows = [tuple(map(int, line.split()[1:])) for line in selftest.stdout.splitlines() if line.startswith("dims ")]
    assert len(rows) > 3000
    for nx, ny, nz, st in rows:
        assert ibp.check_dims(nx, ny, nz) == st, (nx, ny, nz, st)

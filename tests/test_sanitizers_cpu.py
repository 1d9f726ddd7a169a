"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two programs are built with g++/gcc -fsanitize=address,undefined and run:
the library's threaded host setup (paper_1512_04629_amd/csrc/host_setup.cpp)
driven by tests/sanitize/host_setup_check.cpp, and the C oracle
(oracle/amg_oracle.c) driven by tests/sanitize/oracle_check.c.  Any
out-of-bounds access, use after free, leak or undefined behaviour aborts the
program with a report and fails the test.  No device code is built here."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-ffp-contract=off"]


def _build_and_run(tmp_path, compiler, std, sources, extra=()):
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not available")
    exe = str(tmp_path / "check")
    cmd = [compiler, *SAN, std, *[os.path.join(ROOT, s) for s in sources], "-o", exe, *extra]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    if b.returncode != 0 and "sanitize" in b.stderr and ("cannot find" in b.stderr or "not found" in b.stderr):
        pytest.skip("sanitizer runtime not installed")
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    return r.stdout


def test_host_setup_under_asan_ubsan(tmp_path):
    out = _build_and_run(tmp_path, "g++", "-std=c++17",
                         ["paper_1512_04629_amd/csrc/host_setup.cpp", "tests/sanitize/host_setup_check.cpp"],
                         ["-pthread"])
    assert "ok" in out


def test_oracle_under_asan_ubsan(tmp_path):
    out = _build_and_run(tmp_path, "gcc", "-std=c99", ["oracle/amg_oracle.c", "tests/sanitize/oracle_check.c"],
                         ["-lm"])
    assert "ok" in out

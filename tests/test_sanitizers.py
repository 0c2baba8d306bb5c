"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two self-test programs are built with gcc/g++ -fsanitize=address,undefined
(every finding fatal) and run:
  * tests/sanitize/oracle_selftest.c with oracle/sfo_oracle.c: every oracle
    entry point on small grids, round trips and norms, and rejected arguments;
  * tests/sanitize/validate_selftest.cpp with the C ABI's argument checks
    (paper_1012_3911_amd/csrc/sfo_validate.h, the code sfo_create_grid and the
    table setters run before they touch a device): valid and invalid
    descriptors, tables and step ranges, including values near the int64
    limits whose arithmetic must not overflow."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(cmd, exe, expect, tmp_path):
    if shutil.which(cmd[0]) is None:
        pytest.skip("%s not available" % cmd[0])
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env, cwd=str(tmp_path))
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert expect in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_selftest")
    cmd = ["gcc", "-std=c11"] + SAN + [os.path.join(ROOT, "tests", "sanitize", "oracle_selftest.c"),
                                       os.path.join(ROOT, "oracle", "sfo_oracle.c"), "-lm", "-o", exe]
    _run(cmd, exe, "oracle selftest ok", tmp_path)


def test_abi_validation_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "validate_selftest")
    cmd = ["g++", "-std=c++17"] + SAN + ["-I", os.path.join(ROOT, "include"),
                                         "-I", os.path.join(ROOT, "paper_1012_3911_amd", "csrc"),
                                         os.path.join(ROOT, "tests", "sanitize", "validate_selftest.cpp"), "-o", exe]
    _run(cmd, exe, "validate selftest ok", tmp_path)

"""The oracle built under AddressSanitizer and UndefinedBehaviorSanitizer
(g++, CPU only): every entry point driven on small inputs by
tests/native/oracle_sanitize_check.cpp, which also checks that the class
oracle at class 0 equals the simple-graph oracle."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_asan_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "oracle_sanitize_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-ffp-contract=off", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", os.path.join(ROOT, "oracle", "gesmc_oracle.cpp"),
           os.path.join(ROOT, "oracle", "gen_oracle.cpp"), os.path.join(ROOT, "tests", "native", "oracle_sanitize_check.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1"))
    if r.returncode != 0 and "LeakSanitizer does not work under ptrace" in r.stderr:
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                           env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr[-3000:]

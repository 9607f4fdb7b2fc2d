"""Host copy pool of the serving loop (paper_2111_03005_amd/csrc/copy_pool.h):
byte-exact copies over many jobs, under ThreadSanitizer and with 0 or many
helper threads."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def build(tmp_path, flags):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "copy_pool_check")
    cmd = [gxx, "-std=c++17", "-pthread", *flags, "-I", os.path.join(ROOT, "paper_2111_03005_amd", "csrc"),
           os.path.join(ROOT, "tests", "native", "copy_pool_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.parametrize("threads", ["0", "1", "7"])
def test_copy_pool_exact(tmp_path, threads):
    exe = build(tmp_path, ["-O2"])
    r = subprocess.run([exe, threads, "100", "9"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr


def test_copy_pool_thread_sanitizer(tmp_path):
    exe = build(tmp_path, ["-O1", "-g", "-fsanitize=thread"])
    r = subprocess.run([exe, "4", "40", "5"], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"))
    if r.returncode != 0 and "FATAL: ThreadSanitizer" in r.stderr and "unexpected memory mapping" in r.stderr:
        pytest.skip("ThreadSanitizer cannot run in this environment")
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr[-3000:]

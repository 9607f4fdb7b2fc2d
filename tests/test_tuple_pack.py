"""Packed dependency-tuple words (paper_2111_03005_amd/csrc/tuple_pack.h) on
the host: the w-bit key hash is a bijection with a working inverse, tag codes
keep the order of the 32-bit tags, the packed word orders as (key, tag), and
structured key sets spread evenly over partitions and cells.  The header is
the one the kernels include; hipcc builds the check as host code."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_tuple_pack_host_checks(tmp_path):
    hipcc = shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)
    if hipcc is None:
        pytest.skip("no hipcc")
    exe = str(tmp_path / "tuple_pack_check")
    cmd = [hipcc, "-x", "hip", "-std=c++17", "-O2", "--offload-arch=gfx950", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "paper_2111_03005_amd", "csrc"),
           os.path.join(ROOT, "tests", "native", "tuple_pack_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr

"""The C-ABI library: it loads, exports every function include/gesmc.h
declares, and the Python binding's constants and struct layouts match the
header.  No compute call is made (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gesmc.h")


def header_text():
    with open(HEADER) as fh:
        return fh.read()


def declared_functions():
    txt = re.sub(r"/\*.*?\*/", "", header_text(), flags=re.S)
    return sorted(set(re.findall(r"\b(gesmc_[a-z_]+)\s*\(", txt)))


def header_defines():
    out = {}
    for name, val in re.findall(r"#define\s+(GESMC_[A-Z_]+)\s+\(?(-?\d+)\)?", header_text()):
        out[name] = int(val)
    return out


@pytest.fixture(scope="module")
def lib():
    import paper_2111_03005_amd as gesmc
    if not os.path.exists(gesmc.LIB_PATH):
        from paper_2111_03005_amd import build
        build.build()
    return gesmc.load_library()


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", os.path.join(ROOT, "paper_2111_03005_amd", "libgesmc.so")],
                         capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (gesmc_\w+)", out))
    assert set(names) <= exported
    import paper_2111_03005_amd as gesmc
    assert set(gesmc.EXPORTS) <= set(names)


def test_binding_constants_match_header():
    import paper_2111_03005_amd as gesmc
    d = header_defines()
    assert d["GESMC_OK"] == gesmc.OK
    for name in ["E_INVAL", "E_NOT_SIMPLE", "E_RANGE", "E_NOMEM", "E_DEVICE", "E_INTERNAL"]:
        assert d["GESMC_" + name] == getattr(gesmc, name), name
    for name in ["BUCKET_AVG", "SORT_CAP", "FAST_ROUNDS", "PROFILE", "STRATEGY", "PERSIST", "PROFILE_ONLY"]:
        assert d["GESMC_OPT_" + name] == getattr(gesmc, "OPT_" + name), name


def test_struct_layouts_match_header():
    from paper_2111_03005_amd import _binding as b
    # gesmc_stats: 6 x u64, 2 x u32, 1 x double; gesmc_step_stats: 8 x u64
    assert ctypes.sizeof(b.Stats) == 6 * 8 + 2 * 4 + 8
    assert ctypes.sizeof(b.StepStats) == 8 * 8
    txt = header_text()
    assert "uint64_t attempts, legal, rej_loop, rej_exists, rej_pl;" in txt
    assert [f for f, _ in b.StepStats._fields_][:5] == ["attempts", "legal", "rej_loop", "rej_exists", "rej_pl"]


def test_kernel_names_without_gpu(lib):
    n = lib.gesmc_kernel_count()
    names = [lib.gesmc_kernel_name(i).decode() for i in range(n)]
    assert len(set(names)) == n and all(x.startswith("k_") for x in names)
    assert lib.gesmc_kernel_name(n) == b""


def test_null_context_rejected_without_gpu(lib):
    import paper_2111_03005_amd as gesmc
    assert lib.gesmc_set_option(None, gesmc.OPT_PROFILE, 1) == gesmc.E_INVAL
    assert lib.gesmc_run(None, None, None, None, 0, 0, 0, 0, 0, 0, 0, None, None) == gesmc.E_INVAL
    assert b"null" in lib.gesmc_last_error()

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
    for name, val in re.findall(r"#define\s+(GESMC_[A-Z0-9_]+)\s+\(?(-?\d+)\)?", header_text()):
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
    for name in ["E_INVAL", "E_NOT_SIMPLE", "E_RANGE", "E_NOMEM", "E_DEVICE", "E_AGAIN", "E_CANCELED", "E_INTERNAL"]:
        assert d["GESMC_" + name] == getattr(gesmc, name), name
    for name in ["BUCKET_AVG", "SORT_CAP", "FAST_ROUNDS", "PROFILE", "STRATEGY", "PERSIST", "PROFILE_ONLY", "LEVEL1_BITS", "FUSE_EMIT", "GRAPH", "SMALL_GRAPHS", "PACK_TUPLES", "ROUND_LIMIT", "UNPERMUTE_BUCKETS", "TUNE_CACHE"]:
        assert d["GESMC_OPT_" + name] == getattr(gesmc, "OPT_" + name), name


C_LAYOUT_PROBE = r"""
#include <stddef.h>
#include <stdio.h>
#include "gesmc.h"
#define F(T, f) printf("%s.%s %zu %zu\n", #T, #f, offsetof(T, f), sizeof(((T *)0)->f));
#define S(T) printf("%s %zu\n", #T, sizeof(T));
int main(void) {
    S(gesmc_stats) F(gesmc_stats, rounds_max) F(gesmc_stats, ms_device) F(gesmc_stats, tuple_bytes)
    S(gesmc_step_stats)
    S(gesmc_server_cfg) F(gesmc_server_cfg, max_graphs) F(gesmc_server_cfg, max_queue)
    S(gesmc_request) F(gesmc_request, m) F(gesmc_request, n) F(gesmc_request, t0) F(gesmc_request, r)
    F(gesmc_request, pl) F(gesmc_request, seed)
    S(gesmc_result) F(gesmc_result, m) F(gesmc_result, edges) F(gesmc_result, stats) F(gesmc_result, t_submit)
    F(gesmc_result, t_done)
    S(gesmc_server_info) F(gesmc_server_info, resident_edges) F(gesmc_server_info, queued)
    F(gesmc_server_info, resident) F(gesmc_server_info, busy_s) F(gesmc_server_info, now_s) F(gesmc_server_info, copy_s) F(gesmc_server_info, wait_s)
    S(gesmc_tuning) F(gesmc_tuning, fuse_emit) F(gesmc_tuning, candidates) F(gesmc_tuning, best_ms)
    F(gesmc_tuning, default_ms)
    return 0;
}
"""


def test_ctypes_layouts_match_c_compiler(tmp_path):
    """Every struct of the header, laid out by the C compiler, against the
    binding's ctypes mirror (sizes and field offsets)."""
    from paper_2111_03005_amd import _binding as b
    src = tmp_path / "probe.c"
    src.write_text(C_LAYOUT_PROBE)
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    mirror = {"gesmc_stats": b.Stats, "gesmc_step_stats": b.StepStats, "gesmc_server_cfg": b.ServerCfg,
              "gesmc_request": b.Request, "gesmc_result": b.Result, "gesmc_server_info": b.ServerInfo,
              "gesmc_tuning": b.Tuning}
    checked = 0
    for line in filter(None, out):
        parts = line.split()
        if "." in parts[0]:
            sname, field = parts[0].split(".")
            off, size = int(parts[1]), int(parts[2])
            f = getattr(mirror[sname], field)
            assert (f.offset, f.size) == (off, size), (sname, field)
        else:
            assert ctypes.sizeof(mirror[parts[0]]) == int(parts[1]), parts[0]
        checked += 1
    assert checked >= 20


def test_struct_layouts_match_header():
    from paper_2111_03005_amd import _binding as b
    # gesmc_stats: 6 x u64, 2 x u32, 1 x double, 2 x u32; gesmc_step_stats: 8 x u64
    assert ctypes.sizeof(b.Stats) == 6 * 8 + 2 * 4 + 8 + 2 * 4
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
    assert lib.gesmc_run_host(None, None, None, 0, 0, 0, 0, 0, 0, 0, None) == gesmc.E_INVAL
    assert b"null" in lib.gesmc_last_error()
    assert lib.gesmc_run_batch(None, None, 1, None, None, None, None, None, None, None, 0, 0, None,
                               None) == gesmc.E_INVAL
    assert lib.gesmc_server_create(None, None, None) == gesmc.E_INVAL
    assert lib.gesmc_submit(None, None, None) == gesmc.E_INVAL
    assert lib.gesmc_poll(None, 1, None) == gesmc.E_INVAL
    assert lib.gesmc_cancel(None, 1) == gesmc.E_INVAL
    lib.gesmc_server_destroy(None)
    lib.gesmc_result_free(None)
    assert lib.gesmc_autotune(None, None, None, 0, 0, 0, 1, None) == gesmc.E_INVAL
    assert lib.gesmc_autotune_batch(None, None, 0, None, None, None, None, 1, None) == gesmc.E_INVAL


def test_tune_cache_file_round_trip_without_gpu(lib, tmp_path):
    """The autotuner's cache: a file in the saved form loads, saves back to
    the same entries, a malformed file is rejected with the cache unchanged,
    and clear empties it.  No device is needed."""
    import json

    import paper_2111_03005_amd as gesmc
    gesmc.tune_cache_clear()
    assert gesmc.tune_cache_size() == 0
    entries = [
        {"key": "gfx950:0000:05:00|plain|26|22|0", "bucket_avg": 768, "level1_bits": 0, "fuse_emit": 1,
         "candidates": 8, "best_ms": 47.5, "default_ms": 47.9},
        {"key": "gfx950:0000:05:00|batch|27|16|12", "bucket_avg": 512, "level1_bits": 8, "fuse_emit": 0,
         "candidates": 8, "best_ms": 210.25, "default_ms": 215.5},
    ]
    src = tmp_path / "in.json"
    src.write_text("[\n" + ",\n".join(json.dumps(e) for e in entries) + "\n]\n")
    gesmc.tune_cache_load(str(src))
    assert gesmc.tune_cache_size() == 2
    dst = tmp_path / "out.json"
    gesmc.tune_cache_save(str(dst))
    back = sorted(json.loads(dst.read_text()), key=lambda e: e["key"])
    assert back == sorted(entries, key=lambda e: e["key"])
    bad = tmp_path / "bad.json"
    bad.write_text('[\n{"key": "x", "bucket_avg": 5000, "level1_bits": 0, "fuse_emit": 1, "candidates": 8, '
                   '"best_ms": 1.0, "default_ms": 1.0}\n]\n')
    with pytest.raises(gesmc.GesmcError):
        gesmc.tune_cache_load(str(bad))
    with pytest.raises(gesmc.GesmcError):
        gesmc.tune_cache_load(str(tmp_path / "missing.json"))
    assert gesmc.tune_cache_size() == 2
    gesmc.tune_cache_clear()
    assert gesmc.tune_cache_size() == 0

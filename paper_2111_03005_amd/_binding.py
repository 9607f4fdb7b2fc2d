"""ctypes binding of libgesmc.so (include/gesmc.h): argument marshalling only.

Every step of the global switch runs in the HIP kernels of the library; this
module passes device pointers, sizes and the current HIP stream.  If the
library is missing the import of a function raises -- there is no CPU path.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgesmc.so")

OK = 0
E_INVAL, E_NOT_SIMPLE, E_RANGE, E_NOMEM, E_DEVICE, E_AGAIN, E_CANCELED, E_INTERNAL = -1, -2, -3, -4, -5, -6, -7, -9
E_ROUNDS = -8
E_NOT_GRAPHICAL = -10
OPT_BUCKET_AVG, OPT_SORT_CAP, OPT_FAST_ROUNDS, OPT_PROFILE, OPT_STRATEGY, OPT_PERSIST, OPT_PROFILE_ONLY = (
    1, 2, 3, 4, 5, 6, 7)
OPT_LEVEL1_BITS = 8
OPT_FUSE_EMIT = 9
OPT_GRAPH = 10
OPT_SMALL_GRAPHS = 11
OPT_PACK_TUPLES = 12
OPT_ROUND_LIMIT = 13
OPT_UNPERMUTE_BUCKETS = 14
OPT_TUNE_CACHE = 15
CHAIN_GLOBAL, CHAIN_ES = 0, 1
CLASS_LOOPS, CLASS_MULTI, CLASS_DIRECTED = 1, 2, 4
NOALLOC_MAX_EDGES = 2000000
STRATEGY_SORTED_TUPLES, STRATEGY_HBM_TABLE = 0, 1


class GesmcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("gesmc status %d: %s" % (status, msg))
        self.status = status


class Stats(ctypes.Structure):
    _fields_ = [("attempts", ctypes.c_uint64), ("legal", ctypes.c_uint64), ("rej_loop", ctypes.c_uint64),
                ("rej_exists", ctypes.c_uint64), ("rej_pl", ctypes.c_uint64), ("rounds_sum", ctypes.c_uint64),
                ("rounds_max", ctypes.c_uint32), ("supersteps", ctypes.c_uint32), ("ms_device", ctypes.c_double),
                ("tuple_bytes", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]

    def as_dict(self):
        return {f: (float(getattr(self, f)) if f == "ms_device" else int(getattr(self, f))) for f, _ in self._fields_}


class StepStats(ctypes.Structure):
    _fields_ = [("attempts", ctypes.c_uint64), ("legal", ctypes.c_uint64), ("rej_loop", ctypes.c_uint64),
                ("rej_exists", ctypes.c_uint64), ("rej_pl", ctypes.c_uint64), ("rounds", ctypes.c_uint64),
                ("undecided_after_round1", ctypes.c_uint64), ("fallback_buckets", ctypes.c_uint64)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class Tuning(ctypes.Structure):
    _fields_ = [("bucket_avg", ctypes.c_uint32), ("level1_bits", ctypes.c_uint32), ("fuse_emit", ctypes.c_uint32),
                ("candidates", ctypes.c_uint32), ("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class EsStats(ctypes.Structure):
    _fields_ = [("attempts", ctypes.c_uint64), ("legal", ctypes.c_uint64), ("rej_loop", ctypes.c_uint64),
                ("rej_exists", ctypes.c_uint64), ("supersteps", ctypes.c_uint64), ("rounds_sum", ctypes.c_uint64),
                ("rounds_max", ctypes.c_uint32), ("epochs", ctypes.c_uint32), ("ms_device", ctypes.c_double)]

    def as_dict(self):
        return {f: (float(getattr(self, f)) if f == "ms_device" else int(getattr(self, f))) for f, _ in self._fields_}


class MixingResult(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("transitions", ctypes.c_uint32), ("tracked", ctypes.c_uint64),
                ("non_independent", ctypes.c_uint64), ("n00", ctypes.c_uint64), ("n01", ctypes.c_uint64),
                ("n10", ctypes.c_uint64), ("n11", ctypes.c_uint64)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class ServerCfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_graphs", ctypes.c_uint32),
                ("max_queue", ctypes.c_uint32)]


class Request(ctypes.Structure):
    _fields_ = [("edges", ctypes.c_void_p), ("m", ctypes.c_uint64), ("n", ctypes.c_uint32), ("t0", ctypes.c_uint32),
                ("r", ctypes.c_uint32), ("pl", ctypes.c_uint32), ("seed", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("m", ctypes.c_uint64), ("edges", ctypes.POINTER(ctypes.c_uint64)),
                ("stats", Stats), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class ServerInfo(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("iterations", ctypes.c_uint64),
                ("attempts", ctypes.c_uint64), ("legal", ctypes.c_uint64), ("resident_edges", ctypes.c_uint64),
                ("queued", ctypes.c_uint32), ("resident", ctypes.c_uint32), ("busy_s", ctypes.c_double),
                ("now_s", ctypes.c_double), ("copy_s", ctypes.c_double), ("wait_s", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


EXPORTS = ["gesmc_create", "gesmc_destroy", "gesmc_last_error", "gesmc_run", "gesmc_run_noalloc", "gesmc_run_host",
           "gesmc_run_batch",
           "gesmc_superstep_outcomes", "gesmc_perm_keys", "gesmc_permutation", "gesmc_set_option",
           "gesmc_kernel_count", "gesmc_kernel_name", "gesmc_profile_get", "gesmc_profile_reset",
           "gesmc_server_create", "gesmc_server_destroy", "gesmc_submit", "gesmc_poll", "gesmc_wait",
           "gesmc_cancel", "gesmc_result_free", "gesmc_server_info_get", "gesmc_autotune", "gesmc_autotune_batch",
           "gesmc_run_es", "gesmc_es_draws", "gesmc_mixing", "gesmc_run_class", "gesmc_gen_gnp",
           "gesmc_gen_pld_degrees", "gesmc_gen_havel_hakimi", "gesmc_gen_relabel", "gesmc_set_allocator",
           "gesmc_tune_cache_save", "gesmc_tune_cache_load", "gesmc_tune_cache_clear", "gesmc_tune_cache_size"]

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_lib = None
_lock = threading.Lock()


def load_library(path: str = LIB_PATH):
    """Loads libgesmc.so; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError("libgesmc.so not built (run __graft_entry__.build() or "
                               "python -m paper_2111_03005_amd.build): %s" % path)
        lib = ctypes.CDLL(path)
        vp, u32, u64, i32, i64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64
        lib.gesmc_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
        lib.gesmc_create.restype = i32
        lib.gesmc_destroy.argtypes = [vp]
        lib.gesmc_destroy.restype = None
        lib.gesmc_last_error.argtypes = []
        lib.gesmc_last_error.restype = ctypes.c_char_p
        lib.gesmc_run.argtypes = [vp, vp, vp, vp, u64, u32, u64, u32, u32, u32, u32, ctypes.POINTER(Stats),
                                  ctypes.POINTER(StepStats)]
        lib.gesmc_run.restype = i32
        lib.gesmc_run_noalloc.argtypes = [vp, vp, vp, vp, u64, u32, u64, u32, u32, u32, u32, ctypes.POINTER(Stats)]
        lib.gesmc_run_noalloc.restype = i32
        lib.gesmc_run_host.argtypes = [vp, vp, vp, u64, u32, u64, u32, u32, u32, u32, ctypes.POINTER(Stats)]
        lib.gesmc_run_host.restype = i32
        lib.gesmc_run_batch.argtypes = [vp, vp, u32, vp, vp, ctypes.POINTER(u64), ctypes.POINTER(u32),
                                        ctypes.POINTER(u64), ctypes.POINTER(u32), ctypes.POINTER(u32), u32, u32,
                                        ctypes.POINTER(Stats), ctypes.POINTER(Stats)]
        lib.gesmc_run_batch.restype = i32
        lib.gesmc_superstep_outcomes.argtypes = [vp, vp, vp, vp, u64, u32, u64, u32, u32, vp,
                                                 ctypes.POINTER(StepStats)]
        lib.gesmc_superstep_outcomes.restype = i32
        lib.gesmc_perm_keys.argtypes = [vp, vp, u64, u64, u32, vp]
        lib.gesmc_perm_keys.restype = i32
        lib.gesmc_permutation.argtypes = [vp, vp, u64, u64, u32, vp]
        lib.gesmc_permutation.restype = i32
        lib.gesmc_set_option.argtypes = [vp, ctypes.c_int, i64]
        lib.gesmc_set_option.restype = i32
        lib.gesmc_kernel_count.argtypes = []
        lib.gesmc_kernel_count.restype = ctypes.c_int
        lib.gesmc_kernel_name.argtypes = [ctypes.c_int]
        lib.gesmc_kernel_name.restype = ctypes.c_char_p
        lib.gesmc_profile_get.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(u64),
                                          ctypes.POINTER(u64)]
        lib.gesmc_profile_get.restype = i32
        lib.gesmc_profile_reset.argtypes = [vp]
        lib.gesmc_profile_reset.restype = i32
        lib.gesmc_server_create.argtypes = [vp, ctypes.POINTER(ServerCfg), ctypes.POINTER(vp)]
        lib.gesmc_server_create.restype = i32
        lib.gesmc_server_destroy.argtypes = [vp]
        lib.gesmc_server_destroy.restype = None
        lib.gesmc_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(u64)]
        lib.gesmc_submit.restype = i32
        for f in (lib.gesmc_poll, lib.gesmc_wait):
            f.argtypes = [vp, u64, ctypes.POINTER(Result)]
            f.restype = i32
        lib.gesmc_cancel.argtypes = [vp, u64]
        lib.gesmc_cancel.restype = i32
        lib.gesmc_result_free.argtypes = [ctypes.POINTER(Result)]
        lib.gesmc_result_free.restype = None
        lib.gesmc_server_info_get.argtypes = [vp, ctypes.POINTER(ServerInfo)]
        lib.gesmc_server_info_get.restype = i32
        lib.gesmc_autotune.argtypes = [vp, vp, vp, u64, u32, u64, u32, ctypes.POINTER(Tuning)]
        lib.gesmc_autotune.restype = i32
        lib.gesmc_autotune_batch.argtypes = [vp, vp, u32, vp, ctypes.POINTER(u64), ctypes.POINTER(u32),
                                             ctypes.POINTER(u64), u32, ctypes.POINTER(Tuning)]
        lib.gesmc_autotune_batch.restype = i32
        lib.gesmc_run_es.argtypes = [vp, vp, vp, vp, u64, u32, u64, u64, u64, u32, vp, ctypes.POINTER(EsStats)]
        lib.gesmc_run_es.restype = i32
        lib.gesmc_es_draws.argtypes = [vp, vp, u64, u64, u64, u64, vp, vp, vp]
        lib.gesmc_es_draws.restype = i32
        lib.gesmc_mixing.argtypes = [vp, vp, vp, u64, u32, u64, u32, u32, u32, ctypes.POINTER(u32), u32,
                                     ctypes.POINTER(MixingResult), ctypes.POINTER(ctypes.c_double)]
        lib.gesmc_mixing.restype = i32
        lib.gesmc_run_class.argtypes = [vp, vp, vp, vp, u64, u32, u64, u32, u32, u32, u32, ctypes.POINTER(Stats),
                                        ctypes.POINTER(StepStats), vp]
        lib.gesmc_run_class.restype = i32
        f64 = ctypes.c_double
        lib.gesmc_gen_gnp.argtypes = [vp, vp, u32, f64, u64, vp, u64, ctypes.POINTER(u64)]
        lib.gesmc_gen_gnp.restype = i32
        lib.gesmc_gen_pld_degrees.argtypes = [vp, vp, u32, f64, u32, u32, u64, vp, ctypes.POINTER(u64)]
        lib.gesmc_gen_pld_degrees.restype = i32
        lib.gesmc_gen_havel_hakimi.argtypes = [vp, vp, u32, vp, vp, u64, ctypes.POINTER(u64)]
        lib.gesmc_gen_havel_hakimi.restype = i32
        lib.gesmc_gen_relabel.argtypes = [vp, vp, vp, u64, u32, u64]
        lib.gesmc_gen_relabel.restype = i32
        lib.gesmc_set_allocator.argtypes = [vp, ALLOC_FN, FREE_FN, vp]
        lib.gesmc_set_allocator.restype = i32
        lib.gesmc_tune_cache_save.argtypes = [ctypes.c_char_p]
        lib.gesmc_tune_cache_save.restype = i32
        lib.gesmc_tune_cache_load.argtypes = [ctypes.c_char_p]
        lib.gesmc_tune_cache_load.restype = i32
        lib.gesmc_tune_cache_clear.argtypes = []
        lib.gesmc_tune_cache_clear.restype = None
        lib.gesmc_tune_cache_size.argtypes = []
        lib.gesmc_tune_cache_size.restype = u32
        _lib = lib
        return lib


def _check(status: int):
    if status != OK:
        raise GesmcError(status, _lib.gesmc_last_error().decode(errors="replace"))


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t: torch.Tensor, dtype_bytes: int, numel: int, name: str):
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous() or t.element_size() != dtype_bytes or t.numel() < numel:
        raise ValueError("%s: need a contiguous %d-byte tensor with >= %d elements" % (name, dtype_bytes, numel))
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """A libgesmc context on one HIP device (device memory is kept between calls)."""

    def __init__(self, device: int | None = None):
        lib = load_library()
        if device is None:
            device = torch.cuda.current_device()
        self.device = device
        h = ctypes.c_void_p()
        _check(lib.gesmc_create(device, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.gesmc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, option: int, value: int):
        _check(_lib.gesmc_set_option(self._h, option, int(value)))

    def set_allocator(self, alloc=None, free=None):
        """gesmc_set_allocator: alloc(nbytes) -> device address (int, 0 = none)
        and free(address) for the context's device buffers; both None restores
        hipMalloc.  The Python callables are kept alive by the context."""
        if (alloc is None) != (free is None):
            raise ValueError("give both alloc and free, or neither")
        if alloc is None:
            _check(_lib.gesmc_set_allocator(self._h, ALLOC_FN(), FREE_FN(), None))
            self._alloc_cbs = None
            return
        a = ALLOC_FN(lambda nbytes, user: int(alloc(int(nbytes))) or None)
        f = FREE_FN(lambda ptr, user: free(int(ptr)))
        _check(_lib.gesmc_set_allocator(self._h, a, f, None))
        # buffers made by earlier pairs still hold their functions: keep them all
        self._alloc_keep = getattr(self, "_alloc_keep", []) + [(a, f)]
        self._alloc_cbs = (a, f)

    def use_torch_allocator(self):
        """Backs the context's device buffers with PyTorch's caching allocator."""
        dev = self.device
        self.set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n, device=dev),
                           lambda p: torch.cuda.caching_allocator_delete(p))

    # ---- the global switch chain -----------------------------------------
    def run(self, edges: torch.Tensor, n: int, seed: int, t0: int = 0, r: int = 1, pl: int = 0,
            out: torch.Tensor | None = None, stream=None, steps: bool = False):
        """r global switches on `edges` (device uint64/int64 keys).  Returns (out, stats[, step list])."""
        m = edges.numel()
        if out is None:
            out = torch.empty_like(edges)
        st = Stats()
        ss = (StepStats * max(r, 1))() if steps else None
        _check(_lib.gesmc_run(self._h, _stream_ptr(stream), _dev_ptr(edges, 8, m, "edges"),
                              _dev_ptr(out, 8, m, "out"), m, n, seed & (2**64 - 1), t0, r, pl, 0,
                              ctypes.byref(st), ss))
        if steps:
            return out, st.as_dict(), [ss[q].as_dict() for q in range(r)]
        return out, st.as_dict()

    def run_class(self, edges: torch.Tensor, n: int, seed: int, cls: int, t0: int = 0, r: int = 1, pl: int = 0,
                  out: torch.Tensor | None = None, stream=None, steps: bool = False, outcomes: bool = False):
        """gesmc_run_class: r global switches of graph class `cls` (CLASS_* bits).
        Returns (out, stats, step list or None, last superstep's outcome codes or None)."""
        m = edges.numel()
        if out is None:
            out = torch.empty_like(edges)
        st = Stats()
        ss = (StepStats * max(r, 1))() if steps else None
        oc = torch.zeros(max(m // 2, 1), dtype=torch.uint8, device=edges.device) if outcomes else None
        _check(_lib.gesmc_run_class(self._h, _stream_ptr(stream), _dev_ptr(edges, 8, m, "edges"),
                                    _dev_ptr(out, 8, m, "out"), m, n, seed & (2**64 - 1), t0, r, pl, cls,
                                    ctypes.byref(st), ss, None if oc is None else ctypes.c_void_p(oc.data_ptr())))
        return (out, st.as_dict(), [ss[q].as_dict() for q in range(r)] if steps else None,
                oc[: m // 2] if outcomes else None)

    # ---- input realisation ------------------------------------------------
    def gen_gnp(self, n: int, p: float, seed: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """G(n,p) on the device (gesmc_gen_gnp) into `out` (int64, its size the
        capacity), or into a new tensor sized by a count call first."""
        m = ctypes.c_uint64(0)
        if out is None:
            _check(_lib.gesmc_gen_gnp(self._h, _stream_ptr(stream), n, float(p), seed & (2**64 - 1), None, 0,
                                      ctypes.byref(m)))
            out = torch.empty(max(m.value, 1), dtype=torch.int64, device="cuda:%d" % self.device)
            m.value = out.numel() if m.value else 0
        else:
            m.value = out.numel()
            _dev_ptr(out, 8, 0, "out")
        _check(_lib.gesmc_gen_gnp(self._h, _stream_ptr(stream), n, float(p), seed & (2**64 - 1),
                                  ctypes.c_void_p(out.data_ptr()), m.value, ctypes.byref(m)))
        return out[: m.value]

    def gen_pld_degrees(self, n: int, gamma: float, dmin: int, dmax: int, seed: int, stream=None):
        """Pld([dmin..dmax], gamma) degrees on the device -> (uint32-valued int32 tensor, sum)."""
        deg = torch.empty(max(n, 1), dtype=torch.int32, device="cuda:%d" % self.device)
        s = ctypes.c_uint64(0)
        _check(_lib.gesmc_gen_pld_degrees(self._h, _stream_ptr(stream), n, float(gamma), dmin, dmax,
                                          seed & (2**64 - 1), ctypes.c_void_p(deg.data_ptr()), ctypes.byref(s)))
        return deg[:n], s.value

    def gen_havel_hakimi(self, deg: torch.Tensor, stream=None) -> torch.Tensor:
        """Havel-Hakimi realisation of a device degree sequence (4-byte ints)."""
        n = deg.numel()
        dp = _dev_ptr(deg, 4, n, "deg")
        m = ctypes.c_uint64(0)
        _check(_lib.gesmc_gen_havel_hakimi(self._h, _stream_ptr(stream), n, dp, None, 0, ctypes.byref(m)))
        out = torch.empty(max(m.value, 1), dtype=torch.int64, device=deg.device)
        _check(_lib.gesmc_gen_havel_hakimi(self._h, _stream_ptr(stream), n, dp, ctypes.c_void_p(out.data_ptr()),
                                           m.value, ctypes.byref(m)))
        return out[: m.value]

    def gen_relabel(self, edges: torch.Tensor, n: int, seed: int, stream=None) -> torch.Tensor:
        """Relabels the vertices of `edges` in place (gesmc_gen_relabel); returns it."""
        m = edges.numel()
        _check(_lib.gesmc_gen_relabel(self._h, _stream_ptr(stream), _dev_ptr(edges, 8, m, "edges") if m else None,
                                      m, n, seed & (2**64 - 1)))
        return edges

    def gen_powerlaw_graph(self, n: int, gamma: float, dmin: int, dmax: int, seed: int, stream=None):
        """Degrees, Havel-Hakimi and relabelling, all on the device: the SynPld input."""
        deg, _ = self.gen_pld_degrees(n, gamma, dmin, dmax, seed, stream)
        E = self.gen_havel_hakimi(deg, stream)
        return self.gen_relabel(E, n, seed, stream)

    def run_noalloc(self, edges: torch.Tensor, n: int, seed: int, t0: int = 0, r: int = 1, pl: int = 0,
                    out: torch.Tensor | None = None, stream=None):
        """gesmc_run_noalloc: as run, with the library's fixed device array as
        its only scratch (no allocation inside the call).  Returns (out, stats)."""
        m = edges.numel()
        if out is None:
            out = torch.empty_like(edges)
        st = Stats()
        _check(_lib.gesmc_run_noalloc(self._h, _stream_ptr(stream), _dev_ptr(edges, 8, m, "edges"),
                                      _dev_ptr(out, 8, m, "out"), m, n, seed & (2**64 - 1), t0, r, pl, 0,
                                      ctypes.byref(st)))
        return out, st.as_dict()

    def run_host(self, uv, n: int, seed: int, t0: int = 0, r: int = 1, pl: int = 0):
        """gesmc_run_host: edges as host vertex-id pairs (numpy, shape (m, 2) or 2m flat,
        any orientation) -> (result as an (m, 2) uint32 array of (min, max) pairs, stats)."""
        import numpy as np
        a = np.ascontiguousarray(uv, dtype=np.uint32).reshape(-1)
        if a.size % 2:
            raise ValueError("uv must hold an even number of vertex ids")
        m = a.size // 2
        out = np.empty(2 * m, dtype=np.uint32)
        st = Stats()
        _check(_lib.gesmc_run_host(self._h, a.ctypes.data if m else None, out.ctypes.data if m else None, m, n,
                                   seed & (2**64 - 1), t0, r, pl, 0, ctypes.byref(st)))
        return out.reshape(m, 2), st.as_dict()

    def run_batch(self, edges: torch.Tensor, offsets, n, seed, r, t0=None, pl: int = 0,
                  out: torch.Tensor | None = None, stream=None, stats: bool = True):
        """G graphs in one call: graph g is edges[offsets[g]:offsets[g+1]] (device
        uint64/int64 keys, local ids < n[g]).  Returns (out, per-graph stats or
        None, total stats)."""
        G = len(offsets) - 1
        if not (len(n) == len(seed) == len(r) == G) or (t0 is not None and len(t0) != G):
            raise ValueError("per-graph arrays need G = len(offsets) - 1 entries")
        total_m = int(offsets[-1])
        if out is None:
            out = torch.empty_like(edges)
        h_off = (ctypes.c_uint64 * (G + 1))(*[int(x) for x in offsets])
        h_n = (ctypes.c_uint32 * G)(*[int(x) for x in n])
        h_seed = (ctypes.c_uint64 * G)(*[int(x) & (2**64 - 1) for x in seed])
        h_r = (ctypes.c_uint32 * G)(*[int(x) for x in r])
        h_t0 = (ctypes.c_uint32 * G)(*[int(x) for x in t0]) if t0 is not None else None
        st = (Stats * G)() if stats else None
        tot = Stats()
        _check(_lib.gesmc_run_batch(self._h, _stream_ptr(stream), G, _dev_ptr(edges, 8, total_m, "edges"),
                                    _dev_ptr(out, 8, total_m, "out"), h_off, h_n, h_seed, h_t0, h_r, pl, 0,
                                    st, ctypes.byref(tot)))
        return out, ([st[g].as_dict() for g in range(G)] if stats else None), tot.as_dict()

    def autotune(self, edges: torch.Tensor, n: int, seed: int = 1, supersteps: int = 2, stream=None):
        """Times candidate option settings on these edges and keeps the fastest."""
        tu = Tuning()
        _check(_lib.gesmc_autotune(self._h, _stream_ptr(stream), _dev_ptr(edges, 8, edges.numel(), "edges"),
                                   edges.numel(), n, seed & (2**64 - 1), supersteps, ctypes.byref(tu)))
        return tu.as_dict()

    def autotune_batch(self, edges: torch.Tensor, offsets, n, seed, supersteps: int = 2, stream=None):
        """The autotuner over a batch (arguments as run_batch)."""
        G = len(offsets) - 1
        h_off = (ctypes.c_uint64 * (G + 1))(*[int(x) for x in offsets])
        h_n = (ctypes.c_uint32 * G)(*[int(x) for x in n])
        h_seed = (ctypes.c_uint64 * G)(*[int(x) & (2**64 - 1) for x in seed])
        tu = Tuning()
        _check(_lib.gesmc_autotune_batch(self._h, _stream_ptr(stream), G,
                                         _dev_ptr(edges, 8, int(offsets[-1]), "edges"), h_off, h_n, h_seed,
                                         supersteps, ctypes.byref(tu)))
        return tu.as_dict()

    def superstep_outcomes(self, edges: torch.Tensor, n: int, seed: int, t: int, pl: int = 0, stream=None):
        """One superstep; returns (edges after, outcome code per switch (uint8), step stats)."""
        m = edges.numel()
        out = torch.empty_like(edges)
        oc = torch.empty(max(m // 2, 1), dtype=torch.uint8, device=edges.device)
        ss = StepStats()
        _check(_lib.gesmc_superstep_outcomes(self._h, _stream_ptr(stream), _dev_ptr(edges, 8, m, "edges"),
                                             _dev_ptr(out, 8, m, "out"), m, n, seed & (2**64 - 1), t, pl,
                                             ctypes.c_void_p(oc.data_ptr()), ctypes.byref(ss)))
        return out, oc[: m // 2], ss.as_dict()

    # ---- ParES: the ES-MC chain (Alg. 2) --------------------------------
    def run_es(self, edges: torch.Tensor, n: int, seed: int, k0: int = 0, r: int = 1, out: torch.Tensor | None = None,
               stream=None, outcomes: bool = False):
        """r ES-MC switches (counters k0 .. k0+r-1) on `edges` (device uint64/int64
        keys).  Returns (out, stats[, per-switch outcome codes (uint8 device tensor)])."""
        m = edges.numel()
        if out is None:
            out = torch.empty_like(edges)
        oc = torch.empty(max(r, 1), dtype=torch.uint8, device=edges.device) if outcomes else None
        st = EsStats()
        _check(_lib.gesmc_run_es(self._h, _stream_ptr(stream), _dev_ptr(edges, 8, m, "edges"),
                                 _dev_ptr(out, 8, m, "out"), m, n, seed & (2**64 - 1), k0, r, 0,
                                 ctypes.c_void_p(oc.data_ptr()) if outcomes else None, ctypes.byref(st)))
        if outcomes:
            return out, st.as_dict(), oc[:r]
        return out, st.as_dict()

    def es_draws(self, m: int, seed: int, k0: int, count: int, stream=None, device=None):
        """The (i, j, g) draws of ES-MC switches k0 .. k0+count-1 on m edges (device tensors)."""
        dev = device or torch.device("cuda", self.device)
        di = torch.empty(max(count, 1), dtype=torch.int64, device=dev)
        dj = torch.empty(max(count, 1), dtype=torch.int64, device=dev)
        dg = torch.empty(max(count, 1), dtype=torch.uint8, device=dev)
        _check(_lib.gesmc_es_draws(self._h, _stream_ptr(stream), m, seed & (2**64 - 1), k0, count,
                                   ctypes.c_void_p(di.data_ptr()), ctypes.c_void_p(dj.data_ptr()),
                                   ctypes.c_void_p(dg.data_ptr())))
        return di[:count], dj[:count], dg[:count]

    # ---- mixing diagnostic (Sec. 6.1) -------------------------------------
    def mixing(self, edges: torch.Tensor, n: int, seed: int, K: int, thin, chain: int = 0, pl: int = 0,
               stream=None):
        """Autocorrelation diagnostic of K supersteps of G-ES-MC (chain 0) or ES-MC
        (chain 1) from `edges` (device keys, unchanged).  Returns (list of per-k
        dicts, wall ms of the chain and its sampling)."""
        m = edges.numel()
        th = (ctypes.c_uint32 * len(thin))(*[int(x) for x in thin])
        res = (MixingResult * len(thin))()
        ms = ctypes.c_double()
        _check(_lib.gesmc_mixing(self._h, _stream_ptr(stream), _dev_ptr(edges, 8, m, "edges") if m else None, m, n,
                                 seed & (2**64 - 1), chain, pl, K, th, len(thin), res, ctypes.byref(ms)))
        return [res[q].as_dict() for q in range(len(thin))], ms.value

    def perm_keys(self, m: int, seed: int, t: int, stream=None, device=None):
        out = torch.empty(max(m, 1), dtype=torch.int64, device=device or torch.device("cuda", self.device))
        _check(_lib.gesmc_perm_keys(self._h, _stream_ptr(stream), m, seed & (2**64 - 1), t,
                                    ctypes.c_void_p(out.data_ptr())))
        return out[:m]

    def permutation(self, m: int, seed: int, t: int, stream=None, device=None):
        out = torch.empty(max(m, 1), dtype=torch.int32, device=device or torch.device("cuda", self.device))
        _check(_lib.gesmc_permutation(self._h, _stream_ptr(stream), m, seed & (2**64 - 1), t,
                                      ctypes.c_void_p(out.data_ptr())))
        return out[:m]

    # ---- kernel timing ---------------------------------------------------
    @staticmethod
    def kernel_names():
        """Kernel names by kernel id."""
        return [_lib.gesmc_kernel_name(k).decode() for k in range(_lib.gesmc_kernel_count())]

    def profile(self):
        """{kernel name: (total ms, launches, items)} of launches timed while OPT_PROFILE was on."""
        res = {}
        for kid in range(_lib.gesmc_kernel_count()):
            ms = ctypes.c_double()
            nl = ctypes.c_uint64()
            it = ctypes.c_uint64()
            _check(_lib.gesmc_profile_get(self._h, kid, ctypes.byref(ms), ctypes.byref(nl), ctypes.byref(it)))
            if nl.value:
                res[_lib.gesmc_kernel_name(kid).decode()] = (ms.value, nl.value, it.value)
        return res

    def profile_reset(self):
        _check(_lib.gesmc_profile_reset(self._h))


class Server:
    """Request loop with continuous batching on one context (gesmc_server_*).
    Requests carry host edge arrays; results come back as host arrays."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int = 0, max_graphs: int = 0, max_queue: int = 0):
        self.ctx = ctx
        cfg = ServerCfg(hbm_budget_bytes, max_graphs, max_queue)
        h = ctypes.c_void_p()
        _check(_lib.gesmc_server_create(ctx._h, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.gesmc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, edges, n: int, seed: int, r: int, t0: int = 0, pl: int = 0) -> int:
        """Queues a request (edges: numpy uint64 keys, copied).  Raises GesmcError
        (status E_AGAIN when the queue is full)."""
        import numpy as np
        e = np.ascontiguousarray(edges, dtype=np.uint64)
        req = Request(e.ctypes.data if e.size else None, e.size, n, t0, r, pl, seed & (2**64 - 1))
        t = ctypes.c_uint64()
        _check(_lib.gesmc_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        return t.value

    @staticmethod
    def _take(res: Result):
        import numpy as np
        edges = None
        if res.status == OK:
            edges = np.ctypeslib.as_array(res.edges, shape=(max(res.m, 1),))[: res.m].copy()
            _lib.gesmc_result_free(ctypes.byref(res))
        return {"status": res.status, "edges": edges, "stats": res.stats.as_dict(), "t_submit": res.t_submit,
                "t_admit": res.t_admit, "t_done": res.t_done}

    def poll(self, ticket: int):
        """The result dict if the request is done, else None."""
        res = Result()
        st = _lib.gesmc_poll(self._h, ticket, ctypes.byref(res))
        if st == E_AGAIN:
            return None
        _check(st)
        return self._take(res)

    def wait(self, ticket: int):
        res = Result()
        _check(_lib.gesmc_wait(self._h, ticket, ctypes.byref(res)))
        return self._take(res)

    def cancel(self, ticket: int):
        _check(_lib.gesmc_cancel(self._h, ticket))

    def info(self):
        i = ServerInfo()
        _check(_lib.gesmc_server_info_get(self._h, ctypes.byref(i)))
        return i.as_dict()


_default = {}


def tune_cache_save(path: str) -> None:
    """Writes the autotuner's choices (per device and shape class) to a JSON file."""
    _check(load_library().gesmc_tune_cache_save(os.fsencode(path)))


def tune_cache_load(path: str) -> None:
    """Merges a file written by tune_cache_save into the autotuner's choices."""
    _check(load_library().gesmc_tune_cache_load(os.fsencode(path)))


def tune_cache_clear() -> None:
    load_library().gesmc_tune_cache_clear()


def tune_cache_size() -> int:
    return int(load_library().gesmc_tune_cache_size())


def default_context(device: int | None = None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def run(edges: torch.Tensor, n: int, seed: int, t0: int = 0, r: int = 1, pl: int = 0, out=None, stream=None):
    """r global switches with the default context of the tensor's device."""
    return default_context(edges.device.index).run(edges, n, seed, t0, r, pl, out, stream)

"""Seeded synthetic starting graphs shared by the HIP path's tests/bench and the oracle.

This module holds no part of the edge-switching method: it only builds graphs
(as packed 64-bit keys ``(min << 32) | max``, directed ``(tail << 32) | head``)
whose shape follows the paper's synthetic families (Sec. 6: SynGnp and
SynPld), graphs of the other classes Sec. 1 names, and the named workloads
used for parity tests and the benchmark.

The C source ``graphgen.c`` is compiled with gcc into ``libgraphgen.so`` next to
it (``build()``); loading compiles it if the library is missing.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build() -> str:
    """Compile graphgen.c into libgraphgen.so (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    u32, u64, i64, dbl = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_double
    vp = ctypes.c_void_p
    lib.gg_gnp.argtypes = [u32, dbl, u64, vp, i64]
    lib.gg_gnp.restype = i64
    lib.gg_powerlaw_degrees.argtypes = [u32, u32, u32, dbl, u64, vp]
    lib.gg_powerlaw_degrees.restype = i64
    lib.gg_havel_hakimi.argtypes = [u32, vp, vp]
    lib.gg_havel_hakimi.restype = i64
    lib.gg_shuffle_ids.argtypes = [u32, u64, vp, i64]
    lib.gg_shuffle_ids.restype = ctypes.c_int
    lib.gg_uniforms.argtypes = [u64, vp, i64]
    lib.gg_uniforms.restype = None
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def gnp(n: int, p: float, seed: int) -> np.ndarray:
    """G(n,p) edge keys (uint64), ordered by (larger id, smaller id)."""
    lib = _load()
    mean = p * n * (n - 1) / 2.0
    cap = int(mean + 10.0 * math.sqrt(mean + 1.0) + 1024)
    while True:
        out = np.empty(max(cap, 1), dtype=np.uint64)
        m = lib.gg_gnp(n, p, seed, _ptr(out), cap)
        if m >= 0:
            return out[:m].copy()
        cap = -m


def powerlaw_degrees(n: int, gamma: float, dmin: int, dmax: int, seed: int) -> np.ndarray:
    """i.i.d. Pld([dmin..dmax], gamma) degrees with an even sum (uint32)."""
    lib = _load()
    deg = np.empty(n, dtype=np.uint32)
    s = lib.gg_powerlaw_degrees(n, dmin, dmax, gamma, seed, _ptr(deg))
    if s < 0:
        raise ValueError("bad power-law parameters")
    return deg


def havel_hakimi(deg: np.ndarray) -> np.ndarray:
    """Deterministic Havel-Hakimi realisation; raises if not graphical."""
    lib = _load()
    deg = np.ascontiguousarray(deg, dtype=np.uint32)
    total = int(deg.sum(dtype=np.int64))
    out = np.empty(max(total // 2, 1), dtype=np.uint64)
    m = lib.gg_havel_hakimi(len(deg), _ptr(deg), _ptr(out))
    if m < 0:
        raise ValueError("degree sequence is not graphical")
    return out[:m].copy()


def shuffle_ids(edges: np.ndarray, n: int, seed: int) -> np.ndarray:
    """Relabel vertices by a seeded uniform permutation; keys re-packed (min, max)."""
    lib = _load()
    e = np.ascontiguousarray(edges, dtype=np.uint64).copy()
    if lib.gg_shuffle_ids(n, seed, _ptr(e), len(e)) != 0:
        raise MemoryError
    return e


def uniforms(seed: int, count: int) -> np.ndarray:
    lib = _load()
    out = np.empty(max(count, 1), dtype=np.float64)
    lib.gg_uniforms(seed, _ptr(out), count)
    return out[:count]


def powerlaw_graph(n: int, gamma: float, dmin: int, dmax: int, seed: int) -> np.ndarray:
    """Pld degrees -> Havel-Hakimi -> vertex-id shuffle.  If a draw is not
    graphical the degree seed is advanced deterministically and redrawn."""
    for attempt in range(64):
        deg = powerlaw_degrees(n, gamma, dmin, dmax, seed + 7919 * attempt)
        try:
            e = havel_hakimi(deg)
        except ValueError:
            continue
        return shuffle_ids(e, n, seed ^ 0x5DEECE66D)
    raise ValueError("no graphical draw in 64 attempts")


def split(keys: np.ndarray):
    """Packed keys -> (u, v) uint32 arrays with u < v."""
    k = np.asarray(keys, dtype=np.uint64)
    return (k >> np.uint64(32)).astype(np.uint32), (k & np.uint64(0xFFFFFFFF)).astype(np.uint32)


def pack(u, v) -> np.ndarray:
    u = np.asarray(u, dtype=np.uint64)
    v = np.asarray(v, dtype=np.uint64)
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    return (lo << np.uint64(32)) | hi


def degrees(keys: np.ndarray, n: int) -> np.ndarray:
    u, v = split(keys)
    return (np.bincount(u, minlength=n) + np.bincount(v, minlength=n)).astype(np.int64)


# ---------------------------------------------------------------------------
# Graphs of the other classes (directed, with loops, with multi-edges).  Keys:
# undirected (min << 32) | max, directed (tail << 32) | head.  cls bits:
# 1 loops allowed, 2 multi-edges allowed, 4 directed.
# ---------------------------------------------------------------------------

def class_graph(n: int, m: int, cls: int, seed: int) -> np.ndarray:
    """m edges with uniform endpoints on [0, n), in random order: a loop is
    redrawn unless the class allows loops, a repeated key unless it allows
    multi-edges."""
    loops, multi, directed = bool(cls & 1), bool(cls & 2), bool(cls & 4)
    cap = n * (n - 1) // (1 if directed else 2) + (n if loops else 0)
    if not multi and m > cap:
        raise ValueError("class %d on %d vertices holds at most %d edges" % (cls, n, cap))
    rng = np.random.default_rng(seed)
    have = np.zeros(0, dtype=np.uint64)
    while len(have) < m:
        want = m - len(have)
        a = rng.integers(0, n, 2 * want + 16, dtype=np.uint64)
        b = rng.integers(0, n, 2 * want + 16, dtype=np.uint64)
        if not loops:
            keep = a != b
            a, b = a[keep], b[keep]
        k = (a << np.uint64(32)) | b if directed else pack(a, b)
        if multi:
            have = np.concatenate([have, k[:want]])
        else:
            allk = np.concatenate([have, k])
            _, first = np.unique(allk, return_index=True)
            first.sort()
            have = allk[first][:m]
    return have[:m].astype(np.uint64)


def config_model_graph(n: int, gamma: float, dmin: int, dmax: int, seed: int, directed: bool = False) -> np.ndarray:
    """The configuration model's loopy multigraph of a Pld([dmin..dmax], gamma)
    degree sequence: stubs paired uniformly at random.  Directed: out-degrees
    from the draw, in-degrees a seeded permutation of them, out-stubs paired
    with in-stubs."""
    deg = powerlaw_degrees(n, gamma, dmin, dmax, seed).astype(np.int64)
    rng = np.random.default_rng(seed ^ 0x9E3779B97F4A7C15)
    stubs = np.repeat(np.arange(n, dtype=np.uint64), deg)
    if directed:
        heads = np.repeat(np.arange(n, dtype=np.uint64), deg[rng.permutation(n)])
        rng.shuffle(heads)
        rng.shuffle(stubs)
        return (stubs << np.uint64(32)) | heads
    rng.shuffle(stubs)
    return pack(stubs[0::2], stubs[1::2])


# ---------------------------------------------------------------------------
# Named workloads.  Each returns (edge keys uint64[m], n).
# ---------------------------------------------------------------------------

def workload_gnp_small():
    """G(n=1024, p=10/1023), generator seed 1 (~5.1k edges)."""
    n = 1024
    return gnp(n, 10.0 / 1023.0, 1), n


def workload_powerlaw_1m():
    """Pld([5..1024], 2.5) on n=2^20 (d_max = sqrt(n)), Havel-Hakimi, ids shuffled."""
    n = 1 << 20
    return powerlaw_graph(n, 2.5, 5, 1024, 2), n


def workload_gnp_large():
    """G(n=2^22, p=32/(2^22-1)): average degree 32, ~67M edges."""
    n = 1 << 22
    return gnp(n, 32.0 / (n - 1), 3), n


def batch_specs(G: int, seed: int, n_lo: float, n_hi: float, g_lo: float = 2.1, g_hi: float = 3.0):
    """Per-graph (n, gamma, d_max) of a batch: n log-uniform in [n_lo, n_hi],
    gamma uniform in [g_lo, g_hi], d_max = floor(sqrt(n))."""
    u = uniforms(seed, 2 * G)
    out = []
    for g in range(G):
        n = int(round(math.exp(math.log(n_lo) + u[2 * g] * (math.log(n_hi) - math.log(n_lo)))))
        gamma = g_lo + u[2 * g + 1] * (g_hi - g_lo)
        out.append((n, gamma, max(2, int(math.isqrt(n)))))
    return out


def batch_graphs(G: int, seed: int, n_lo: float, n_hi: float, dmin: int = 2):
    """G power-law graphs (Havel-Hakimi, ids shuffled): list of (edges, n)."""
    return [(powerlaw_graph(n, gamma, dmin, dmax, seed * 1000003 + g), n)
            for g, (n, gamma, dmax) in enumerate(batch_specs(G, seed, n_lo, n_hi))]


def concat(graphs):
    """[(edges, n)] -> (edges concatenated, offsets[G+1] int64, n[G] int64)."""
    offs = np.zeros(len(graphs) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(e) for e, _ in graphs])
    E = np.concatenate([e for e, _ in graphs]) if graphs else np.zeros(0, dtype=np.uint64)
    return E.astype(np.uint64), offs, np.array([n for _, n in graphs], dtype=np.int64)


def workload_batch_4096():
    """4096 power-law graphs, n log-uniform in [1e2, 1e5], gamma in [2.1, 3.0],
    d_min = 2, d_max = floor(sqrt(n)); generator seed 4."""
    return batch_graphs(4096, 4, 1e2, 1e5)


def workload_powerlaw_hubs():
    """Pld([1..n^(1/(gamma-1))], 2.01) on n=2^20 (SynPld's degree range at
    gamma near 2: hubs adjacent to half the vertices), Havel-Hakimi, ids
    shuffled; generator seed 11."""
    n, gamma = 1 << 20, 2.01
    return powerlaw_graph(n, gamma, 1, int(n ** (1.0 / (gamma - 1.0))), 11), n


WORKLOADS = {
    "gnp_n1024_d10": (workload_gnp_small, 10),
    "pld_n2^20_g2.5": (workload_powerlaw_1m, 20),
    "gnp_n2^22_d32": (workload_gnp_large, 10),
    "pld_n2^20_g2.01": (workload_powerlaw_hubs, 10),
}

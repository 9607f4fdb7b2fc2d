"""ORACLE -- test infrastructure only.

The plain sequential CPU implementation of G-ES-MC (``gesmc_oracle.cpp``,
compiled with g++ into ``liboracle.so``) and a naive pure-Python replay
(``naive.py``).  Only the tests, the smoke check and the benchmark's CPU
baseline leg may import this package; the HIP library never does, and the
two share no code.  See ``gesmc_oracle.cpp`` for the definitions followed.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gesmc_oracle.cpp")
_SRC_GEN = os.path.join(_HERE, "gen_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

LEGAL, LOOP, EXISTS, PL = 1, 2, 3, 4

MUT_FLIP_G = 1
MUT_NO_LOOP = 2
MUT_NO_EXISTS = 4
MUT_TAU_SWAP = 8
MUT_WRITE_SWAP = 16
MUT_NO_ERASE = 32
MUT_PAIR_SHIFT = 64
MUT_KEY_SWAP = 128
MUT_ES_J_ANY = 1 << 16
MUT_ES_G_HIGH = 1 << 17
MUT_ES_NO_SKIP = 1 << 18


class Counts(ctypes.Structure):
    _fields_ = [("attempts", ctypes.c_uint64), ("legal", ctypes.c_uint64), ("rej_loop", ctypes.c_uint64),
                ("rej_exists", ctypes.c_uint64), ("rej_pl", ctypes.c_uint64)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


def build() -> str:
    """Compile the oracle with g++ (always recompiles)."""
    tmp = _LIB + ".tmp"
    # no fused multiply-adds: the portable ln / exp must round every step
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared", "-o", tmp, _SRC,
                           _SRC_GEN])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    u32, u64, vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p
    lib.oracle_philox4x32_10.argtypes = [vp, vp, vp]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_perm_key.argtypes = [u64, u32, u64]
    lib.oracle_perm_key.restype = u64
    lib.oracle_perm_keys.argtypes = [u64, u32, u64, vp]
    lib.oracle_perm_keys.restype = None
    lib.oracle_pl_skip.argtypes = [u64, u32, u64, u32]
    lib.oracle_pl_skip.restype = ctypes.c_int
    lib.oracle_permutation_mut.argtypes = [u64, u64, u32, vp, u32]
    lib.oracle_permutation_mut.restype = None
    lib.oracle_permutation.argtypes = [u64, u64, u32, vp]
    lib.oracle_permutation.restype = None
    lib.oracle_validate.argtypes = [vp, u64, u32]
    lib.oracle_validate.restype = ctypes.c_int
    lib.oracle_global_switch.argtypes = [vp, u64, vp, vp, vp, vp, u32]
    lib.oracle_global_switch.restype = ctypes.c_int
    lib.oracle_run.argtypes = [vp, u64, u32, u64, u32, u32, u32, vp, vp, u32]
    lib.oracle_run.restype = ctypes.c_int
    lib.oracle_es_draws.argtypes = [u64, u64, u64, u64, vp, vp, vp, u32]
    lib.oracle_es_draws.restype = None
    lib.oracle_edge_switch.argtypes = [vp, u64, u64, u64, ctypes.c_int]
    lib.oracle_edge_switch.restype = ctypes.c_int
    lib.oracle_es_run.argtypes = [vp, u64, u32, u64, u64, u64, vp, vp, u32]
    lib.oracle_es_run.restype = ctypes.c_int
    lib.oracle_validate_class.argtypes = [vp, u64, u32, u32]
    lib.oracle_validate_class.restype = ctypes.c_int
    lib.oracle_run_class.argtypes = [vp, u64, u32, u64, u32, u32, u32, u32, vp, vp, u32]
    lib.oracle_run_class.restype = ctypes.c_int
    lib.oracle_edge_switch_class.argtypes = [vp, u64, u64, u64, ctypes.c_int, u32, u32]
    lib.oracle_edge_switch_class.restype = ctypes.c_int
    f64, i64 = ctypes.c_double, ctypes.c_int64
    lib.oracle_gen_set_mutate.argtypes = [u32]
    lib.oracle_gen_set_mutate.restype = None
    lib.oracle_ln_p.argtypes = [f64]
    lib.oracle_ln_p.restype = f64
    lib.oracle_exp_p.argtypes = [f64]
    lib.oracle_exp_p.restype = f64
    lib.oracle_pair_of.argtypes = [u64, vp, vp]
    lib.oracle_pair_of.restype = None
    lib.oracle_gnp_chunk.argtypes = [f64]
    lib.oracle_gnp_chunk.restype = u64
    lib.oracle_gen_gnp.argtypes = [u32, f64, u64, vp, i64]
    lib.oracle_gen_gnp.restype = i64
    lib.oracle_gen_pld.argtypes = [u32, f64, u32, u32, u64, vp, vp]
    lib.oracle_gen_pld.restype = i64
    lib.oracle_gen_havel_hakimi.argtypes = [u32, vp, vp, i64]
    lib.oracle_gen_havel_hakimi.restype = i64
    lib.oracle_gen_relabel.argtypes = [vp, u64, u32, u64]
    lib.oracle_gen_relabel.restype = None
    lib.oracle_selftest_edgeset.argtypes = [u64, u64]
    lib.oracle_selftest_edgeset.restype = u64
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data


def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def perm_keys(m: int, seed: int, t: int) -> np.ndarray:
    out = np.empty(max(m, 1), dtype=np.uint64)
    _load().oracle_perm_keys(seed, t, m, _p(out))
    return out[:m]


def pl_skip(seed: int, t: int, k: int, pl: int) -> bool:
    return bool(_load().oracle_pl_skip(seed, t, k, pl))


def permutation(m: int, seed: int, t: int, mutate: int = 0) -> np.ndarray:
    pi = np.empty(max(m, 1), dtype=np.uint32)
    _load().oracle_permutation_mut(m, seed, t, _p(pi), mutate)
    return pi[:m]


def validate(E: np.ndarray, n: int) -> int:
    E = np.ascontiguousarray(E, dtype=np.uint64)
    return _load().oracle_validate(_p(E), len(E), n)


def global_switch(E: np.ndarray, pi, skip=None, mutate: int = 0):
    """One global switch with explicit pi / skip mask.  Returns (E', outcomes, counts)."""
    E = np.ascontiguousarray(E, dtype=np.uint64).copy()
    m = len(E)
    pi = np.ascontiguousarray(pi, dtype=np.uint32)
    sk = None if skip is None else np.ascontiguousarray(skip, dtype=np.uint8)
    oc = np.zeros(max(m // 2, 1), dtype=np.uint8)
    c = Counts()
    _load().oracle_global_switch(_p(E), m, _p(pi), _p(sk), _p(oc), ctypes.byref(c), mutate)
    return E, oc[: m // 2], c.as_dict()


def run(E: np.ndarray, n: int, seed: int, t0: int, r: int, pl: int = 0, mutate: int = 0, outcomes: bool = False):
    """r global switches.  Returns (status, E', [per-superstep counts], last outcomes or None)."""
    E = np.ascontiguousarray(E, dtype=np.uint64).copy()
    m = len(E)
    per = (Counts * max(r, 1))()
    oc = np.zeros(max(m // 2, 1), dtype=np.uint8) if outcomes else None
    rc = _load().oracle_run(_p(E), m, n, seed, t0, r, pl, per, _p(oc), mutate)
    counts = [per[s].as_dict() for s in range(r)]
    return rc, E, counts, (oc[: m // 2] if outcomes else None)


def run_batch(graphs, seeds, rs, t0s=None, pl: int = 0):
    """Independent graphs, each run on its own: [(E_g, n_g)] -> list of
    (status, E_g', counts).  A batch has no arithmetic of its own -- every
    graph is a separate chain (Alg. 3 with its own seed, t0 and r), so this
    is the definition the batched form must equal."""
    out = []
    for g, (E, n) in enumerate(graphs):
        rc, E2, counts, _ = run(E, n, seeds[g], 0 if t0s is None else t0s[g], rs[g], pl)
        out.append((rc, E2, counts))
    return out


def es_draws(seed: int, k0: int, count: int, m: int, mutate: int = 0):
    """ES-MC draws of switches k0 .. k0+count-1 on m edges: (i, j, g) arrays."""
    i = np.empty(max(count, 1), dtype=np.uint64)
    j = np.empty(max(count, 1), dtype=np.uint64)
    g = np.empty(max(count, 1), dtype=np.uint8)
    _load().oracle_es_draws(seed & (2**64 - 1), k0, count, m, _p(i), _p(j), _p(g), mutate)
    return i[:count], j[:count], g[:count]


def edge_switch(E: np.ndarray, i: int, j: int, g: int):
    """One edge switch (Def. 2.1) on a copy of E: (E', outcome code)."""
    E = np.ascontiguousarray(E, dtype=np.uint64).copy()
    oc = _load().oracle_edge_switch(_p(E), len(E), i, j, g)
    return E, oc


def es_run(E: np.ndarray, n: int, seed: int, k0: int, r: int, mutate: int = 0, outcomes: bool = False):
    """ES-MC (Def. 2.1; the chain Alg. 2 parallelises): r switches from switch
    counter k0.  Returns (status, E', counts, per-switch outcomes or None)."""
    E = np.ascontiguousarray(E, dtype=np.uint64).copy()
    c = Counts()
    oc = np.zeros(max(r, 1), dtype=np.uint8) if outcomes else None
    rc = _load().oracle_es_run(_p(E), len(E), n, seed & (2**64 - 1), k0, r, ctypes.byref(c), _p(oc), mutate)
    return rc, E, c.as_dict(), (oc[:r] if outcomes else None)


CLS_LOOPS, CLS_MULTI, CLS_DIRECTED = 1, 2, 4
CMUT_DIR_TAILS, CMUT_NO_SAME, CMUT_LOOPS_ALWAYS, CMUT_LOOP_BOTH_G = 1, 2, 4, 8


def run_class(E: np.ndarray, n: int, seed: int, t0: int, r: int, pl: int = 0, cls: int = 0, outcomes: bool = False,
              mutate: int = 0):
    """Alg. 3 for a graph class (bits CLS_LOOPS, CLS_MULTI, CLS_DIRECTED): r
    global switches.  Returns (status, E', [per-superstep counts], last outcomes)."""
    E = np.ascontiguousarray(E, dtype=np.uint64).copy()
    m = len(E)
    per = (Counts * max(r, 1))()
    oc = np.zeros(max(m // 2, 1), dtype=np.uint8) if outcomes else None
    rc = _load().oracle_run_class(_p(E), m, n, seed & (2**64 - 1), t0, r, pl, cls, per, _p(oc), mutate)
    return rc, E, [per[s].as_dict() for s in range(r)], (oc[: m // 2] if outcomes else None)


def validate_class(E: np.ndarray, n: int, cls: int) -> int:
    E = np.ascontiguousarray(E, dtype=np.uint64)
    return _load().oracle_validate_class(_p(E), len(E), n, cls)


def edge_switch_class(E: np.ndarray, i: int, j: int, g: int, cls: int, mutate: int = 0):
    """One switch of a graph class on a copy of E: (E', outcome code)."""
    E = np.ascontiguousarray(E, dtype=np.uint64).copy()
    oc = _load().oracle_edge_switch_class(_p(E), len(E), i, j, g, cls, mutate)
    return E, oc


# ---- input realisation (gen_oracle.cpp) -----------------------------------

GMUT_LN_TERMS, GMUT_GNP_NO_ADVANCE, GMUT_GNP_CEIL, GMUT_GNP_CHUNK_SKIP = 1, 2, 4, 8
GMUT_PLD_SIGN, GMUT_PLD_OFF1, GMUT_HH_TIE, GMUT_HH_PICK, GMUT_RELABEL_INV, GMUT_EXP_TERMS = 16, 32, 64, 128, 256, 512


class gen_mutation:
    """Context manager planting a mistake in the input-realisation oracle."""

    def __init__(self, mutate: int):
        self.mutate = mutate

    def __enter__(self):
        _load().oracle_gen_set_mutate(self.mutate)
        return self

    def __exit__(self, *exc):
        _load().oracle_gen_set_mutate(0)
        return False


def ln_p(x: float) -> float:
    return _load().oracle_ln_p(float(x))


def exp_p(x: float) -> float:
    return _load().oracle_exp_p(float(x))


def pair_of(q: int):
    w, v = ctypes.c_uint32(), ctypes.c_uint32()
    _load().oracle_pair_of(q, ctypes.byref(w), ctypes.byref(v))
    return w.value, v.value


def gnp_chunk(p: float) -> int:
    return int(_load().oracle_gnp_chunk(float(p)))


def gen_gnp(n: int, p: float, seed: int) -> np.ndarray:
    """G(n,p) edge keys in pair order (see gen_oracle.cpp)."""
    lib = _load()
    m = lib.oracle_gen_gnp(n, float(p), seed & (2**64 - 1), None, 0)
    out = np.empty(max(m, 1), dtype=np.uint64)
    m2 = lib.oracle_gen_gnp(n, float(p), seed & (2**64 - 1), _p(out), m)
    assert m2 == m
    return out[:m]


def gen_pld(n: int, gamma: float, dmin: int, dmax: int, seed: int):
    """(degrees uint32[n], degree sum, redraws of vertex 0), or None on failure."""
    deg = np.empty(max(n, 1), dtype=np.uint32)
    rd = ctypes.c_uint32(0)
    s = _load().oracle_gen_pld(n, float(gamma), dmin, dmax, seed & (2**64 - 1), _p(deg), ctypes.byref(rd))
    if s < 0:
        return None
    return deg[:n], int(s), rd.value


def gen_havel_hakimi(deg) -> np.ndarray | None:
    """Havel-Hakimi realisation (edge keys), or None if not graphical."""
    d = np.ascontiguousarray(deg, dtype=np.uint32)
    half = int(d.astype(np.int64).sum()) // 2
    out = np.empty(max(half, 1), dtype=np.uint64)
    m = _load().oracle_gen_havel_hakimi(len(d), _p(d), _p(out), half)
    if m < 0:
        return None
    assert m == half
    return out[:m]


def gen_relabel(E, n: int, seed: int) -> np.ndarray:
    E = np.ascontiguousarray(E, dtype=np.uint64).copy()
    _load().oracle_gen_relabel(_p(E), len(E), n, seed & (2**64 - 1))
    return E


def selftest_edgeset(ops: int = 200000, seed: int = 1) -> int:
    return int(_load().oracle_selftest_edgeset(ops, seed))

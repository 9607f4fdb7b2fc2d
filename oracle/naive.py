"""ORACLE (test infrastructure only): a naive, pure-Python replay of G-ES-MC.

An independent second implementation of the same sequential chain as
``gesmc_oracle.cpp``, for small inputs only: its edge set is a plain Python
list scanned linearly, its Philox4x32-10 is written separately, and its
permutation is Python's ``sorted``.  Used to cross-check the C++ oracle.

Definitions followed (arXiv 2111.03005):
  * Def. 2.1: edge switch sigma = (i, j, g) and the tau map; reject on a loop
    or an existing target; otherwise E[i] <- e3, E[j] <- e4.
  * Def. 3.2: switch k uses (pi[2k], pi[2k+1]) with g = [pi[2k] < pi[2k+1]].
  * Sec. 3: each switch independently skipped with probability pl / 2^32.
Random choices use Philox4x32-10 (Salmon et al., SC'11) keyed by the seed
with counter (i, 0, t, 0) for the permutation key of edge i and (k, 0, t, 1)
for the skip test of switch k.
"""
from __future__ import annotations

M32 = 0xFFFFFFFF
LEGAL, LOOP, EXISTS, PL = 1, 2, 3, 4


def philox4x32_10(ctr, key):
    c = list(ctr)
    k0, k1 = key
    for rnd in range(10):
        if rnd:
            k0 = (k0 + 0x9E3779B9) & M32
            k1 = (k1 + 0xBB67AE85) & M32
        p0 = 0xD2511F53 * c[0]
        p1 = 0xCD9E8D57 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & M32, p1 & M32, ((p0 >> 32) ^ c[3] ^ k1) & M32, p0 & M32]
    return c


def perm_key(seed: int, t: int, i: int) -> int:
    x = philox4x32_10((i & M32, i >> 32, t, 0), (seed & M32, seed >> 32))
    return (x[0] << 32) | x[1]


def permutation(m: int, seed: int, t: int):
    return sorted(range(m), key=lambda i: (perm_key(seed, t, i), i))


def pl_skip(seed: int, t: int, k: int, pl: int) -> bool:
    if pl == 0:
        return False
    return philox4x32_10((k & M32, k >> 32, t, 1), (seed & M32, seed >> 32))[0] < pl


def _split(e):
    return e >> 32, e & M32


def _key(a, b):
    return (min(a, b) << 32) | max(a, b)


def global_switch(E, pi, skip=None):
    """Apply one global switch in place; returns the list of outcome codes."""
    m = len(E)
    out = []
    for k in range(m // 2):
        i, j = pi[2 * k], pi[2 * k + 1]
        if skip is not None and skip[k]:
            out.append(PL)
            continue
        g = 1 if i < j else 0
        u, v = _split(E[i])
        x, y = _split(E[j])
        if g == 0:
            a, b = (u, x), (v, y)
        else:
            a, b = (u, y), (v, x)
        if a[0] == a[1] or b[0] == b[1]:
            out.append(LOOP)
            continue
        e3, e4 = _key(*a), _key(*b)
        present = list(E)  # the current edge list is the edge set
        if e3 in present or e4 in present:
            out.append(EXISTS)
            continue
        E[i], E[j] = e3, e4
        out.append(LEGAL)
    return out


def run(E, seed: int, t0: int, r: int, pl: int = 0):
    """r global switches; returns (E, per-superstep counts, last outcomes)."""
    E = [_key(*_split(e)) for e in E]
    counts = []
    last = []
    m = len(E)
    for s in range(r):
        t = t0 + s
        if m < 2:
            counts.append(dict(attempts=0, legal=0, rej_loop=0, rej_exists=0, rej_pl=0))
            continue
        pi = permutation(m, seed, t)
        skip = [pl_skip(seed, t, k, pl) for k in range(m // 2)]
        last = global_switch(E, pi, skip)
        counts.append(dict(attempts=m // 2, legal=last.count(LEGAL), rej_loop=last.count(LOOP),
                           rej_exists=last.count(EXISTS), rej_pl=last.count(PL)))
    return E, counts, last


# ---------------------------------------------------------------------------
# ES-MC (Def. 2.1, the chain Alg. 2 parallelises), written out separately
# ---------------------------------------------------------------------------

def es_draw(seed: int, k: int, m: int):
    """Switch k's (i, j, g): Philox at counter (k_lo, k_hi, 0, 2); i uniform on
    [0, m) from the first 64-bit word, j uniform on [0, m) without i from the
    second (the value j' on [0, m-1) moved up past i), g the lowest bit of x1."""
    x = philox4x32_10((k & M32, k >> 32, 0, 2), (seed & M32, seed >> 32))
    w0 = (x[0] << 32) | x[1]
    w1 = (x[2] << 32) | x[3]
    i = (w0 * m) >> 64
    jp = (w1 * (m - 1)) >> 64
    j = jp + 1 if jp >= i else jp
    return i, j, x[1] & 1


def es_run(E, seed: int, k0: int, r: int):
    """r ES-MC switches from counter k0, one at a time: (E, outcome codes)."""
    E = [_key(*_split(e)) for e in E]
    m = len(E)
    out = []
    if m < 2:
        return E, out
    for k in range(k0, k0 + r):
        i, j, g = es_draw(seed, k, m)
        u, v = _split(E[i])
        x, y = _split(E[j])
        a, b = ((u, x), (v, y)) if g == 0 else ((u, y), (v, x))
        if a[0] == a[1] or b[0] == b[1]:
            out.append(LOOP)
            continue
        e3, e4 = _key(*a), _key(*b)
        if e3 in E or e4 in E:
            out.append(EXISTS)
            continue
        E[i], E[j] = e3, e4
        out.append(LEGAL)
    return E, out


# ---------------------------------------------------------------------------
# Graph classes (Sec. 1): loops allowed (1), multi-edges allowed (2),
# directed (4), written out separately
# ---------------------------------------------------------------------------

def _ckey(a, b, cls):
    return (a << 32) | b if cls & 4 else _key(a, b)


def run_class(E, seed: int, t0: int, r: int, pl: int, cls: int):
    """r global switches of class cls, one at a time: (E, per-superstep counts)."""
    E = [_ckey(*_split(e), cls) for e in E]
    m = len(E)
    counts = []
    for s in range(r):
        t = t0 + s
        c = dict(attempts=0, legal=0, rej_loop=0, rej_exists=0, rej_pl=0)
        if m >= 2:
            pi = permutation(m, seed, t)
            for k in range(m // 2):
                c["attempts"] += 1
                if pl_skip(seed, t, k, pl):
                    c["rej_pl"] += 1
                    continue
                i, j = pi[2 * k], pi[2 * k + 1]
                u, v = _split(E[i])
                x, y = _split(E[j])
                if cls & 4:
                    a, b = (u, y), (x, v)
                elif i < j:
                    a, b = (u, y), (v, x)
                else:
                    a, b = (u, x), (v, y)
                if not (cls & 1) and (a[0] == a[1] or b[0] == b[1]):
                    c["rej_loop"] += 1
                    continue
                if cls & 7 == 1 and i < j and (u == v or x == y):
                    c["rej_loop"] += 1  # a loop source: g = 1 gives g = 0's targets again
                    continue
                e3, e4 = _ckey(*a, cls), _ckey(*b, cls)
                if not (cls & 2) and (e3 == e4 or e3 in E or e4 in E):
                    c["rej_exists"] += 1
                    continue
                E[i], E[j] = e3, e4
                c["legal"] += 1
        counts.append(c)
    return E, counts

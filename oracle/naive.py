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


# ---------------------------------------------------------------------------
# Input realisation (the definitions in gen_oracle.cpp), written out again in
# plain Python for small cases: Python floats are IEEE doubles whose +, -, *,
# / round correctly and never fuse, so the portable ln / exp give the same
# bits here as there.
# ---------------------------------------------------------------------------
import math as _math
import struct as _struct

_LN2_HI = 6.93147180369123816490e-01
_LN2_LO = 1.90821492927058770002e-10


def ln_p(x: float) -> float:
    b = _struct.unpack("<Q", _struct.pack("<d", x))[0]
    e = ((b >> 52) & 0x7FF) - 1023
    m = _struct.unpack("<d", _struct.pack("<Q", (b & ((1 << 52) - 1)) | (1023 << 52)))[0]
    if m > 1.4142135623730951:
        m *= 0.5
        e += 1
    f = m - 1.0
    s = f / (2.0 + f)
    z = s * s
    P = 1.0 / 23.0
    for j in range(10, 0, -1):
        P = P * z + 1.0 / (2 * j + 1)
    t = 2.0 * s
    return e * _LN2_HI + (e * _LN2_LO + (t + t * (z * P)))


def exp_p(x: float) -> float:
    kd = _math.floor(x * 1.4426950408889634 + 0.5)
    r = (x - kd * _LN2_HI) - kd * _LN2_LO
    p = 1.0 / _math.factorial(13)
    for j in range(12, -1, -1):
        p = p * r + 1.0 / _math.factorial(j)
    return p * 2.0 ** kd


def gnp(n: int, p: float, seed: int):
    """G(n,p) by the chunked geometric skips, pair index decoded by search."""
    if n < 2 or not p > 0:
        return []
    N = n * (n - 1) // 2
    rows = [(v * (v - 1) // 2, v) for v in range(1, n)]

    def pair(q):
        base, v = max(r for r in rows if r[0] <= q)
        return ((q - base) << 32) | v

    if p >= 1:
        return [pair(q) for q in range(N)]
    L = 64
    while L * p < 64 and L < 2 ** 40:
        L *= 2
    lq = ln_p(1.0 - p)
    out = []
    j = 0
    while j * L < N:
        end, c, t = min(j * L + L, N), j * L, 0
        while True:
            x = philox4x32_10((j & M32, j >> 32, t, 3), (seed & M32, (seed >> 32) & M32))
            U = (((x[0] << 32 | x[1]) >> 11) + 1) / 2.0 ** 53
            G = ln_p(U) / lq
            t += 1
            if not G < end - c:
                break
            q = c + int(G)
            out.append(pair(q))
            c = q + 1
            if c >= end:
                break
        j += 1
    return out


def pld(n: int, gamma: float, dmin: int, dmax: int, seed: int):
    """Degrees by the integer-weight inverse CDF; None if no even sum."""
    W = [int(exp_p(-(gamma * (ln_p(float(k)) - ln_p(float(dmin))))) * 2.0 ** 43) for k in range(dmin, dmax + 1)]
    C, acc = [], 0
    for w in W:
        acc += w
        C.append(acc)

    def draw(v, r):
        x = philox4x32_10((v, r, 0, 4), (seed & M32, (seed >> 32) & M32))
        u = ((x[0] << 32 | x[1]) * acc) >> 64
        return dmin + next(i for i, c in enumerate(C) if c > u)

    deg = [draw(v, 0) for v in range(n)]
    r = 0
    while sum(deg) % 2:
        if dmin == dmax or r == 65535:
            return None
        r += 1
        deg[0] = draw(0, r)
    return deg


def havel_hakimi(deg):
    """The Havel-Hakimi construction by exhaustive scans: positions by
    (degree desc, id asc); v = largest residual, smallest position; partners
    the d others of positive residual with the largest (residual, position).
    Returns the edge keys, or None if not graphical."""
    n = len(deg)
    order = sorted(range(n), key=lambda v: (-deg[v], v))
    res = [deg[v] for v in order]
    out = []
    while any(res):
        top = max(res)
        s = min(p for p in range(n) if res[p] == top)
        d = res[s]
        res[s] = 0
        cand = sorted((p for p in range(n) if res[p] > 0), key=lambda p: (res[p], p), reverse=True)
        if len(cand) < d:
            return None
        for p in sorted(cand[:d]):
            res[p] -= 1
            a, b = order[s], order[p]
            out.append((min(a, b) << 32) | max(a, b))
    return out


def erdos_gallai(deg) -> bool:
    """Graphicality by the Erdos-Gallai inequalities."""
    d = sorted(deg, reverse=True)
    if sum(d) % 2:
        return False
    n = len(d)
    for k in range(1, n + 1):
        if sum(d[:k]) > k * (k - 1) + sum(min(x, k) for x in d[k:]):
            return False
    return True

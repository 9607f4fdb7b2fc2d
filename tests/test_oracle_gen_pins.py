"""Pins of the input-realisation oracle (``oracle/gen_oracle.cpp``: G(n,p),
power-law degrees, Havel-Hakimi, relabelling -- the steps before the chain
that Sec. 6 uses to build its synthetic inputs), each against something
other than the oracle itself:

* the portable ln / exp against the platform's libm within 2 ulp, and their
  exact values at 1 and 0;
* the pair index decode against plain enumeration;
* G(n,p): per-pair frequencies and edge counts against the binomial law,
  gaps against the geometric law, the special cases p = 0 and p = 1;
* degrees: the histogram against the exact Pld pmf by chi-square, the even
  sum and its failure cases;
* Havel-Hakimi: an independent brute-force replay (``oracle/naive.py``),
  the realised degrees, simplicity, and failure exactly on the sequences the
  Erdos-Gallai inequalities reject (every sequence on up to 6 vertices);
* relabelling: the bijection of the (pinned) permutation of Def. 3.2;
* the whole definitions against the pure-Python replay at small sizes.

Every planted mistake (``oracle.GMUT_*``) fails at least one pin.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import naive

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def ulps(a: float, b: float) -> float:
    return abs(a - b) / math.ulp(b) if b != 0 else abs(a) / math.ulp(1.0)


# ---- portable ln / exp ------------------------------------------------------

def pin_ln():
    rng = np.random.default_rng(1)
    xs = list(rng.uniform(2.0 ** -53, 1.0, 4000)) + list(np.exp(rng.uniform(-40, 20, 4000)))
    xs += [float(k) for k in range(1, 3000)] + [2.0 ** k for k in range(-60, 40)]
    xs += [1.4142135623730951, np.nextafter(1.4142135623730951, 2.0), np.nextafter(1.0, 0.0), 1.0 - 1e-9]
    worst = max(ulps(oracle.ln_p(x), math.log(x)) for x in xs if x != 1.0)
    return worst <= 2.0 and oracle.ln_p(1.0) == 0.0


def pin_exp():
    rng = np.random.default_rng(2)
    xs = list(rng.uniform(-700.0, 0.0, 4000)) + list(rng.uniform(-1.0, 0.0, 4000)) + [-0.0, -1e-300, -0.5, -700.0]
    worst = max(ulps(oracle.exp_p(x), math.exp(x)) for x in xs)
    return worst <= 2.0 and oracle.exp_p(0.0) == 1.0 and oracle.exp_p(-0.0) == 1.0


def test_ln_exp_accuracy():
    assert pin_ln()
    assert pin_exp()


def test_ln_exp_python_replay_same_bits():
    rng = np.random.default_rng(3)
    for x in list(rng.uniform(2.0 ** -53, 1.0, 500)) + [float(k) for k in range(1, 200)]:
        assert oracle.ln_p(x) == naive.ln_p(x)
    for x in list(rng.uniform(-700.0, 0.0, 500)):
        assert oracle.exp_p(x) == naive.exp_p(x)


def test_pair_decode_enumeration():
    q = 0
    for v in range(1, 400):
        for w in range(v):
            assert oracle.pair_of(q) == (w, v)
            q += 1
    for v in [1 << 20, (1 << 22) - 1, (1 << 31) + 12345, (1 << 32) - 1]:
        base = v * (v - 1) // 2
        for w in [0, 1, v // 2, v - 1]:
            assert oracle.pair_of(base + w) == (w, v)


# ---- G(n,p) -----------------------------------------------------------------

def split(E):
    E = np.asarray(E, dtype=np.uint64)
    return (E >> np.uint64(32)).astype(np.int64), (E & np.uint64(0xFFFFFFFF)).astype(np.int64)


def pin_gnp_structure():
    for n, p, seed in [(50, 0.3, 1), (1000, 0.01, 2), (3000, 0.002, 3), (200, 0.9, 4)]:
        E = oracle.gen_gnp(n, p, seed)
        w, v = split(E)
        q = v * (v - 1) // 2 + w
        if not (np.all(w < v) and np.all(v < n) and np.all(np.diff(q) > 0)):
            return False
    N = 40 * 39 // 2
    full = oracle.gen_gnp(40, 1.0, 5)
    w, v = split(full)
    return (len(full) == N and np.array_equal(v * (v - 1) // 2 + w, np.arange(N)) and len(oracle.gen_gnp(40, 0.0, 5)) == 0
            and len(oracle.gen_gnp(1, 0.5, 5)) == 0)


def pin_gnp_marginals():
    """n = 12 (66 pairs), p = 0.3, 3000 seeds: each pair's count and the
    per-graph edge count against the binomial law (5 sigma)."""
    n, p, S = 12, 0.3, 3000
    N = n * (n - 1) // 2
    hits = np.zeros(N)
    counts = []
    for s in range(S):
        w, v = split(oracle.gen_gnp(n, p, 1000 + s))
        np.add.at(hits, v * (v - 1) // 2 + w, 1)
        counts.append(len(w))
    sd = math.sqrt(S * p * (1 - p))
    if np.max(np.abs(hits - S * p)) > 5 * sd:
        return False
    c = np.array(counts, dtype=np.float64)
    return abs(c.mean() - N * p) < 5 * math.sqrt(N * p * (1 - p) / S) and abs(c.var() / (N * p * (1 - p)) - 1) < 0.15


def pin_gnp_gaps():
    """Gaps between consecutive pair indices (across chunk boundaries) are
    geometric: chi-square against (1-p)^k p over 20 bins."""
    n, p = 4000, 0.003
    assert oracle.gnp_chunk(p) * p >= 64
    w, v = split(oracle.gen_gnp(n, p, 77))
    q = v * (v - 1) // 2 + w
    gaps = np.diff(np.concatenate([[-1], q])) - 1
    edges = np.unique(np.floor(-np.log(1 - np.linspace(0, 0.999, 21)) / p)).astype(np.int64)
    obs, exp = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        obs.append(np.sum((gaps >= a) & (gaps < b)))
        exp.append(len(gaps) * ((1 - p) ** a - (1 - p) ** b))
    obs.append(np.sum(gaps >= edges[-1]))
    exp.append(len(gaps) * (1 - p) ** edges[-1])
    chi2 = sum((o - e) ** 2 / e for o, e in zip(obs, exp))
    return chi2 < 60.0  # 20 degrees of freedom: p-value ~ 1e-5


def test_gnp_structure_and_laws():
    assert pin_gnp_structure()
    assert pin_gnp_marginals()
    assert pin_gnp_gaps()


def test_gnp_chunk_rule():
    assert oracle.gnp_chunk(0.5) == 128 and oracle.gnp_chunk(0.99) == 128 and oracle.gnp_chunk(0.25) == 256
    assert oracle.gnp_chunk(32.0 / ((1 << 22) - 1)) == 1 << 23
    assert oracle.gnp_chunk(1e-15) == 1 << 40


def test_gnp_python_replay():
    for n, p, seed in [(30, 0.2, 5), (70, 0.05, 6), (25, 0.7, 7), (12, 1.0, 8), (40, 0.01, 2**63 + 5)]:
        assert [int(x) for x in oracle.gen_gnp(n, p, seed)] == naive.gnp(n, p, seed)


# ---- power-law degrees --------------------------------------------------------

def pin_pld_law():
    for gamma, a, b in [(2.5, 5, 64), (2.1, 1, 30), (3.0, 2, 20)]:
        r = oracle.gen_pld(200000, gamma, a, b, 11)
        if r is None:
            return False
        deg, s, _ = r
        if s % 2 or s != int(deg.astype(np.int64).sum()) or deg.min() < a or deg.max() > b:
            return False
        ks = np.arange(a, b + 1)
        pmf = ks.astype(np.float64) ** -gamma
        pmf /= pmf.sum()
        obs = np.bincount(deg - a, minlength=len(ks)).astype(np.float64)
        exp = len(deg) * pmf
        keep = exp >= 5
        chi2 = np.sum((obs[keep] - exp[keep]) ** 2 / exp[keep]) + (obs[~keep].sum() - exp[~keep].sum()) ** 2 / max(
            exp[~keep].sum(), 1)
        if chi2 > 3 * keep.sum() + 40:
            return False
    return True


def pin_pld_cases():
    if oracle.gen_pld(7, 2.0, 3, 3, 1) is not None:  # odd sum, a single value
        return False
    d = oracle.gen_pld(8, 2.0, 3, 3, 1)
    if d is None or list(d[0]) != [3] * 8:
        return False
    return oracle.gen_pld(10, 2.0, 0, 5, 1) is None and oracle.gen_pld(10, 2.0, 6, 5, 1) is None


def test_pld_law_and_cases():
    assert pin_pld_law()
    assert pin_pld_cases()


def test_pld_python_replay():
    for args in [(40, 2.3, 2, 12, 9), (25, 2.01, 1, 5, 3), (31, 3.0, 4, 40, 2**40 + 1)]:
        r = oracle.gen_pld(*args)
        assert list(r[0]) == naive.pld(*args)


# ---- Havel-Hakimi -------------------------------------------------------------

def pin_hh_naive():
    rng = np.random.default_rng(5)
    for trial in range(400):
        n = int(rng.integers(1, 16))
        deg = [int(x) for x in rng.integers(0, n, n)]
        if sum(deg) % 2:
            deg[0] = deg[0] - 1 if deg[0] > 0 else 1
        o = oracle.gen_havel_hakimi(np.array(deg, dtype=np.uint32))
        nv = naive.havel_hakimi(deg)
        if (o is None) != (nv is None) or (o is not None and [int(x) for x in o] != nv):
            return False
    return True


def realises(E, deg):
    w, v = split(E)
    got = np.bincount(np.concatenate([w, v]), minlength=len(deg))
    return np.all(w < v) and len(np.unique(E)) == len(E) and np.array_equal(got, np.asarray(deg))


def pin_hh_realises():
    for n, gamma, a, b, seed in [(5000, 2.5, 2, 70, 1), (20000, 2.1, 1, 141, 2), (3000, 3.0, 5, 54, 3)]:
        deg = oracle.gen_pld(n, gamma, a, b, seed)[0]
        E = oracle.gen_havel_hakimi(deg)
        if E is None or not realises(E, deg):
            return False
    return True


def pin_hh_erdos_gallai():
    for n in range(1, 7):
        for deg in itertools.product(range(n), repeat=n):
            if sum(deg) % 2:
                continue
            E = oracle.gen_havel_hakimi(np.array(deg, dtype=np.uint32))
            if (E is not None) != naive.erdos_gallai(deg):
                return False
            if E is not None and not realises(E, deg):
                return False
    return True


def test_havel_hakimi_pins():
    assert pin_hh_naive()
    assert pin_hh_realises()
    assert pin_hh_erdos_gallai()


# ---- relabelling --------------------------------------------------------------

def pin_relabel():
    n, seed = 300, 99
    deg = oracle.gen_pld(n, 2.5, 2, 17, 4)[0]
    E = oracle.gen_havel_hakimi(deg)
    R = oracle.gen_relabel(E, n, seed)
    pi = oracle.permutation(n, seed ^ 0x9E3779B97F4A7C15, 0)
    sigma = np.empty(n, dtype=np.int64)
    sigma[pi] = np.arange(n)
    w, v = split(E)
    a, b = sigma[w], sigma[v]
    want = (np.minimum(a, b).astype(np.uint64) << np.uint64(32)) | np.maximum(a, b).astype(np.uint64)
    return np.array_equal(R, want) and realises(R, np.bincount(np.concatenate(split(R)), minlength=n))


def test_relabel_pin():
    assert pin_relabel()


# ---- every planted mistake is caught -------------------------------------------

@pytest.mark.parametrize("mut,pins", [
    (oracle.GMUT_LN_TERMS, [pin_ln]),
    (oracle.GMUT_EXP_TERMS, [pin_exp]),
    (oracle.GMUT_GNP_NO_ADVANCE, [pin_gnp_structure]),
    (oracle.GMUT_GNP_CEIL, [pin_gnp_marginals]),
    (oracle.GMUT_GNP_CHUNK_SKIP, [pin_gnp_marginals]),
    (oracle.GMUT_PLD_SIGN, [pin_pld_law]),
    (oracle.GMUT_PLD_OFF1, [pin_pld_law]),
    (oracle.GMUT_HH_TIE, [pin_hh_naive]),
    (oracle.GMUT_HH_PICK, [pin_hh_naive]),
    (oracle.GMUT_RELABEL_INV, [pin_relabel]),
])
def test_planted_mistakes_caught(mut, pins):
    with oracle.gen_mutation(mut):
        caught = [not pin() for pin in pins]
    assert any(caught), mut

"""Pins for the oracle: checks against things other than the oracle itself.

  * rocRAND's Philox4x32-10 engine evaluated on the host (an independent,
    published implementation) for the generator and the permutation keys;
  * hand-derived worked examples: Fig. 1 (Def. 2.1) and global switches
    evaluated by hand from Def. 3.2 (tests/golden/);
  * properties fixed by the paper: degree sequence and simplicity preserved,
    pi is a permutation sorted by its keys, unbiased direction bits (Sec. 3);
  * Thm. 3.3: the exact transition matrix over all permutations is symmetric
    and (with P_L > 0) irreducible;  chi-square uniformity over brute-force
    enumerated G(d);
  * an independent naive replay (oracle/naive.py);
  * planted mistakes (oracle mutation flags) are each caught by some pin.
"""
import itertools
import json
import math
import os
import shutil
import subprocess
import tempfile
from collections import Counter

import numpy as np
import pytest
from scipy import stats
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

import graphgen
import oracle
from oracle import naive

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")
OUTCOME = {"legal": oracle.LEGAL, "loop": oracle.LOOP, "exists": oracle.EXISTS, "pl": oracle.PL}


def key(a, b):
    return (min(a, b) << 32) | max(a, b)


def keys(pairs):
    return np.array([key(a, b) for a, b in pairs], dtype=np.uint64)


# ---------------------------------------------------------------------------
# rocRAND host helper
# ---------------------------------------------------------------------------
_ROC = {}


def rocrand_bin():
    if "bin" in _ROC:
        return _ROC["bin"]
    src = os.path.join(HERE, "rocrand_philox_host.cpp")
    out = os.path.join(tempfile.mkdtemp(prefix="rocrand_host_"), "philox_host")
    inc = "/opt/rocm/include"
    cmd = None
    if shutil.which("g++") and os.path.isdir(os.path.join(inc, "rocrand")):
        cmd = ["g++", "-O1", "-std=c++17", "-I" + inc, "-D__HIP_PLATFORM_AMD__", src, "-o", out]
    if cmd is None:
        pytest.skip("rocRAND headers or host compiler unavailable")
    subprocess.check_call(cmd)
    _ROC["bin"] = out
    return out


def rocrand_query(text):
    r = subprocess.run([rocrand_bin()], input=text, capture_output=True, text=True, check=True)
    return r.stdout.split()


def philox_grid():
    rng = np.random.default_rng(12345)
    edge = [0, 1, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFF]
    rows = []
    for c in itertools.product(edge, repeat=2):
        rows.append((c[0], c[1], c[0] ^ 0x55, c[1], 0x01234567, 0x89ABCDEF))
    for _ in range(200):
        rows.append(tuple(int(x) for x in rng.integers(0, 2**32, size=6, dtype=np.uint64)))
    return rows


# ---------------------------------------------------------------------------
# Philox and the permutation
# ---------------------------------------------------------------------------

def test_philox_matches_rocrand():
    rows = philox_grid()
    got = rocrand_query("".join("R %d %d %d %d %d %d\n" % r for r in rows))
    ref = np.array(got, dtype=np.uint64).reshape(-1, 4)
    for r, exp in zip(rows, ref):
        out = oracle.philox(r[:4], r[4:])
        assert [int(x) for x in out] == [int(x) for x in exp], r


def test_naive_philox_matches_oracle():
    for r in philox_grid()[:60]:
        assert naive.philox4x32_10(r[:4], r[4:]) == [int(x) for x in oracle.philox(r[:4], r[4:])]


def pin_perm_keys_rocrand(mutate=0):
    """pi sorts the indices by rocRAND-computed keys (x0<<32|x1 at (i,0,t,0)), ties by index."""
    ok = True
    for seed, t, m in [(42, 0, 257), (0xDEADBEEFCAFEF00D, 7, 100), (1, 123456, 33)]:
        kk = np.array(rocrand_query("K %d %d %d\n" % (seed, t, m)), dtype=np.uint64)
        pi = oracle.permutation(m, seed, t, mutate=mutate)
        exp = np.array(sorted(range(m), key=lambda i: (int(kk[i]), i)), dtype=np.uint32)
        ok &= np.array_equal(pi, exp)
    return ok


def test_perm_keys_match_rocrand():
    seed, t, m = 0x0123456789ABCDEF, 3, 64
    kk = np.array(rocrand_query("K %d %d %d\n" % (seed, t, m)), dtype=np.uint64)
    assert np.array_equal(oracle.perm_keys(m, seed, t), kk)
    assert pin_perm_keys_rocrand()


def test_permutation_is_sorted_permutation():
    for m, seed, t in [(1, 1, 0), (2, 5, 1), (1000, 42, 9), (5209, 42, 0)]:
        pi = oracle.permutation(m, seed, t)
        assert sorted(pi.tolist()) == list(range(m))
        k = oracle.perm_keys(m, seed, t)
        pairs = list(zip(k[pi].tolist(), pi.tolist()))
        assert all(a < b for a, b in zip(pairs, pairs[1:]))
        assert pi.tolist() == naive.permutation(m, seed, t) if m <= 1000 else True


@pytest.mark.parametrize("m,trials", [(4, 24000), (5, 36000)])
def test_permutation_uniform_chi2(m, trials):
    """pi over supersteps t is uniform on S_m (Def. 3.2 draws pi uniformly)."""
    cnt = Counter(tuple(oracle.permutation(m, 99, t).tolist()) for t in range(trials))
    k = math.factorial(m)
    assert len(cnt) == k
    obs = np.array([cnt[p] for p in itertools.permutations(range(m))])
    p = stats.chisquare(obs).pvalue
    assert p > 1e-4, p


def test_direction_bits_unbiased():
    """g_k = [pi[2k] < pi[2k+1]] are unbiased bits (remark after Def. 3.2)."""
    ones = total = 0
    for t in range(200):
        pi = oracle.permutation(2001, 7, t)
        g = pi[0:2000:2] < pi[1:2000:2]
        ones += int(g.sum())
        total += len(g)
    assert stats.binomtest(ones, total, 0.5).pvalue > 1e-4


def test_pl_rate():
    pl = 1 << 30  # P_L = 1/4
    hits = sum(oracle.pl_skip(5, t, k, pl) for t in range(40) for k in range(500))
    assert stats.binomtest(hits, 20000, 0.25).pvalue > 1e-4
    assert not any(oracle.pl_skip(5, t, k, 0) for t in range(3) for k in range(100))
    assert all(naive.pl_skip(5, t, k, pl) == oracle.pl_skip(5, t, k, pl) for t in range(5) for k in range(50))


# ---------------------------------------------------------------------------
# Worked examples (golden)
# ---------------------------------------------------------------------------

def pin_fig1(mutate=0):
    g = json.load(open(os.path.join(GOLD, "fig1_edge_switch.json")))
    ok = True
    for c in g["cases"]:
        E = keys(c["E"])
        pi = np.array(c["pi"], dtype=np.uint32)
        assert int(pi[0] < pi[1]) == c["g"]
        E2, oc, _ = oracle.global_switch(E, pi, mutate=mutate)
        ok &= int(oc[0]) == OUTCOME[c["outcome"]]
        ok &= np.array_equal(E2, keys(c["E_after"]))
    return ok


def pin_by_hand(mutate=0):
    g = json.load(open(os.path.join(GOLD, "global_switch_by_hand.json")))
    ok = True
    for c in g["cases"]:
        E = keys(c["E"])
        pi = np.array(c["pi"], dtype=np.uint32)
        E2, oc, cnt = oracle.global_switch(E, pi, mutate=mutate)
        ok &= [int(x) for x in oc] == [OUTCOME[o] for o in c["outcomes"]]
        ok &= np.array_equal(E2, keys(c["E_after"]))
    return ok


def test_fig1_worked_example():
    assert pin_fig1()


def test_global_switch_by_hand():
    assert pin_by_hand()


def test_naive_on_golden():
    for name in ["fig1_edge_switch.json", "global_switch_by_hand.json"]:
        for c in json.load(open(os.path.join(GOLD, name)))["cases"]:
            E = [int(x) for x in keys(c["E"])]
            out = naive.global_switch(E, c["pi"])
            assert E == [int(x) for x in keys(c["E_after"])]
            exp = c["outcomes"] if "outcomes" in c else [c["outcome"]]
            assert out == [OUTCOME[o] for o in exp]


# ---------------------------------------------------------------------------
# Invariants on real workloads
# ---------------------------------------------------------------------------

def pin_invariants(mutate=0):
    ok = True
    cases = [graphgen.workload_gnp_small(), (graphgen.powerlaw_graph(3000, 2.1, 2, 60, 11), 3000),
             (graphgen.gnp(30, 0.9, 4), 30)]
    for E, n in cases:
        rc, E2, counts, _ = oracle.run(E, n, 42, 0, 6, 1 << 28, mutate=mutate)
        ok &= rc == 0 and len(E2) == len(E)
        u, v = graphgen.split(E2)
        ok &= bool((u < v).all()) and bool((v < n).all())
        ok &= len(np.unique(E2)) == len(E2)
        ok &= np.array_equal(graphgen.degrees(E2, n), graphgen.degrees(E, n))
        for c in counts:
            ok &= c["attempts"] == len(E) // 2
            ok &= c["legal"] + c["rej_loop"] + c["rej_exists"] + c["rej_pl"] == c["attempts"]
    return ok


def test_invariants_degrees_simple():
    assert pin_invariants()


def test_validate_rejects_nonsimple_and_range():
    assert oracle.validate(keys([(0, 1), (1, 2)]), 3) == 0
    assert oracle.validate(keys([(0, 1), (1, 0)]), 3) == -2  # duplicate
    assert oracle.validate(np.array([(2 << 32) | 2], dtype=np.uint64), 3) == -2  # loop
    assert oracle.validate(keys([(0, 3)]), 3) == -3  # id >= n
    rc, E, _, _ = oracle.run(keys([(0, 1), (0, 1)]), 3, 1, 0, 2)
    assert rc == -2


def test_noncanonical_input_and_tiny_m():
    E = np.array([(1 << 32) | 0, (3 << 32) | 2], dtype=np.uint64)  # (1,0), (3,2)
    rc, E2, _, _ = oracle.run(E, 4, 3, 0, 0)
    assert rc == 0 and E2.tolist() == [key(0, 1), key(2, 3)]
    for m in (0, 1):
        E = keys([(0, 1)][:m])
        rc, E2, c, _ = oracle.run(E, 2, 1, 0, 3)
        assert rc == 0 and E2.tolist() == E.tolist() and all(x["attempts"] == 0 for x in c)


def test_edgeset_selftest():
    assert oracle.selftest_edgeset(300000, 11) == 0


def test_star_all_rejected():
    """Every pair of edges of a star shares the centre: all switches reject."""
    E = keys([(0, v) for v in range(1, 40)])
    rc, E2, counts, oc = oracle.run(E, 40, 9, 0, 5, outcomes=True)
    assert rc == 0 and E2.tolist() == E.tolist()
    assert all(c["legal"] == 0 for c in counts)


def test_complete_graph_all_rejected():
    n = 9
    E = keys([(a, b) for a in range(n) for b in range(a + 1, n)])
    rc, E2, counts, _ = oracle.run(E, n, 3, 0, 4)
    assert E2.tolist() == E.tolist() and all(c["legal"] == 0 for c in counts)


# ---------------------------------------------------------------------------
# Naive replay equality
# ---------------------------------------------------------------------------

def pin_naive(mutate=0):
    ok = True
    cases = [(graphgen.gnp(30, 0.3, s), 30) for s in range(3)]
    cases += [(graphgen.gnp(12, 0.8, 5), 12), (keys([(0, v) for v in range(1, 9)]), 9),
              (graphgen.powerlaw_graph(200, 2.2, 1, 14, 3), 200)]
    for E, n in cases:
        for seed, pl in [(1, 0), (77, 1 << 31)]:
            En, cn, ln = naive.run([int(x) for x in E], seed, 5, 4, pl)
            rc, Eo, co, lo = oracle.run(E, n, seed, 5, 4, pl, mutate=mutate, outcomes=True)
            ok &= [int(x) for x in Eo] == En and co == cn and [int(x) for x in lo] == ln
    return ok


def test_naive_equals_oracle():
    assert pin_naive()


def test_oracle_resumes_exactly():
    """Alg. 3 is r global switches in a row, each a function of the edge list
    and its superstep t only: oracle.run(E, t0, a + b) equals oracle.run on
    the output of oracle.run(E, t0, a), from t0 + a, for b more.  (The
    largest GPU parity check splits the oracle's run at superstep boundaries
    on this identity.)  Checked against the naive replay's single run too."""
    for E, n, seed, pl in [(graphgen.powerlaw_graph(3000, 2.2, 2, 54, 5), 3000, 9, 0),
                           (graphgen.gnp(400, 0.05, 4), 400, 1 << 40, 1 << 30)]:
        rc, full, cf, _ = oracle.run(E, n, seed, 3, 6, pl)
        assert rc == 0
        cur, cs = E, []
        for a, b in [(3, 2), (5, 3), (8, 1)]:
            rc, cur, c, _ = oracle.run(cur, n, seed, a, b, pl)
            assert rc == 0
            cs += c
        assert np.array_equal(cur, full)
        assert cs == cf
    E = graphgen.gnp(60, 0.2, 2)
    En, cn, _ = naive.run([int(x) for x in E], 5, 2, 3, 0)
    cur = E
    for t in (2, 3, 4):
        _, cur, _, _ = oracle.run(cur, 60, 5, t, 1, 0)
    assert [int(x) for x in cur] == En


# ---------------------------------------------------------------------------
# Thm. 3.3: exact transition matrix; chi-square uniformity over G(d)
# ---------------------------------------------------------------------------

def enumerate_gd(deg):
    n = len(deg)
    m = sum(deg) // 2
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n)]
    out = []
    for comb in itertools.combinations(pairs, m):
        d = [0] * n
        for a, b in comb:
            d[a] += 1
            d[b] += 1
        if d == list(deg):
            out.append(tuple(sorted(key(a, b) for a, b in comb)))
    return out


def transition_counts(states, masks=True, mutate=0):
    """counts[s][(A,B)] = #(pi, skip mask with s skips) taking A to B."""
    m = len(states[0])
    ell = m // 2
    idx = {s: i for i, s in enumerate(states)}
    counts = {}
    perms = [np.array(p, dtype=np.uint32) for p in itertools.permutations(range(m))]
    mask_list = [np.array(b, dtype=np.uint8) for b in itertools.product([0, 1], repeat=ell)] if masks else [
        np.zeros(ell, dtype=np.uint8)]
    for A in states:
        E = np.array(A, dtype=np.uint64)
        for pi in perms:
            for mk in mask_list:
                E2, _, _ = oracle.global_switch(E, pi, mk, mutate=mutate)
                B = tuple(sorted(int(x) for x in E2))
                if B not in idx:
                    return None  # left G(d): not a valid transition at all
                k = (int(mk.sum()), idx[A], idx[B])
                counts[k] = counts.get(k, 0) + 1
    return counts


def pin_symmetry(mutate=0):
    ok = True
    for deg, masks in [((1,) * 6, True), ((2,) * 5, True), ((3, 3, 2, 1, 1), True), ((2, 2, 2, 2, 1, 1), False)]:
        states = enumerate_gd(deg)
        c = transition_counts(states, masks, mutate)
        if c is None:
            return False
        for (s, a, b), v in c.items():
            ok &= c.get((s, b, a), 0) == v
    return ok


def test_transition_matrix_symmetric_doubly_stochastic_irreducible():
    assert pin_symmetry()
    deg = (2,) * 5
    states = enumerate_gd(deg)
    assert len(states) == 12  # labelled 5-cycles
    c = transition_counts(states, True)
    m, ell = 5, 2
    pl = 0.3
    P = np.zeros((len(states), len(states)))
    for (s, a, b), v in c.items():
        P[a, b] += v * pl**s * (1 - pl) ** (ell - s) / math.factorial(m)
    assert np.allclose(P.sum(1), 1) and np.allclose(P.sum(0), 1) and np.allclose(P, P.T)
    ncomp, _ = connected_components(csr_matrix(P > 0), directed=True, connection="strong")
    assert ncomp == 1


def chi2_uniform_p(deg, runs, T, mutate=0, pl=1 << 30):
    states = enumerate_gd(deg)
    n = len(deg)
    start = np.array(states[0], dtype=np.uint64)
    cnt = Counter()
    for s in range(runs):
        rc, E, _, _ = oracle.run(start, n, 1000 + s, 0, T, pl, mutate=mutate)
        st = tuple(sorted(int(x) for x in E))
        cnt[st] += 1
    if set(cnt) - set(states):
        return 0.0
    obs = np.array([cnt[s] for s in states])
    return stats.chisquare(obs).pvalue


def pin_uniform(mutate=0):
    # T = 40 supersteps from one fixed start: enough for these tiny chains to
    # mix (the irregular sequence is still visibly non-uniform at T = 12).
    return all(chi2_uniform_p(deg, runs, 40, mutate) > 1e-4 for deg, runs in
               [((1,) * 6, 3000), ((2,) * 5, 3000), ((3, 3, 2, 1, 1), 3000), ((2,) * 6, 7000)])


def test_chi2_uniform_over_gd():
    assert len(enumerate_gd((1,) * 6)) == 15  # perfect matchings on 6 vertices
    assert len(enumerate_gd((2,) * 6)) == 70  # 60 six-cycles + 10 pairs of triangles
    assert pin_uniform()


# ---------------------------------------------------------------------------
# Planted mistakes are caught
# ---------------------------------------------------------------------------

PINS = [pin_fig1, pin_by_hand, pin_invariants, pin_naive, pin_perm_keys_rocrand]


@pytest.mark.parametrize("mut", [oracle.MUT_FLIP_G, oracle.MUT_NO_LOOP, oracle.MUT_NO_EXISTS, oracle.MUT_TAU_SWAP,
                                 oracle.MUT_WRITE_SWAP, oracle.MUT_NO_ERASE, oracle.MUT_PAIR_SHIFT,
                                 oracle.MUT_KEY_SWAP])
def test_planted_mistake_is_caught(mut):
    caught = [p.__name__ for p in PINS if not p(mut)]
    assert caught, "mutation %d passed every pin" % mut

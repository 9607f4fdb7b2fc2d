"""Pins of the ES-MC oracle (the sequential chain that ParES, Alg. 2,
parallelises), each against something other than the oracle itself:

* the draws (i, j, g): exhaustive chi-square uniformity over the 2 m (m - 1)
  triples with i != j (Alg. 2 samples distinct indices), and independence of
  g from i;
* the switch (Def. 2.1): the independent pure-Python replay
  (``oracle/naive.py``), Obs. 2.2 (every accepted switch is undone by one
  switch on the same two positions, a rejected one changes nothing), and
  the degree sequence and simplicity invariants;
* the chain: its exact transition matrix over G(d), enumerated by brute
  force for tiny degree sequences, is symmetric with rows summing to
  2 m (m - 1) and is irreducible; chi-square uniformity of the final state
  over brute-force G(d) after many runs;
* resuming: r1 switches then r2 more from counter k0 + r1 equal r1 + r2.

Every planted mistake (``oracle.MUT_ES_*`` and the switch mutations) fails
at least one pin.
"""
import itertools
from collections import Counter

import numpy as np
import pytest
from scipy import stats
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

import graphgen
import oracle
from oracle import naive
from test_oracle_pins import enumerate_gd, key


# ---------------------------------------------------------------------------
# Draws
# ---------------------------------------------------------------------------

def pin_draws_uniform(mutate=0):
    ok = True
    for m, count in [(2, 20000), (3, 60000), (5, 100000), (7, 150000)]:
        i, j, g = oracle.es_draws(99, 1 << 33, count, m, mutate)
        if (i == j).any() or (i >= m).any() or (j >= m).any():
            return False
        cells = Counter(zip(i.tolist(), j.tolist(), g.tolist()))
        obs = [cells[(a, b, c)] for a in range(m) for b in range(m) if a != b for c in (0, 1)]
        ok &= stats.chisquare(obs).pvalue > 1e-4 and sum(obs) == count
        # g independent of i
        joint = Counter(zip(i.tolist(), g.tolist()))
        tab = np.array([[joint[(a, c)] for c in (0, 1)] for a in range(m)])
        ok &= stats.chi2_contingency(tab).pvalue > 1e-4
    return ok


def pin_draws_naive(mutate=0):
    ok = True
    for seed, k0, m in [(0, 0, 2), (42, 7, 5209), (2**63 + 5, 2**32 - 3, 67125011), (3, 2**40, 1000003)]:
        i, j, g = oracle.es_draws(seed, k0, 40, m, mutate)
        for q in range(40):
            ok &= naive.es_draw(seed, k0 + q, m) == (int(i[q]), int(j[q]), int(g[q]))
    return ok


def test_es_draws_uniform_and_distinct():
    assert pin_draws_uniform()


def test_es_draws_equal_naive():
    assert pin_draws_naive()


# ---------------------------------------------------------------------------
# The switch and the chain against the naive replay
# ---------------------------------------------------------------------------

def es_cases():
    return [(graphgen.gnp(40, 0.15, 1), 40), (graphgen.gnp(12, 0.7, 2), 12),
            (np.array([key(0, v) for v in range(1, 20)], dtype=np.uint64), 20),  # star: every switch rejected
            (graphgen.powerlaw_graph(300, 2.1, 1, 17, 3), 300),
            (np.array([key(0, 1), key(2, 3)], dtype=np.uint64), 4),
            (np.array([key(0, 1), key(2, 3), key(4, 5)], dtype=np.uint64), 6)]


def pin_es_naive(mutate=0):
    ok = True
    for E, n in es_cases():
        for seed, k0, r in [(5, 0, 300), (2**40 + 1, 2**32 - 100, 250)]:
            rc, Eo, c, oc = oracle.es_run(E, n, seed, k0, r, mutate=mutate, outcomes=True)
            En, on = naive.es_run([int(x) for x in E], seed, k0, r)
            ok &= rc == 0 and [int(x) for x in Eo] == En and [int(x) for x in oc] == on
            ok &= c["attempts"] == r and c["legal"] == on.count(naive.LEGAL)
    return ok


def test_es_naive_equals_oracle():
    assert pin_es_naive()


def test_es_star_all_rejected_and_tiny_m():
    E = np.array([key(0, v) for v in range(1, 30)], dtype=np.uint64)
    rc, E2, c, _ = oracle.es_run(E, 30, 3, 0, 1000)
    assert rc == 0 and np.array_equal(E2, E) and c["legal"] == 0 and c["attempts"] == 1000
    for m in (0, 1):
        E = np.array([key(2, 5)] * m, dtype=np.uint64)
        rc, E2, c, _ = oracle.es_run(E, 10, 3, 0, 50)
        assert rc == 0 and np.array_equal(E2, E) and c["attempts"] == 0
    rc, _, _, _ = oracle.es_run(np.array([key(1, 2), key(1, 2)], dtype=np.uint64), 3, 1, 0, 5)
    assert rc == -2


def as_set(E):
    return frozenset(int(x) for x in E)


def pin_es_inverse(mutate=0):
    """Obs. 2.2 on the graph (the edge set): an accepted switch (i, j, g) is
    undone by exactly one of (i, j, 0) and (i, j, 1) -- with edges stored as
    (min, max) the orientation that made (i, j, 0) the inverse is not kept, and
    the two positions may come back exchanged -- and a rejected one leaves E
    exactly as it was.  Checked on the chain's own steps (mutations included)
    and on random switches of the plain switch."""
    rng = np.random.default_rng(4)
    for E, n in es_cases()[:4]:
        m = len(E)
        for _ in range(300):
            i, j = (int(x) for x in rng.choice(m, 2, replace=False))
            g = int(rng.integers(0, 2))
            E2, oc = oracle.edge_switch(E, i, j, g)
            if oc != oracle.LEGAL:
                if not np.array_equal(E2, E):
                    return False
                continue
            back = [as_set(oracle.edge_switch(E2, i, j, h)[0]) == as_set(E) for h in (0, 1)]
            if sum(back) != 1:
                return False
        cur = E
        for k in range(60):  # the chain's steps one at a time
            rc, nxt, c, _ = oracle.es_run(cur, n, 8, k, 1, mutate=mutate)
            if rc != 0:
                return False
            ii, jj, _ = oracle.es_draws(8, k, 1, m, mutate)
            if c["legal"]:
                back = [as_set(oracle.edge_switch(nxt, int(ii[0]), int(jj[0]), h)[0]) == as_set(cur) for h in (0, 1)]
                if sum(back) != 1:
                    return False
            elif not np.array_equal(nxt, cur):
                return False
            cur = nxt
    return True


def test_es_inverse_switch():
    assert pin_es_inverse()


def pin_es_invariants(mutate=0):
    for E, n in es_cases():
        rc, E2, c, _ = oracle.es_run(E, n, 11, 0, 2000, mutate=mutate)
        if rc != 0:
            return False
        u, v = graphgen.split(E2)
        if not ((u < v).all() and len(np.unique(E2)) == len(E2)):
            return False
        if not np.array_equal(graphgen.degrees(E2, n), graphgen.degrees(E, n)):
            return False
        if c["legal"] + c["rej_loop"] + c["rej_exists"] != c["attempts"]:
            return False
    return True


def test_es_invariants():
    assert pin_es_invariants()


def test_es_resumes_exactly():
    for E, n in es_cases()[:4]:
        rc, full, cf, _ = oracle.es_run(E, n, 21, 1000, 900)
        _, a, ca, _ = oracle.es_run(E, n, 21, 1000, 400)
        _, b, cb, _ = oracle.es_run(a, n, 21, 1400, 500)
        assert np.array_equal(b, full)
        assert all(ca[k] + cb[k] == cf[k] for k in cf)


# ---------------------------------------------------------------------------
# The chain: exact transition matrix and uniformity over G(d)
# ---------------------------------------------------------------------------

def es_transition_counts(states, mutate=0):
    """counts[(A, B)] = number of (i, j != i, g) taking edge set A to B, with A
    stored as its sorted edge list (the count does not depend on the order)."""
    m = len(states[0])
    idx = {s: q for q, s in enumerate(states)}
    counts = Counter()
    for A in states:
        E = np.array(A, dtype=np.uint64)
        for i, j in itertools.permutations(range(m), 2):
            for g in (0, 1):
                E2, _ = oracle.edge_switch(E, i, j, g)
                B = tuple(sorted(int(x) for x in E2))
                if B not in idx:
                    return None
                counts[(idx[A], idx[B])] += 1
    return counts


def pin_es_symmetric(mutate=0):
    for deg in [(1,) * 6, (2,) * 5, (3, 3, 2, 1, 1), (2, 2, 2, 2, 1, 1)]:
        states = enumerate_gd(deg)
        m = len(states[0])
        c = es_transition_counts(states, mutate)
        if c is None:
            return False
        for (a, b), v in c.items():
            if c.get((b, a), 0) != v:
                return False
        rows = Counter()
        for (a, b), v in c.items():
            rows[a] += v
        if any(rows[a] != 2 * m * (m - 1) for a in range(len(states))):
            return False
        S = len(states)
        adj = csr_matrix(([1] * len(c), ([a for a, _ in c], [b for _, b in c])), shape=(S, S))
        if connected_components(adj, directed=True, connection="strong")[0] != 1:
            return False
    return True


def test_es_transition_matrix_symmetric_stochastic_irreducible():
    assert pin_es_symmetric()


def chi2_es_p(deg, runs, r, mutate=0):
    states = enumerate_gd(deg)
    n = len(deg)
    start = np.array(states[0], dtype=np.uint64)
    cnt = Counter()
    for s in range(runs):
        rc, E, _, _ = oracle.es_run(start, n, 5000 + s, 0, r, mutate=mutate)
        cnt[tuple(sorted(int(x) for x in E))] += 1
    if set(cnt) - set(states):
        return 0.0
    return stats.chisquare(np.array([cnt[s] for s in states])).pvalue


def pin_es_uniform(mutate=0):
    return all(chi2_es_p(deg, runs, 200, mutate) > 1e-4 for deg, runs in
               [((1,) * 6, 3000), ((2,) * 5, 3000), ((3, 3, 2, 1, 1), 3000), ((2,) * 6, 7000)])


def test_es_chi2_uniform_over_gd():
    assert pin_es_uniform()


# ---------------------------------------------------------------------------
# Planted mistakes are caught
# ---------------------------------------------------------------------------

ES_PINS = [pin_draws_uniform, pin_draws_naive, pin_es_naive, pin_es_inverse, pin_es_invariants, pin_es_uniform]


@pytest.mark.parametrize("mut", [oracle.MUT_ES_J_ANY, oracle.MUT_ES_G_HIGH, oracle.MUT_ES_NO_SKIP,
                                 oracle.MUT_NO_LOOP, oracle.MUT_NO_EXISTS, oracle.MUT_TAU_SWAP,
                                 oracle.MUT_WRITE_SWAP, oracle.MUT_NO_ERASE])
def test_es_planted_mistake_is_caught(mut):
    caught = [p.__name__ for p in ES_PINS if not p(mut)]
    assert caught, "mutation %d passed every pin" % mut

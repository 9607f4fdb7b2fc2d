"""Pins of the graph-class oracle (Sec. 1: directed graphs, graphs with loops,
with multi-edges), each against something other than the oracle itself:

* class 0 is the pinned simple-graph oracle, exactly;
* an independent pure-Python replay (``oracle/naive.py``) for every class;
* switches derived by hand for each class (directed head exchange, a loop
  target, coinciding targets);
* invariants: undirected degrees (a loop counts twice) or directed out- and
  in-degrees are kept, and every state stays in its class (no loop unless
  allowed, no doubled edge unless allowed);
* the exact transition matrix over all permutations (and skip masks) of
  tiny graphs: symmetric (so uniform) for the classes without multi-edges,
  as Thm. 3.3's argument gives, and in detailed balance with the
  configuration model's weight 1 / (prod multiplicity! * 2^loops) for those
  with multi-edges.

Every planted mistake (``oracle.CMUT_*``) fails at least one pin.
"""
import itertools
import math
from collections import Counter

import numpy as np
import pytest

import graphgen
import oracle
from oracle import naive

CLASSES = list(range(8))


def dk(a, b):
    return (a << 32) | b


def uk(a, b):
    return (min(a, b) << 32) | max(a, b)


def random_class_graph(n, m, cls, seed):
    """A random graph of class cls: loops / repeats / antiparallel pairs where allowed."""
    rng = np.random.default_rng(seed)
    out, seen = [], set()
    while len(out) < m:
        a, b = (int(x) for x in rng.integers(0, n, 2))
        if a == b and not (cls & 1):
            continue
        key = dk(a, b) if cls & 4 else uk(a, b)
        if key in seen and not (cls & 2):
            continue
        seen.add(key)
        out.append(key)
    return np.array(out, dtype=np.uint64)


def pin_naive(mutate=0):
    for cls in CLASSES:
        for q, (n, m) in enumerate([(12, 20), (30, 41), (6, 9)]):
            E = random_class_graph(n, m, cls, 10 * cls + q)
            for seed, pl in [(3, 0), (99, 1 << 30)]:
                rc, Eo, co, _ = oracle.run_class(E, n, seed, 2, 6, pl, cls, mutate=mutate)
                En, cn = naive.run_class([int(x) for x in E], seed, 2, 6, pl, cls)
                if rc != 0 or [int(x) for x in Eo] != En or co != cn:
                    return False
    return True


def test_naive_equals_oracle_every_class():
    assert pin_naive()


def test_class0_is_the_simple_oracle():
    for E, n in [(graphgen.gnp(60, 0.1, 3), 60), (graphgen.powerlaw_graph(300, 2.2, 1, 17, 4), 300)]:
        a = oracle.run(E, n, 5, 0, 7, 1 << 29)
        b = oracle.run_class(E, n, 5, 0, 7, 1 << 29, 0)
        assert a[0] == b[0] == 0 and np.array_equal(a[1], b[1]) and a[2] == b[2]


def pin_by_hand(mutate=0):
    """Switches worked out by hand.  In a chain g = [i < j], so each case is
    written with the index order that gives its g and checked both as one
    switch and as the first switch of a one-superstep run whose permutation
    pairs (i, j)."""
    cases = [  # (cls, E, i, j, outcome, E'); g = [i < j]
        (4, [dk(0, 1), dk(2, 3)], 0, 1, oracle.LEGAL, [dk(0, 3), dk(2, 1)]),
        (4, [dk(2, 3), dk(0, 1)], 1, 0, oracle.LEGAL, [dk(2, 1), dk(0, 3)]),      # g has no effect
        (4, [dk(0, 1), dk(1, 2)], 0, 1, oracle.LOOP, [dk(0, 1), dk(1, 2)]),       # (1->1)
        (5, [dk(0, 1), dk(1, 2)], 0, 1, oracle.LEGAL, [dk(0, 2), dk(1, 1)]),
        (0, [uk(0, 2), uk(0, 1)], 1, 0, oracle.LOOP, [uk(0, 2), uk(0, 1)]),       # g = 0: (0,0)
        (1, [uk(0, 2), uk(0, 1)], 1, 0, oracle.LEGAL, [uk(1, 2), uk(0, 0)]),
        (1, [uk(1, 1), uk(0, 0)], 1, 0, oracle.EXISTS, [uk(1, 1), uk(0, 0)]),     # targets (0,1) twice
        (3, [uk(1, 1), uk(0, 0)], 1, 0, oracle.LEGAL, [uk(0, 1), uk(0, 1)]),
        (1, [uk(2, 3), uk(1, 1)], 1, 0, oracle.LEGAL, [uk(1, 3), uk(1, 2)]),
        (1, [uk(1, 1), uk(2, 3)], 0, 1, oracle.LOOP, [uk(1, 1), uk(2, 3)]),       # loop source, g = 1
        (3, [uk(1, 1), uk(2, 3)], 0, 1, oracle.LEGAL, [uk(1, 3), uk(1, 2)]),      # with multi-edges: no rule
        (2, [uk(2, 3), uk(0, 1)], 1, 0, oracle.LEGAL, [uk(1, 3), uk(0, 2)]),
        (0, [uk(0, 1), uk(2, 3), uk(0, 2)], 0, 1, oracle.LEGAL, [uk(0, 3), uk(1, 2), uk(0, 2)]),
        (0, [uk(2, 3), uk(0, 1), uk(0, 2)], 1, 0, oracle.EXISTS, [uk(2, 3), uk(0, 1), uk(0, 2)]),
        (2, [uk(2, 3), uk(0, 1), uk(0, 2)], 1, 0, oracle.LEGAL, [uk(1, 3), uk(0, 2), uk(0, 2)]),
    ]
    for cls, E, i, j, oc, exp in cases:
        E = np.array(E, dtype=np.uint64)
        got, code = oracle.edge_switch_class(E, i, j, int(i < j), cls, mutate)
        if code != oc or [int(x) for x in got] != exp:
            return False
        for t in range(256):  # the same switch as the first of a global switch
            pi = oracle.permutation(len(E), 7, t)
            if (int(pi[0]), int(pi[1])) == (i, j):
                rc, got, _, last = oracle.run_class(E, 4, 7, t, 1, 0, cls, outcomes=True, mutate=mutate)
                if rc != 0 or int(last[0]) != oc:
                    return False
                if len(E) == 2 and [int(x) for x in got] != exp:
                    return False
                break
        else:
            return False
    return True


def test_switches_by_hand():
    assert pin_by_hand()


def degrees(E, n, cls):
    u = (E >> np.uint64(32)).astype(np.int64)
    v = (E & np.uint64(0xFFFFFFFF)).astype(np.int64)
    if cls & 4:
        return np.bincount(u, minlength=n).tolist() + np.bincount(v, minlength=n).tolist()
    return (np.bincount(u, minlength=n) + np.bincount(v, minlength=n)).tolist()


def pin_invariants(mutate=0):
    for cls in CLASSES:
        n = 25
        E = random_class_graph(n, 60, cls, 100 + cls)
        rc, E2, counts, _ = oracle.run_class(E, n, 11, 0, 30, 0, cls, mutate=mutate)
        if rc != 0 or degrees(E2, n, cls) != degrees(E, n, cls):
            return False
        if oracle.validate_class(E2, n, cls) != 0:  # still in its class
            return False
        if not (cls & 4):
            u, v = E2 >> np.uint64(32), E2 & np.uint64(0xFFFFFFFF)
            if not (u <= v).all():
                return False
        for c in counts:
            if c["legal"] + c["rej_loop"] + c["rej_exists"] + c["rej_pl"] != c["attempts"]:
                return False
    return True


def test_invariants_every_class():
    assert pin_invariants()


def transition_counts_class(start, cls, mutate=0):
    """All edge multisets reachable from `start` by global switches, and
    counts[(A, B)] over every pi of its 2..4 edges (with every skip mask)."""
    m = len(start)
    seen, todo, counts = {tuple(sorted(start))}, [tuple(sorted(start))], Counter()
    perms = list(itertools.permutations(range(m)))
    while todo:
        A = todo.pop()
        for pi in perms:
            for mask in itertools.product([0, 1], repeat=m // 2):
                E = np.array(A, dtype=np.uint64)
                for k in range(m // 2):
                    if mask[k]:
                        continue
                    i, j = pi[2 * k], pi[2 * k + 1]
                    E, _ = oracle.edge_switch_class(E, i, j, int(i < j), cls, mutate)
                B = tuple(sorted(int(x) for x in E))
                counts[(A, B)] += 1
                if B not in seen:
                    seen.add(B)
                    todo.append(B)
    return seen, counts


def class_weight(state, cls):
    """The stationary weight the class's chain balances: 1 for classes without
    multi-edges (uniform); the configuration model's 1 / (prod multiplicity!
    * 2^loops) with them (directed: 1 / prod multiplicity!)."""
    if not (cls & 2):
        return 1.0
    w = 1.0
    for c in Counter(state).values():
        w /= math.factorial(c)
    if not (cls & 4):
        w /= 2.0 ** sum(1 for e in state if (e >> 32) == (e & 0xFFFFFFFF))
    return w


def pin_balance(mutate=0):
    """Detailed balance w(A) P(A -> B) = w(B) P(B -> A) over every reachable
    state (Thm. 3.3's symmetry for the classes without multi-edges)."""
    cases = [(0, [uk(0, 1), uk(2, 3), uk(0, 2), uk(1, 3)]), (1, [uk(0, 1), uk(2, 3), uk(1, 1)]),
             (1, [uk(0, 0), uk(1, 2), uk(1, 3), uk(2, 3)]), (4, [dk(0, 1), dk(2, 3), dk(3, 0), dk(1, 2)]),
             (5, [dk(0, 1), dk(1, 2), dk(2, 0)]), (2, [uk(0, 1), uk(0, 1), uk(2, 3), uk(0, 2)]),
             (3, [uk(0, 1), uk(2, 2), uk(0, 3)]), (3, [uk(0, 0), uk(1, 1), uk(0, 1), uk(2, 3)]),
             (6, [dk(0, 1), dk(0, 1), dk(2, 3), dk(1, 0)]), (7, [dk(0, 1), dk(0, 1), dk(1, 0), dk(2, 2)])]
    for cls, start in cases:
        states, c = transition_counts_class(start, cls, mutate)
        for (a, b), v in c.items():
            if abs(class_weight(a, cls) * v - class_weight(b, cls) * c.get((b, a), 0)) > 1e-9:
                return False
    return True


def test_transition_matrix_balanced_every_class():
    assert pin_balance()


PINS = [pin_naive, pin_by_hand, pin_invariants, pin_balance]


@pytest.mark.parametrize("mut", [oracle.CMUT_DIR_TAILS, oracle.CMUT_NO_SAME, oracle.CMUT_LOOPS_ALWAYS,
                                 oracle.CMUT_LOOP_BOTH_G])
def test_class_planted_mistake_is_caught(mut):
    caught = [p.__name__ for p in PINS if not p(mut)]
    assert caught, "mutation %d passed every pin" % mut

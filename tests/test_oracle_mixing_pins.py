"""Pins of the mixing diagnostic's oracle (Sec. 6.1), each against something
other than the oracle itself:

* G^2 equals scipy's log-likelihood statistic of the 2x2 contingency table;
* the thinned transition counts equal a brute-force count over Python sets;
* crafted series with known answers: a constant series is independent at
  every thinning (G^2 = 0); a strictly alternating one is not independent at
  k = 1 (G^2 = 2 N ln 2 > ln N) and constant, so independent, at k = 2;
* i.i.d. Bernoulli series: the fraction flagged matches the chi-square(1)
  tail P(chi2 > ln N) that BIC's threshold implies, within a binomial band;
* a chain whose switches are all rejected (a star) is independent everywhere,
  and a mixing chain is flagged less at larger thinning values.

Every planted mistake (``mixing.MIX_*``) fails at least one pin.
"""
import math

import numpy as np
import pytest
from scipy import stats

import graphgen
from oracle import mixing


def test_g2_equals_scipy_log_likelihood():
    assert pin_g2()


def pin_g2(mutate=0):
    rng = np.random.default_rng(3)
    for _ in range(200):
        t = rng.integers(1, 60, size=(2, 2))
        g = stats.chi2_contingency(t, correction=False, lambda_="log-likelihood")[0]
        if not math.isclose(mixing.g2(t[None], mutate)[0], g, rel_tol=1e-12, abs_tol=1e-12):
            return False
    return True


def random_states(rng, universe, K, p=0.4, size=30):
    return [np.array(sorted(rng.choice(universe, size=size, replace=False)), dtype=np.uint64) for _ in range(K + 1)]


def pin_counts(mutate=0):
    rng = np.random.default_rng(5)
    universe = np.arange(100, 160, dtype=np.uint64)
    for K, k in [(20, 1), (21, 2), (30, 7), (5, 5), (4, 9)]:
        X = random_states(rng, universe, K)
        U, counts, N = mixing.transition_counts(X, k, mutate)
        if N != K // k:
            return False
        sets = [set(int(e) for e in X[j * k]) for j in range(K // k + 1)]
        every = sorted(set().union(*sets))
        if [int(u) for u in U] != every:
            return False
        for q, e in enumerate(every):
            ref = [[0, 0], [0, 0]]
            for j in range(N):
                ref[int(e in sets[j])][int(e in sets[j + 1])] += 1
            if counts[q].tolist() != ref:
                return False
    return True


def test_thinned_counts_brute_force():
    assert pin_counts()


def pin_crafted(mutate=0):
    A = np.array([1, 2, 3], dtype=np.uint64)
    B = np.array([4, 5, 6], dtype=np.uint64)
    K = 40
    const = mixing.diagnostic_of_states([A] * (K + 1), [1, 2, 5], mutate)
    if any(r["non_independent"] != 0 or r["tracked"] != 3 for r in const):
        return False
    alt = mixing.diagnostic_of_states([A if j % 2 == 0 else B for j in range(K + 1)], [1, 2], mutate)
    if alt[0]["non_independent"] != 6 or alt[0]["tracked"] != 6:
        return False
    if alt[1]["tracked"] != 3 or alt[1]["non_independent"] != 0:
        return False
    _, counts, N = mixing.transition_counts([A if j % 2 == 0 else B for j in range(K + 1)], 1, mutate)
    if not math.isclose(mixing.g2(counts[:1], mutate)[0], 2 * N * math.log(2), rel_tol=1e-12):
        return False
    return True


def test_crafted_series():
    assert pin_crafted()


def pin_iid(mutate=0):
    """i.i.d. presence: flagged fraction ~ P(chi2_1 > ln N) (BIC's implied test level)."""
    rng = np.random.default_rng(11)
    E, K = 4000, 400
    Z = rng.random((E, K + 1)) < 0.3
    X = [np.flatnonzero(Z[:, j]).astype(np.uint64) for j in range(K + 1)]
    r = mixing.diagnostic_of_states(X, [1], mutate)[0]
    p = stats.chi2.sf(math.log(K), 1)
    mean, sd = E * p, math.sqrt(E * p * (1 - p))
    return r["tracked"] == E and abs(r["non_independent"] - mean) <= 5 * sd + 3


def test_iid_series_flag_rate():
    assert pin_iid()


def pin_chains(mutate=0):
    star = np.array([(0 << 32) | v for v in range(1, 40)], dtype=np.uint64)
    for chain in ("global", "es"):
        r = mixing.diagnostic(star, 40, 3, 30, [1, 2, 3], chain=chain, mutate=mutate)
        if any(x["non_independent"] != 0 or x["tracked"] != 39 for x in r):
            return False
    E = graphgen.powerlaw_graph(128, 2.2, 1, 11, 4)
    for chain in ("global", "es"):
        r = mixing.diagnostic(E, 128, 9, 120, [1, 8], chain=chain, mutate=mutate)
        if not (r[0]["fraction"] > r[1]["fraction"] and r[0]["tracked"] >= len(E)):
            return False
        for x in r:  # per-edge invariants behind the totals
            tot = np.array(x["counts_total"])
            if tot.sum() != x["N"] * x["tracked"]:
                return False
    return True


def test_star_and_mixing_chains():
    assert pin_chains()


PINS = [pin_g2, pin_counts, pin_crafted, pin_iid, pin_chains]


@pytest.mark.parametrize("mut", [mixing.MIX_NO_FACTOR2, mixing.MIX_SHIFT, mixing.MIX_LOG2, mixing.MIX_MARGINS])
def test_mixing_planted_mistake_is_caught(mut):
    caught = [p.__name__ for p in PINS if not p(mut)]
    assert caught, "mutation %d passed every pin" % mut

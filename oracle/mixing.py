"""ORACLE (test infrastructure only): the autocorrelation mixing diagnostic of
Sec. 6.1, written out from its definition.

Only the tests, the smoke check and the benchmark's CPU baseline may import
this module; the HIP library never does.

What it computes (Sec. 6.1, after Ray, Pinar and Seshadhri's stopping rule):

* run a chain for K supersteps from the input graph X_0, keeping every state
  X_1 .. X_K.  A superstep is one global switch for G-ES-MC (Def. 3.2,
  ``chain="global"``) and floor(m/2) edge switches for ES-MC (Def. 2.1,
  ``chain="es"``, switch counters t*floor(m/2) .. (t+1)*floor(m/2)-1 in
  superstep t), as the paper aligns the two chains;
* for a thinning value k, the k-thinned series samples X_0, X_k, ..., X_{Nk}
  with N = floor(K / k) transitions; the edges tracked are those present in
  at least one sample; edge e has the binary series Z_j = [e in X_{jk}];
* n_ab = #{0 <= j < N : Z_j = a, Z_{j+1} = b} (a, b in {0, 1});
* G^2 = 2 * sum_ab n_ab * ln(n_ab * N / (n_a. * n_.b)) (terms with n_ab = 0
  vanish), the likelihood-ratio statistic of first-order dependence against
  independence of consecutive samples;
* by the Bayesian information criterion the Markov model has one more
  parameter, so e is deemed independent iff G^2 <= ln N;
* reported per k: edges tracked, edges not independent, and their fraction.

Each k is judged on its own, whatever smaller thinning values gave (Sec. 6.1).
"""
from __future__ import annotations

import math

import numpy as np

from . import es_run, run

# Planted mistakes, for tests that show a pin catches them.  0 = the definition.
MIX_NO_FACTOR2 = 1   # G^2 without its factor 2
MIX_SHIFT = 2        # the thinned series samples X_{jk+1} instead of X_{jk}
MIX_LOG2 = 4         # BIC threshold log2(N) instead of ln(N)
MIX_MARGINS = 8      # expected counts from the row margins only


def states(E, n: int, seed: int, K: int, chain: str = "global", pl: int = 0):
    """X_0 .. X_K as uint64 edge-key arrays (position order)."""
    E = np.ascontiguousarray(E, dtype=np.uint64)
    m = len(E)
    ell = m // 2
    out = [E.copy()]
    cur = E
    for t in range(K):
        if chain == "global":
            rc, cur, _, _ = run(cur, n, seed, t, 1, pl)
        elif chain == "es":
            rc, cur, _, _ = es_run(cur, n, seed, t * ell, ell)
        else:
            raise ValueError("chain must be 'global' or 'es'")
        if rc != 0:
            raise ValueError("invalid input graph (status %d)" % rc)
        out.append(cur.copy())
    return out


def transition_counts(X, k: int, mutate: int = 0):
    """For the k-thinned series of the states X: (tracked edge keys sorted,
    counts int64[|U|, 2, 2] with counts[e, a, b] = n_ab, N)."""
    K = len(X) - 1
    N = K // k
    off = 1 if (mutate & MIX_SHIFT) else 0
    if off and N * k + off > K:
        N -= 1
    samples = [np.unique(X[j * k + off]) for j in range(N + 1)]
    U = np.unique(np.concatenate(samples)) if samples else np.zeros(0, dtype=np.uint64)
    Z = np.stack([np.isin(U, s) for s in samples], axis=1)  # |U| x (N + 1)
    counts = np.zeros((len(U), 2, 2), dtype=np.int64)
    if N > 0:
        a, b = Z[:, :-1], Z[:, 1:]
        for x in (0, 1):
            for y in (0, 1):
                counts[:, x, y] = np.sum((a == bool(x)) & (b == bool(y)), axis=1)
    return U, counts, N


def g2(counts, mutate: int = 0):
    """G^2 of each 2x2 table counts[..., a, b] (float64)."""
    c = np.asarray(counts, dtype=np.float64)
    N = c.sum(axis=(-2, -1), keepdims=True)
    row = c.sum(axis=-1, keepdims=True)
    col = c.sum(axis=-2, keepdims=True)
    if mutate & MIX_MARGINS:
        col = N / 2.0
    with np.errstate(divide="ignore", invalid="ignore"):
        term = np.where(c > 0, c * np.log(c * N / (row * col)), 0.0)
    return (1.0 if (mutate & MIX_NO_FACTOR2) else 2.0) * term.sum(axis=(-2, -1))


def decide(counts, N: int, mutate: int = 0):
    """(non-independent flags, G^2 values, borderline flags): an edge is not
    independent iff G^2 > ln N; borderline marks |G^2 - ln N| within 1e-9
    relative, where two correct float64 evaluations may decide differently."""
    G = g2(counts, mutate)
    ln_n = (math.log2(N) if (mutate & MIX_LOG2) else math.log(N)) if N > 0 else 0.0
    non_indep = G > ln_n
    border = np.abs(G - ln_n) <= 1e-9 * max(1.0, ln_n)
    return non_indep, G, border


def diagnostic(E, n: int, seed: int, K: int, thin, chain: str = "global", pl: int = 0, mutate: int = 0):
    """Per thinning value k: dict(k, N, tracked, non_independent, fraction,
    counts_total = sum of n_ab over tracked edges as [[n00, n01], [n10, n11]],
    borderline)."""
    return diagnostic_of_states(states(E, n, seed, K, chain, pl), thin, mutate)


def diagnostic_of_states(X, thin, mutate: int = 0):
    """The diagnostic of a given state sequence X_0 .. X_K (see diagnostic)."""
    out = []
    for k in thin:
        U, counts, N = transition_counts(X, k, mutate)
        if N == 0 or len(U) == 0:
            out.append(dict(k=k, N=N, tracked=int(len(U)), non_independent=0, fraction=0.0,
                            counts_total=[[0, 0], [0, 0]], borderline=0))
            continue
        ni, G, border = decide(counts, N, mutate)
        out.append(dict(k=k, N=N, tracked=int(len(U)), non_independent=int(ni.sum()),
                        fraction=float(ni.sum()) / len(U), counts_total=counts.sum(axis=0).tolist(),
                        borderline=int(border.sum())))
    return out

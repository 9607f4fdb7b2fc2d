"""Batched form (gesmc_run_batch) through the C ABI against the oracle.

A batch has no arithmetic of its own: every graph is an independent chain, so
each graph's slice of the output must equal the oracle run on that graph
alone, bit for bit, together with its outcome counts.
"""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_03005_amd as gesmc
    c = gesmc.Context(0)
    yield c
    c.close()


def to_dev(E):
    return torch.from_numpy(np.ascontiguousarray(E, dtype=np.uint64).view(np.int64).copy()).to("cuda")


def to_host(t):
    return t.cpu().numpy().view(np.uint64)


def key(a, b):
    return (min(a, b) << 32) | max(a, b)


def keys(pairs):
    return np.array([key(a, b) for a, b in pairs], dtype=np.uint64).reshape(-1)


def special_graphs():
    """Degenerate members: empty, one edge, two disjoint edges, odd m, a star
    (every switch shares a vertex), a complete graph (every target exists)."""
    return [
        (np.zeros(0, dtype=np.uint64), 3),
        (keys([(0, 2)]), 3),
        (keys([(0, 1), (2, 3)]), 4),
        (keys([(0, 1), (2, 3), (4, 5)]), 6),
        (keys([(0, v) for v in range(1, 60)]), 60),
        (keys([(a, b) for a in range(12) for b in range(a + 1, 12)]), 12),
    ]


def run_batch(ctx, graphs, seeds, rs, t0s=None, pl=0):
    E, offs, ns = graphgen.concat(graphs)
    print("batch: G=%d total m=%d pl=%d" % (len(graphs), offs[-1], pl), flush=True)
    out, stats, tot = ctx.run_batch(to_dev(E), offs, ns, seeds, rs, t0=t0s, pl=pl)
    return to_host(out), offs, stats, tot


def check_against_oracle(graphs, got, offs, stats, seeds, rs, t0s, pl, ids):
    for g in ids:
        E, n = graphs[g]
        t0 = 0 if t0s is None else t0s[g]
        rc, exp, counts, _ = oracle.run(E, n, seeds[g], t0, rs[g], pl)
        assert rc == 0
        sl = got[offs[g]:offs[g + 1]]
        diff = np.flatnonzero(sl != exp)
        assert diff.size == 0, "graph %d (m=%d n=%d r=%d): %d positions differ" % (g, len(E), n, rs[g], diff.size)
        s = stats[g]
        assert s["attempts"] == sum(c["attempts"] for c in counts), g
        for k in ("legal", "rej_loop", "rej_exists", "rej_pl"):
            assert s[k] == sum(c[k] for c in counts), (g, k, s)


def mixed_batch(seed=7, G=40):
    graphs = graphgen.batch_graphs(G, seed, 1e2, 3e3) + special_graphs()
    rng = np.random.default_rng(seed)
    seeds = [int(x) for x in rng.integers(0, 2**63, len(graphs))]
    rs = [int(x) for x in rng.integers(0, 7, len(graphs))]
    t0s = [int(x) for x in rng.integers(0, 1000, len(graphs))]
    return graphs, seeds, rs, t0s


@pytest.mark.parametrize("pl", [0, 1 << 30])
def test_mixed_batch_exact(ctx, pl):
    graphs, seeds, rs, t0s = mixed_batch()
    got, offs, stats, tot = run_batch(ctx, graphs, seeds, rs, t0s, pl)
    check_against_oracle(graphs, got, offs, stats, seeds, rs, t0s, pl, range(len(graphs)))
    assert tot["attempts"] == sum(s["attempts"] for s in stats)
    assert tot["legal"] == sum(s["legal"] for s in stats)


def test_batch_shrinking_prefix_exact(ctx):
    """Graphs large enough for the radix pipeline (not the LDS chain) with r
    from 1 to 6, so the switched prefix of ranks shrinks from step to step;
    each step's first radix level is counted by the previous step's first
    decision round for the next (smaller) prefix.  Every graph exact."""
    graphs = graphgen.batch_graphs(12, 31, 1e4, 6e4)
    assert all(len(E) > 6144 for E, _ in graphs)
    rng = np.random.default_rng(31)
    seeds = [int(x) for x in rng.integers(0, 2**63, len(graphs))]
    rs = [1 + g % 6 for g in range(len(graphs))]
    t0s = [int(x) for x in rng.integers(0, 100, len(graphs))]
    got, offs, stats, _ = run_batch(ctx, graphs, seeds, rs, t0s)
    check_against_oracle(graphs, got, offs, stats, seeds, rs, t0s, 0, range(len(graphs)))


def test_batch_equals_single_runs(ctx):
    """Each graph's result is the same alone (gesmc_run) and in the mix."""
    graphs, seeds, rs, t0s = mixed_batch(seed=11, G=24)
    got, offs, _, _ = run_batch(ctx, graphs, seeds, rs, t0s)
    for g, (E, n) in enumerate(graphs):
        out, _ = ctx.run(to_dev(E), n, seeds[g], t0=t0s[g], r=rs[g])
        assert np.array_equal(to_host(out), got[offs[g]:offs[g + 1]]), g


def test_batch_order_and_company_do_not_matter(ctx):
    """Reordering the batch and dropping members leaves every result unchanged."""
    graphs, seeds, rs, t0s = mixed_batch(seed=13, G=30)
    got, offs, _, _ = run_batch(ctx, graphs, seeds, rs, t0s)
    perm = np.random.default_rng(5).permutation(len(graphs))[: len(graphs) // 2]
    sub = [graphs[g] for g in perm]
    got2, offs2, _, _ = run_batch(ctx, sub, [seeds[g] for g in perm], [rs[g] for g in perm],
                                  [t0s[g] for g in perm])
    for j, g in enumerate(perm):
        assert np.array_equal(got2[offs2[j]:offs2[j + 1]], got[offs[g]:offs[g + 1]]), g


def test_batch_schedule_independence(ctx):
    """Bucket sizes, the LDS capacity (incl. the slow exact paths) and the
    number of multi-workgroup rounds never change the result."""
    import paper_2111_03005_amd as gesmc
    graphs, seeds, rs, t0s = mixed_batch(seed=17, G=32)
    ref = None
    for avg, cap, fr in [(512, 1024, 2), (64, 1024, 0), (64, 64, 1), (768, 96, 4)]:
        c = gesmc.Context(0)
        try:
            c.set_option(gesmc.OPT_BUCKET_AVG, avg)
            c.set_option(gesmc.OPT_SORT_CAP, cap)
            c.set_option(gesmc.OPT_FAST_ROUNDS, fr)
            got, offs, stats, _ = run_batch(c, graphs, seeds, rs, t0s)
            if ref is None:
                ref = got
                check_against_oracle(graphs, got, offs, stats, seeds, rs, t0s, 0, range(len(graphs)))
            assert np.array_equal(got, ref), (avg, cap, fr)
        finally:
            c.close()


def test_batch_invalid_inputs(ctx):
    import paper_2111_03005_amd as gesmc
    good = graphgen.batch_graphs(5, 3, 1e2, 1e3)
    # (position in the batch, edges, n, r, status, message names the graph)
    cases = [
        (3, keys([(0, 1), (1, 2), (0, 1)]), 3, 2, gesmc.E_NOT_SIMPLE, True),    # duplicate, switched graph
        (3, keys([(0, 1), (1, 2), (0, 1)]), 3, 0, gesmc.E_NOT_SIMPLE, True),    # duplicate, graph with r = 0
        (1, np.array([(2 << 32) | 2, key(0, 1)], dtype=np.uint64), 3, 2, gesmc.E_NOT_SIMPLE, True),  # loop
        (4, keys([(0, 1), (1, 7)]), 5, 1, gesmc.E_RANGE, True),                 # id >= n of its graph
    ]
    for pos, E, n, r, code, named in cases:
        graphs = list(good)
        graphs.insert(pos, (E, n))
        E_all, offs, ns = graphgen.concat(graphs)
        sentinel = torch.full((len(E_all),), 777, dtype=torch.int64, device="cuda")
        with pytest.raises(gesmc.GesmcError) as ei:
            ctx.run_batch(to_dev(E_all), offs, ns, [1] * len(graphs), [r if g == pos else 2 for g in
                                                                       range(len(graphs))], out=sentinel)
        assert ei.value.status == code, (pos, r, ei.value)
        if named:
            assert ("graph %d" % pos) in str(ei.value), str(ei.value)
        assert (sentinel.cpu() == 777).all()
    # the context stays usable
    graphs, seeds, rs, t0s = mixed_batch(seed=19, G=8)
    got, offs, stats, _ = run_batch(ctx, graphs, seeds, rs, t0s)
    check_against_oracle(graphs, got, offs, stats, seeds, rs, t0s, 0, range(len(graphs)))


def test_batch_argument_checks(ctx):
    import paper_2111_03005_amd as gesmc
    E, offs, ns = graphgen.concat(special_graphs())
    d = to_dev(E)
    with pytest.raises(gesmc.GesmcError) as ei:  # offsets must start at 0
        ctx.run_batch(d, [1] + list(offs[1:]), ns, [1] * len(ns), [1] * len(ns))
    assert ei.value.status == gesmc.E_INVAL
    with pytest.raises(gesmc.GesmcError) as ei:  # decreasing offsets
        bad = list(offs)
        bad[2], bad[3] = bad[3], bad[2]
        ctx.run_batch(d, bad, ns, [1] * len(ns), [1] * len(ns))
    assert ei.value.status == gesmc.E_INVAL
    c = gesmc.Context(0)
    try:
        c.set_option(gesmc.OPT_STRATEGY, gesmc.STRATEGY_HBM_TABLE)
        with pytest.raises(gesmc.GesmcError) as ei:
            c.run_batch(d, offs, ns, [1] * len(ns), [1] * len(ns))
        assert ei.value.status == gesmc.E_INVAL
    finally:
        c.close()


def oracle_pool(graphs, seeds, rs, t0s=None, pl=0, ids=None):
    """oracle.run of the given graphs, one graph per task on a thread pool
    (the oracle's C calls release the GIL): {g: (status, E', counts)}."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    ids = list(range(len(graphs))) if ids is None else list(ids)
    oracle._load()

    def one(g):
        E, n = graphs[g]
        rc, exp, counts, _ = oracle.run(E, n, seeds[g], 0 if t0s is None else t0s[g], rs[g], pl)
        return g, (rc, exp, counts)

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return dict(ex.map(one, ids))


def test_full_batch_4096_exact(ctx):
    """The 4096-graph workload at full size, 20 global switches each, in the
    benchmark's configuration: every graph exactly against the oracle (its
    edge list in position order and its outcome counts)."""
    graphs = graphgen.workload_batch_4096()
    G = len(graphs)
    seeds = [42 + g for g in range(G)]
    rs = [20] * G
    got, offs, stats, tot = run_batch(ctx, graphs, seeds, rs)
    exp = oracle_pool(graphs, seeds, rs)
    bad = []
    for g in range(G):
        rc, e, counts = exp[g]
        assert rc == 0
        if not np.array_equal(got[offs[g]:offs[g + 1]], e):
            bad.append(g)
            continue
        s = stats[g]
        assert s["attempts"] == sum(c["attempts"] for c in counts), g
        for k in ("legal", "rej_loop", "rej_exists", "rej_pl"):
            assert s[k] == sum(c[k] for c in counts), (g, k, s)
    assert not bad, "%d graphs differ, first %s" % (len(bad), bad[:5])
    sizes = np.diff(offs)
    assert tot["attempts"] == sum(20 * (s // 2) for s in sizes)


def test_large_batch_graph_local_tags_sampled_exact(ctx):
    """512 power-law graphs, four copies of a pool of 128 with n log-uniform in
    [1e3, 1e6] (about 2e8 edges): batch-wide switch ids no longer fit the packed
    tuple word, so the tags are local to each graph and the tuples stay 8 bytes.
    Every 16th graph against the oracle."""
    pool = graphgen.batch_graphs(128, 5, 1e3, 1e6)
    graphs = pool * 4
    G = len(graphs)
    seeds = [1000 + g for g in range(G)]
    rs = [3] * G
    got, offs, stats, tot = run_batch(ctx, graphs, seeds, rs)
    assert tot["tuple_bytes"] == 8, tot
    ids = list(range(0, G, 16))
    exp = oracle_pool(graphs, seeds, rs, ids=ids)
    for g in ids:
        rc, e, counts = exp[g]
        assert rc == 0
        assert np.array_equal(got[offs[g]:offs[g + 1]], e), g
        for k in ("legal", "rej_loop", "rej_exists"):
            assert stats[g][k] == sum(c[k] for c in counts), (g, k)


def test_autotuned_batch_computes_the_same():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_03005_amd as gesmc
    graphs, seeds, rs, t0s = mixed_batch(seed=23, G=20)
    E, offs, ns = graphgen.concat(graphs)
    gesmc.tune_cache_clear()
    c = gesmc.Context(0)
    try:
        tu = c.autotune_batch(to_dev(E), offs, ns, seeds, supersteps=2)
        print("tuning:", tu, flush=True)
        assert tu["candidates"] == 8
        again = c.autotune_batch(to_dev(E), offs, ns, seeds, supersteps=2)  # same device and shape class
        assert again["candidates"] == 0
        assert {k: again[k] for k in ("bucket_avg", "level1_bits", "fuse_emit")} == \
            {k: tu[k] for k in ("bucket_avg", "level1_bits", "fuse_emit")}
        got, offs, stats, _ = run_batch(c, graphs, seeds, rs, t0s)
        check_against_oracle(graphs, got, offs, stats, seeds, rs, t0s, 0, range(len(graphs)))
    finally:
        c.close()


def test_batch_graph_capture_and_replay():
    """GESMC_OPT_GRAPH: the second call of a shape is captured into a hipGraph
    and later calls replay it with new seeds.  Every replay is checked against
    the oracle, with eager work of other shapes on the same context in between."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_03005_amd as gesmc
    graphs, seeds, rs, t0s = mixed_batch(seed=29, G=24)
    other, o_seeds, o_rs, o_t0s = mixed_batch(seed=31, G=6)
    E, offs, ns = graphgen.concat(graphs)
    c = gesmc.Context(0)
    stream = torch.cuda.Stream()
    try:
        c.set_option(gesmc.OPT_GRAPH, 1)
        c.set_option(gesmc.OPT_PROFILE, 1)
        d_in = to_dev(E)
        out = torch.empty_like(d_in)
        for rep in range(5):
            seeds_rep = [s + 1000003 * rep for s in seeds]
            with torch.cuda.stream(stream):
                out, stats, _ = c.run_batch(d_in, offs, ns, seeds_rep, rs, t0=t0s, out=out, stream=stream)
            stream.synchronize()
            check_against_oracle(graphs, to_host(out), offs, stats, seeds_rep, rs, t0s, 0, range(len(graphs)))
            if rep == 2:  # eager work of another shape between replays
                got, o_offs, o_stats, _ = run_batch(c, other, o_seeds, o_rs, o_t0s)
                check_against_oracle(other, got, o_offs, o_stats, o_seeds, o_rs, o_t0s, 0, range(len(other)))
        # launches timed by events happen only in eager calls: the first call of the
        # captured shape and the eager call of the other shape (and, if that call
        # moved buffers, one more eager call of the first shape)
        loads = c.profile()["k_load"][1]
        assert loads <= 3, loads
    finally:
        c.close()


def small_batch(seed=37):
    """Graphs around the LDS-resident size limits (1024 edges on 256 threads,
    4096 on 1024, 6144 on 1024 with vertex ids below 2^16): G(n,p) graphs
    cut to exactly 1023, 1024, 1025, 4095, 4096, 4097, 6143, 6144 and 6145
    edges, one of 5000 edges whose ids exceed 2^16, dense ones where most
    targets exist, and small power-law graphs, with long chains (up to 40
    global switches) so that many supersteps run inside one workgroup."""
    rng = np.random.default_rng(seed)
    graphs = []
    for m in (1023, 1024, 1025):
        E = graphgen.gnp(300, 0.03, seed + m)
        assert len(E) >= m
        graphs.append((np.sort(E[:m]), 300))
    for m in (4095, 4096, 4097, 6143, 6144, 6145):
        E = graphgen.gnp(900, 0.02, seed + m)
        assert len(E) >= m
        graphs.append((np.sort(E[:m]), 900))
    # ids above 2^16: the compact class does not apply, the multi-kernel path runs
    E = graphgen.gnp(900, 0.02, seed + 9)[:5000]
    graphs.append(((E + np.uint64((70000 << 32) | 70000)).astype(np.uint64), 71000))
    graphs.append((graphgen.gnp(40, 0.9, seed + 1), 40))
    graphs.append((graphgen.gnp(48, 0.85, seed + 2), 48))
    graphs += graphgen.batch_graphs(24, seed, 20, 400)
    graphs += special_graphs()
    seeds = [int(x) for x in rng.integers(0, 2**63, len(graphs))]
    rs = [int(x) for x in rng.integers(0, 41, len(graphs))]
    t0s = [int(x) for x in rng.integers(0, 1 << 20, len(graphs))]
    return graphs, seeds, rs, t0s


@pytest.mark.parametrize("pl", [0, 1 << 31])
def test_small_graph_path_exact(pl):
    """GESMC_OPT_SMALL_GRAPHS: graphs of at most 4096 edges (6144 with ids
    below 2^16) run every superstep in one LDS-resident workgroup.  With the option on and off the
    results and counts are identical and equal the oracle's."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_03005_amd as gesmc
    graphs, seeds, rs, t0s = small_batch()
    res = []
    for on in (1, 0):
        c = gesmc.Context(0)
        try:
            c.set_option(gesmc.OPT_SMALL_GRAPHS, on)
            got, offs, stats, tot = run_batch(c, graphs, seeds, rs, t0s, pl)
            res.append((got, stats, tot))
        finally:
            c.close()
    check_against_oracle(graphs, res[0][0], offs, res[0][1], seeds, rs, t0s, pl, range(len(graphs)))
    assert np.array_equal(res[0][0], res[1][0])
    outcome = ("attempts", "legal", "rej_loop", "rej_exists", "rej_pl", "supersteps")
    for g in range(len(graphs)):  # rounds and times depend on the schedule, outcomes do not
        assert all(res[0][1][g][k] == res[1][1][g][k] for k in outcome), g
    for k in outcome[:5]:
        assert res[0][2][k] == res[1][2][k], k

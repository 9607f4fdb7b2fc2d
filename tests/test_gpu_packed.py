"""Packed 8-byte dependency tuples (GESMC_OPT_PACK_TUPLES) through the C ABI.

The tuple layout is a schedule choice: with packing on or off every output
edge and every per-superstep count must equal the oracle's, bit for bit.
The cases cover the LDS resolve and its exact slow path (hub keys, small
sort capacities), both radix level splits, odd m and P_L, the word filled
to exactly 64 bits, one bit too many (12-byte fallback), and in batches the
per-graph attribution of a duplicate edge (whose vertex the packed word
recovers by inverting the key hash) and graph-local tags (forced with
option value 2, and where batch-wide switch ids no longer fit the word).
"""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def to_dev(E):
    return torch.from_numpy(np.ascontiguousarray(E, dtype=np.uint64).view(np.int64).copy()).to("cuda")


def to_host(t):
    return t.cpu().numpy().view(np.uint64)


def key(a, b):
    return (min(a, b) << 32) | max(a, b)


def keys(pairs):
    return np.array([key(a, b) for a, b in pairs], dtype=np.uint64).reshape(-1)


def random_simple(n, m, seed):
    """m distinct random edges on [0, n) (most vertices isolated for large n)."""
    rng = np.random.default_rng(seed)
    out = set()
    while len(out) < m:
        u = rng.integers(0, n, 2 * m, dtype=np.uint64)
        v = rng.integers(0, n, 2 * m, dtype=np.uint64)
        for a, b in zip(u.tolist(), v.tolist()):
            if a != b and len(out) < m:
                out.add(key(a, b))
    E = np.array(sorted(out), dtype=np.uint64)
    rng.shuffle(E)
    return E


COUNT_KEYS = ("attempts", "legal", "rej_loop", "rej_exists", "rej_pl")


def run_both(E, n, seed, t0, r, pl=0, options=(), label=""):
    """Runs with packing on and off; both must equal the oracle.  Returns the
    tuple sizes reported (packing on, packing off)."""
    import paper_2111_03005_amd as gesmc
    print("case %s: m=%d n=%d r=%d pl=%d options=%s" % (label, len(E), n, r, pl, options), flush=True)
    rc, exp, counts, _ = oracle.run(E, n, seed, t0, r, pl)
    assert rc == 0
    sizes = []
    for pack in (1, 0):
        c = gesmc.Context(0)
        try:
            c.set_option(gesmc.OPT_PACK_TUPLES, pack)
            for opt, val in options:
                c.set_option(opt, val)
            out, st, steps = c.run(to_dev(E), n, seed, t0=t0, r=r, pl=pl, steps=True)
            got = to_host(out)
            diff = np.flatnonzero(got != exp)
            assert diff.size == 0, "%s pack=%d: %d positions differ, first %s" % (label, pack, diff.size, diff[:5])
            for q, (s, cnt) in enumerate(zip(steps, counts)):
                for k in COUNT_KEYS:
                    assert s[k] == cnt[k], (label, pack, q, k)
            sizes.append(st["tuple_bytes"])
        finally:
            c.close()
    assert sizes[1] == 12, (label, sizes)
    return sizes[0]


def test_packed_small_and_powerlaw():
    _require_gpu()
    import paper_2111_03005_amd as gesmc
    E, n = graphgen.workload_gnp_small()
    assert run_both(E, n, 42, 0, 10, label="gnp_n1024_d10") == 8
    E = graphgen.powerlaw_graph(40000, 2.05, 1, 400, 21)
    assert run_both(E, 40000, 77, 2, 5, label="pld40000") == 8
    assert run_both(E, 40000, 78, 0, 3, pl=1 << 30, label="pld40000_pl") == 8
    # odd m: the idle position's STAYS tuple
    assert run_both(E[:-1], 40000, 79, 0, 3, label="pld40000_odd") == 8
    # small LDS capacities send partitions to the exact slow path; level splits
    for opts in ([(gesmc.OPT_SORT_CAP, 64)], [(gesmc.OPT_BUCKET_AVG, 96), (gesmc.OPT_SORT_CAP, 128)],
                 [(gesmc.OPT_LEVEL1_BITS, 1)], [(gesmc.OPT_LEVEL1_BITS, 10), (gesmc.OPT_BUCKET_AVG, 64)]):
        assert run_both(E, 40000, 80, 0, 2, options=opts, label="pld40000_opts") == 8


def test_packed_hub_keys_slow_path():
    """Thousands of inserters of one target key: partitions above the LDS
    capacity take the exact merge over packed words."""
    _require_gpu()
    n = 4000
    E = keys([(a, b) for a in range(6) for b in range(6, n) if (a + b) % 3 != 0])
    assert run_both(E, n, 3, 0, 3, label="hubs") == 8
    assert run_both(E, n, 4, 0, 2, pl=1 << 31, label="hubs_pl") == 8


def test_packed_word_exactly_full_and_one_bit_over():
    """n = 2^25, m = 65536: 50 hash bits, 4 of them dropped by the first
    level, an 18-bit tag code -- exactly 64 bits, packed.  n = 2^26: 66 bits,
    the 12-byte layout."""
    _require_gpu()
    E = random_simple(1 << 25, 65536, 5)
    assert run_both(E, 1 << 25, 11, 0, 3, label="full_word") == 8
    E = random_simple(1 << 26, 65536, 6)
    assert run_both(E, 1 << 26, 12, 0, 3, label="one_bit_over") == 12
    E = random_simple((1 << 31) + 5, 2000, 7)
    assert run_both(E, (1 << 31) + 5, 13, 0, 2, label="wide_ids") == 12


@pytest.mark.parametrize("pack", [1, 0, 2])
def test_packed_batch_and_duplicate_attribution(pack):
    """Multi-kernel batch supersteps (the LDS small-graph path off) with and
    without packing, and with graph-local tags (2), equal the oracle per
    graph; a duplicate edge in one graph is reported for that graph."""
    _require_gpu()
    import paper_2111_03005_amd as gesmc
    graphs = graphgen.batch_graphs(12, 41, 1e2, 2e4)
    rng = np.random.default_rng(3)
    seeds = [int(x) for x in rng.integers(0, 2**63, len(graphs))]
    rs = [int(x) for x in rng.integers(1, 6, len(graphs))]
    E_all, offs, ns = graphgen.concat(graphs)
    c = gesmc.Context(0)
    try:
        c.set_option(gesmc.OPT_PACK_TUPLES, pack)
        c.set_option(gesmc.OPT_SMALL_GRAPHS, 0)
        print("batch pack=%d: G=%d total m=%d" % (pack, len(graphs), offs[-1]), flush=True)
        out, stats, tot = c.run_batch(to_dev(E_all), offs, ns, seeds, rs)
        got = to_host(out)
        assert tot["tuple_bytes"] == (8 if pack else 12), tot
        for g, (E, n) in enumerate(graphs):
            rc, exp, counts, _ = oracle.run(E, n, seeds[g], 0, rs[g])
            assert rc == 0
            assert np.array_equal(got[offs[g]:offs[g + 1]], exp), g
            assert stats[g]["legal"] == sum(x["legal"] for x in counts), g
        for pos in (0, 5, len(graphs)):
            bad = list(graphs)
            E, n = graphs[min(pos, len(graphs) - 1)]
            dup = np.concatenate([E, E[len(E) // 2: len(E) // 2 + 1]])
            bad.insert(pos, (dup, n))
            Eb, ob, nb = graphgen.concat(bad)
            sentinel = torch.full((len(Eb),), 777, dtype=torch.int64, device="cuda")
            print("duplicate in graph %d" % pos, flush=True)
            with pytest.raises(gesmc.GesmcError) as ei:
                c.run_batch(to_dev(Eb), ob, nb, [1] * len(bad), [2] * len(bad), out=sentinel)
            assert ei.value.status == gesmc.E_NOT_SIMPLE
            assert ("graph %d" % pos) in str(ei.value), str(ei.value)
            assert (sentinel.cpu() == 777).all()
    finally:
        c.close()


def test_packed_batch_graph_replay_with_wider_ids():
    """hipGraph replay: the tuple layout depends on the vertex id width, so a
    call whose n grows past a power of two must not replay a graph captured
    for narrower ids."""
    _require_gpu()
    import paper_2111_03005_amd as gesmc
    graphs = graphgen.batch_graphs(6, 43, 2e3, 2e4)
    rng = np.random.default_rng(9)
    seeds = [int(x) for x in rng.integers(0, 2**63, len(graphs))]
    rs = [3] * len(graphs)
    E_all, offs, ns = graphgen.concat(graphs)
    c = gesmc.Context(0)
    stream = torch.cuda.Stream()
    try:
        c.set_option(gesmc.OPT_GRAPH, 1)
        c.set_option(gesmc.OPT_SMALL_GRAPHS, 0)
        d_in = to_dev(E_all)
        out = torch.empty_like(d_in)
        for rep, widen in enumerate([0, 0, 0, 1, 1, 0]):
            ns_rep = list(ns)
            if widen:  # graph 0's range grows: every later graph's ids move past 2^26
                ns_rep[0] = ns[0] + (1 << 26)
            print("replay %d widen=%d" % (rep, widen), flush=True)
            with torch.cuda.stream(stream):
                out, stats, tot = c.run_batch(d_in, offs, ns_rep, seeds, rs, out=out, stream=stream)
            stream.synchronize()
            got = to_host(out)
            for g, (E, n) in enumerate(graphs):
                rc, exp, _, _ = oracle.run(E, ns_rep[g], seeds[g], 0, rs[g])
                assert rc == 0
                assert np.array_equal(got[offs[g]:offs[g + 1]], exp), (rep, g)
    finally:
        c.close()


def test_packed_batch_wide_vertex_range():
    """600 sparse graphs of 10^5 vertices: ids need 26 bits, offsets v - u
    only 17, so the (u, v - u) coding packs (57 bits) where two 26-bit ids
    would not (66).  Every graph equals the oracle."""
    _require_gpu()
    import paper_2111_03005_amd as gesmc
    graphs = [(random_simple(100000, 200, 100 + g), 100000) for g in range(600)]
    rng = np.random.default_rng(11)
    seeds = [int(x) for x in rng.integers(0, 2**63, len(graphs))]
    rs = [int(x) for x in rng.integers(1, 5, len(graphs))]
    E_all, offs, ns = graphgen.concat(graphs)
    c = gesmc.Context(0)
    try:
        c.set_option(gesmc.OPT_SMALL_GRAPHS, 0)
        print("wide batch: G=%d total m=%d" % (len(graphs), offs[-1]), flush=True)
        out, stats, tot = c.run_batch(to_dev(E_all), offs, ns, seeds, rs)
        assert tot["tuple_bytes"] == 8, tot
        got = to_host(out)
        for g, (E, n) in enumerate(graphs):
            rc, exp, counts, _ = oracle.run(E, n, seeds[g], 0, rs[g])
            assert rc == 0
            assert np.array_equal(got[offs[g]:offs[g + 1]], exp), g
            for k in ("legal", "rej_loop", "rej_exists"):
                assert stats[g][k] == sum(x[k] for x in counts), (g, k)
    finally:
        c.close()


def check_batch(c, graphs, seeds, rs, tuple_bytes, label):
    E_all, offs, ns = graphgen.concat(graphs)
    print("%s: G=%d total m=%d" % (label, len(graphs), offs[-1]), flush=True)
    out, stats, tot = c.run_batch(to_dev(E_all), offs, ns, seeds, rs)
    assert tot["tuple_bytes"] == tuple_bytes, (label, tot)
    got = to_host(out)
    for g, (E, n) in enumerate(graphs):
        rc, exp, counts, _ = oracle.run(E, n, seeds[g], 0, rs[g])
        assert rc == 0
        assert np.array_equal(got[offs[g]:offs[g + 1]], exp), (label, g)
        for k in ("legal", "rej_loop", "rej_exists"):
            assert stats[g][k] == sum(x[k] for x in counts), (label, g, k)


def test_packed_batch_graph_local_tags_natural():
    """16 sparse graphs of 2^24 vertices, 20000 edges each: 52 hash bits, and
    batch-wide switch ids (19-bit codes) would need 67 bits, so the batch
    packs with tags local to each graph (15-bit codes, 63 bits) instead of
    falling back to 12-byte tuples.  Every graph equals the oracle."""
    _require_gpu()
    import paper_2111_03005_amd as gesmc
    graphs = [(random_simple(1 << 24, 20000, 300 + g), 1 << 24) for g in range(16)]
    rng = np.random.default_rng(13)
    seeds = [int(x) for x in rng.integers(0, 2**63, len(graphs))]
    rs = [int(x) for x in rng.integers(1, 4, len(graphs))]
    c = gesmc.Context(0)
    try:
        c.set_option(gesmc.OPT_SMALL_GRAPHS, 0)
        check_batch(c, graphs, seeds, rs, 8, "local tags")
    finally:
        c.close()


def test_packed_batch_graph_local_tags_hubs_slow_path():
    """Graph-local tags through the exact slow path: hub graphs (thousands of
    inserters of one key) beside power-law graphs, with small LDS capacities,
    in one batch; every graph equals the oracle."""
    _require_gpu()
    import paper_2111_03005_amd as gesmc
    hub = keys([(a, b) for a in range(6) for b in range(6, 3000) if (a + b) % 3 != 0])
    graphs = [(hub, 3000), (graphgen.powerlaw_graph(20000, 2.05, 1, 300, 5), 20000), (hub, 3000),
              (graphgen.powerlaw_graph(5000, 2.3, 2, 70, 6), 5000)]
    seeds = [5, 6, 7, 8]
    rs = [3, 2, 3, 1]
    for opts in ([], [(gesmc.OPT_SORT_CAP, 64)], [(gesmc.OPT_BUCKET_AVG, 96), (gesmc.OPT_SORT_CAP, 128)]):
        c = gesmc.Context(0)
        try:
            c.set_option(gesmc.OPT_SMALL_GRAPHS, 0)
            c.set_option(gesmc.OPT_PACK_TUPLES, 2)
            for opt, val in opts:
                c.set_option(opt, val)
            check_batch(c, graphs, seeds, rs, 8, "local tags hubs %s" % (opts,))
        finally:
            c.close()

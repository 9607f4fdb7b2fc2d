"""Parity of the HIP path (through the C ABI) with the oracle, bit for bit.

Everything here is integer work, so the bar is exact equality: the output
edge list in position order, every per-superstep count, the per-switch
outcome codes, the permutation keys and the permutation itself.
"""
import os
import tempfile

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


STRATEGIES = {"sorted-tuples": 0, "hbm-table": 1}


@pytest.fixture(scope="module", params=list(STRATEGIES), ids=list(STRATEGIES))
def ctx(request):
    """A context per dependency-resolution strategy; results must not depend on it."""
    _require_gpu()
    import paper_2111_03005_amd as gesmc
    c = gesmc.Context(0)
    c.set_option(gesmc.OPT_STRATEGY, STRATEGIES[request.param])
    yield c
    c.close()


_ORACLE_CACHE = {}


def oracle_run(E, n, seed, t0, r, pl=0, outcomes=False):
    """oracle.run, memoised per input content (full-size runs take seconds)."""
    key = (E.tobytes().__hash__(), len(E), n, seed, t0, r, pl, outcomes)
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = oracle.run(E, n, seed, t0, r, pl, outcomes=outcomes)
    return _ORACLE_CACHE[key]


def to_dev(E):
    return torch.from_numpy(np.ascontiguousarray(E, dtype=np.uint64).view(np.int64).copy()).to("cuda")


def to_host(t):
    return t.cpu().numpy().view(np.uint64)


def key(a, b):
    return (min(a, b) << 32) | max(a, b)


def keys(pairs):
    return np.array([key(a, b) for a, b in pairs], dtype=np.uint64)


COUNT_KEYS = ("attempts", "legal", "rej_loop", "rej_exists", "rej_pl")


def check_run(ctx, E, n, seed, t0, r, pl=0, label=""):
    print("case %s: m=%d n=%d seed=%d t0=%d r=%d pl=%d" % (label, len(E), n, seed, t0, r, pl), flush=True)
    out, st, steps = ctx.run(to_dev(E), n, seed, t0=t0, r=r, pl=pl, steps=True)
    got = to_host(out)
    rc, exp, counts, _ = oracle_run(E, n, seed, t0, r, pl)
    assert rc == 0
    diff = np.flatnonzero(got != exp)
    assert diff.size == 0, "%s: %d positions differ, first %s" % (label, diff.size, diff[:5])
    for q, (s, c) in enumerate(zip(steps, counts)):
        for k in COUNT_KEYS:
            assert s[k] == c[k], (label, q, k, s, c)
    return st, steps


# ---------------------------------------------------------------------------
# Building blocks: Philox keys and the permutation
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m,seed,t", [(1, 1, 0), (1000, 42, 3), (300001, 0xDEADBEEFCAFEF00D, 77)])
def test_perm_keys(ctx, m, seed, t):
    got = ctx.perm_keys(m, seed, t).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, oracle.perm_keys(m, seed, t))


@pytest.mark.parametrize("m", [1, 2, 3, 64, 512, 513, 5209, 70001, 131072, 131073 + 4096 * 37, 6654522])
def test_permutation(ctx, m):
    for seed, t in [(42, 0), (7, 13)]:
        print("perm m=%d seed=%d t=%d" % (m, seed, t), flush=True)
        got = ctx.permutation(m, seed, t).cpu().numpy().view(np.uint32)
        assert np.array_equal(got, oracle.permutation(m, seed, t))


def test_hub_key_partition_fallback(ctx):
    """A few vertices of huge degree: one target key gets thousands of
    inserters, so its partition exceeds the LDS capacity."""
    n = 4000
    hubs = [(a, b) for a in range(6) for b in range(6, n) if (a + b) % 3 != 0]
    E = keys(hubs)
    st, steps = check_run(ctx, E, n, 3, 0, 3, label="hubs")
    check_run(ctx, E, n, 4, 0, 2, pl=1 << 31, label="hubs_pl")


def test_permutation_small_buckets_and_fallback(ctx):
    import paper_2111_03005_amd as gesmc
    c = gesmc.Context(0)
    try:
        m = 50000
        exp = oracle.permutation(m, 3, 5)
        for avg, cap in [(64, 1024), (64, 64), (768, 64), (300, 256)]:
            c.set_option(gesmc.OPT_BUCKET_AVG, avg)
            c.set_option(gesmc.OPT_SORT_CAP, cap)
            got = c.permutation(m, 3, 5).cpu().numpy().view(np.uint32)
            assert np.array_equal(got, exp), (avg, cap)
    finally:
        c.close()


# ---------------------------------------------------------------------------
# Whole chain against the oracle
# ---------------------------------------------------------------------------

def test_gnp_small_10_supersteps(ctx):
    E, n = graphgen.workload_gnp_small()
    check_run(ctx, E, n, 42, 0, 10, label="gnp_n1024_d10")


def test_superstep_outcomes(ctx):
    for (E, n), pl in [(graphgen.workload_gnp_small(), 0), ((graphgen.powerlaw_graph(20000, 2.1, 2, 141, 9), 20000), 1 << 30)]:
        for t in (0, 5):
            out, oc, step = ctx.superstep_outcomes(to_dev(E), n, 11, t, pl)
            rc, exp, counts, exp_oc = oracle_run(E, n, 11, t, 1, pl, outcomes=True)
            assert np.array_equal(to_host(out), exp)
            assert np.array_equal(oc.cpu().numpy(), exp_oc)


@pytest.mark.parametrize("pl", [0, 1 << 31])
def test_powerlaw_small(ctx, pl):
    E = graphgen.powerlaw_graph(50000, 2.2, 2, 223, 5)
    check_run(ctx, E, 50000, 5, 3, 6, pl, label="pld_50k")


def test_edge_cases(ctx):
    cases = [
        ("m0", np.zeros(0, dtype=np.uint64), 4),
        ("m1", keys([(0, 3)]), 4),
        ("m2", keys([(0, 1), (2, 3)]), 4),
        ("m3", keys([(0, 1), (2, 3), (4, 5)]), 6),
        ("star", keys([(0, v) for v in range(1, 200)]), 200),
        ("complete_K40", keys([(a, b) for a in range(40) for b in range(a + 1, 40)]), 40),
        ("dense_gnp_0.9", graphgen.gnp(300, 0.9, 8), 300),
        ("hub_powerlaw_2.01", graphgen.powerlaw_graph(30000, 2.01, 1, int(30000 ** (1 / 1.01)) // 4, 12), 30000),
        ("odd_gnp", graphgen.gnp(2001, 0.003, 2), 2001),
    ]
    for name, E, n in cases:
        for seed, pl in [(42, 0), (9, 1 << 30)]:
            check_run(ctx, E, n, seed, 0, 4, pl, label=name)


def test_noncanonical_and_r0(ctx):
    E = np.array([(1 << 32) | 0, (3 << 32) | 2, key(4, 5)], dtype=np.uint64)
    out, st = ctx.run(to_dev(E), 6, 1, r=0)
    assert to_host(out).tolist() == [key(0, 1), key(2, 3), key(4, 5)]
    check_run(ctx, E, 6, 1, 0, 3, label="noncanonical")


def test_invalid_inputs_rejected_output_untouched(ctx):
    import paper_2111_03005_amd as gesmc
    bad = [
        (keys([(0, 1), (1, 2), (0, 1)]), 3, gesmc.E_NOT_SIMPLE),           # duplicate
        (np.array([(2 << 32) | 2, key(0, 1)], dtype=np.uint64), 3, gesmc.E_NOT_SIMPLE),  # loop
        (keys([(0, 1), (1, 7)]), 5, gesmc.E_RANGE),                         # id >= n
    ]
    for E, n, code in bad:
        for r in (0, 2):
            sentinel = torch.full((len(E),), 12345, dtype=torch.int64, device="cuda")
            with pytest.raises(gesmc.GesmcError) as ei:
                ctx.run(to_dev(E), n, 1, r=r, out=sentinel)
            assert ei.value.status == code
            assert (sentinel.cpu() == 12345).all()
    # the context stays usable
    E, n = graphgen.workload_gnp_small()
    check_run(ctx, E, n, 1, 0, 1, label="after_errors")


def test_size_limits_rejected_on_the_host(ctx):
    """The largest sizes the library takes: m < 2^30 edges per graph (and a
    batch of G graphs below 2^30 - G positions), vertex ids below 2^32 - 1,
    a 32-bit superstep counter.  Requests past them fail with a status before
    any device work, so a one-element buffer stands in for the edges."""
    import ctypes
    import paper_2111_03005_amd as gesmc
    from paper_2111_03005_amd import _binding as b
    lib = b._lib
    buf = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    p_in, p_out = ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(out.data_ptr())
    st = b.Stats()
    for m in (1 << 30, (1 << 30) + 1, 1 << 40):
        assert lib.gesmc_run(ctx._h, None, p_in, p_out, m, 8, 1, 0, 1, 0, 0, ctypes.byref(st), None) == gesmc.E_RANGE
        assert lib.gesmc_perm_keys(ctx._h, None, m, 1, 0, p_out) == gesmc.E_RANGE
        assert lib.gesmc_permutation(ctx._h, None, m, 1, 0, p_out) == gesmc.E_RANGE
    # superstep counter: t0 + r must fit 32 bits
    assert lib.gesmc_run(ctx._h, None, p_in, p_out, 1, 8, 1, 0xFFFFFFFF, 2, 0, 0, ctypes.byref(st), None) == gesmc.E_INVAL
    G = 2
    u64s, u32s = ctypes.c_uint64 * (G + 1), ctypes.c_uint32 * G
    seeds, t0s, rs = (ctypes.c_uint64 * G)(1, 2), u32s(0, 0), u32s(1, 1)
    tot = b.Stats()
    big = u64s(0, 1 << 29, (1 << 30) - 1)  # 2^30 - 1 positions + G padding records > limit
    assert lib.gesmc_run_batch(ctx._h, None, G, p_in, p_out, big, u32s(8, 8), seeds, t0s, rs, 0, 0, None,
                               ctypes.byref(tot)) == gesmc.E_RANGE
    small = u64s(0, 1, 1)
    wide = u32s(1 << 31, 1 << 31)  # 2^32 vertices in all
    assert lib.gesmc_run_batch(ctx._h, None, G, p_in, p_out, small, wide, seeds, t0s, rs, 0, 0, None,
                               ctypes.byref(tot)) == gesmc.E_RANGE
    # nothing was touched, and the context stays usable
    assert int(out.cpu()[0]) == 0
    E, n = graphgen.workload_gnp_small()
    check_run(ctx, E, n, 3, 0, 1, label="after_limits")


def test_host_entry_point(ctx):
    """gesmc_run_host (host vertex-id pairs in any orientation) equals
    gesmc_run on the device and the oracle; the output may alias the input;
    invalid input leaves the output untouched."""
    import ctypes
    import paper_2111_03005_amd as gesmc
    from paper_2111_03005_amd import _binding as b
    rng = np.random.default_rng(3)
    cases = [graphgen.workload_gnp_small(), (graphgen.powerlaw_graph(20000, 2.2, 2, 141, 5), 20000),
             (keys([(0, 3)]), 4), (keys([(0, 1), (2, 3)]), 4), (keys([(0, 1), (2, 3), (4, 5)]), 6),
             (np.zeros(0, dtype=np.uint64), 3)]
    for E, n in cases:
        uv = np.stack([(E >> np.uint64(32)).astype(np.uint32), (E & np.uint64(0xFFFFFFFF)).astype(np.uint32)], 1)
        flip = rng.random(len(E)) < 0.5
        uv[flip] = uv[flip][:, ::-1]  # either orientation is accepted
        got, st = ctx.run_host(uv, n, 17, t0=3, r=4, pl=1 << 29)
        keys_got = (got[:, 0].astype(np.uint64) << np.uint64(32)) | got[:, 1].astype(np.uint64)
        rc, exp, counts, _ = oracle_run(E, n, 17, 3, 4, 1 << 29)
        assert rc == 0
        assert np.array_equal(keys_got, exp), len(E)
        dev, _ = ctx.run(to_dev(E), n, 17, t0=3, r=4, pl=1 << 29) if len(E) else (None, None)
        if len(E):
            assert np.array_equal(to_host(dev), exp)
        assert st["attempts"] == sum(c["attempts"] for c in counts)
        assert st["legal"] == sum(c["legal"] for c in counts)
    # in place (uv_out == uv)
    E, n = graphgen.workload_gnp_small()
    buf = np.stack([(E >> np.uint64(32)).astype(np.uint32), (E & np.uint64(0xFFFFFFFF)).astype(np.uint32)], 1).copy()
    p = ctypes.c_void_p(buf.ctypes.data)
    st = b.Stats()
    assert b._lib.gesmc_run_host(ctx._h, p, p, len(E), n, 9, 0, 2, 0, 0, ctypes.byref(st)) == gesmc.OK
    rc, exp, _, _ = oracle_run(E, n, 9, 0, 2)
    assert np.array_equal((buf[:, 0].astype(np.uint64) << np.uint64(32)) | buf[:, 1].astype(np.uint64), exp)
    # invalid input: status, output untouched
    for pairs, n, code in [([(0, 1), (1, 2), (1, 0)], 3, gesmc.E_NOT_SIMPLE), ([(2, 2), (0, 1)], 3, gesmc.E_NOT_SIMPLE),
                           ([(0, 1), (1, 7)], 5, gesmc.E_RANGE)]:
        uv = np.array(pairs, dtype=np.uint32)
        out = np.full_like(uv, 12345)
        assert b._lib.gesmc_run_host(ctx._h, ctypes.c_void_p(uv.ctypes.data), ctypes.c_void_p(out.ctypes.data),
                                     len(uv), n, 1, 0, 2, 0, 0, None) == code
        assert (out == 12345).all()


def test_schedule_independence(ctx):
    """Bucket sizes, LDS sort capacity (incl. the slow exact path) and the
    number of multi-workgroup rounds change the schedule, never the result."""
    import paper_2111_03005_amd as gesmc
    E = graphgen.powerlaw_graph(40000, 2.05, 1, 400, 21)
    n = 40000
    ref = None
    for avg, cap, fr, strat, fuse in [(512, 1024, 4, 0, 1), (64, 1024, 0, 0, 1), (256, 64, 1, 0, 0),
                                      (700, 512, 8, 0, 0), (768, 1024, 0, 1, 1), (64, 64, 3, 1, 1),
                                      (128, 96, 2, 0, 1), (768, 1024, 2, 0, 0)]:
        c = gesmc.Context(0)
        try:
            c.set_option(gesmc.OPT_STRATEGY, strat)
            c.set_option(gesmc.OPT_FUSE_EMIT, fuse)
            c.set_option(gesmc.OPT_BUCKET_AVG, avg)
            c.set_option(gesmc.OPT_SORT_CAP, cap)
            c.set_option(gesmc.OPT_FAST_ROUNDS, fr)
            out, st, steps = c.run(to_dev(E), n, 77, t0=2, r=5, steps=True)
            got = to_host(out)
            if ref is None:
                ref = got
                rc, exp, _, _ = oracle_run(E, n, 77, 2, 5)
                assert np.array_equal(got, exp)
            assert np.array_equal(got, ref), (avg, cap, fr, strat, fuse)
        finally:
            c.close()


def test_level_split_independence(ctx):
    """The split of the bucket bits between the two radix levels (balanced,
    or a first level of 1..10 bits, the second level then clamped to at most
    12 bits) changes the schedule, never the result.  G(n,p) with about 1M
    edges and 64-record buckets: 14 bucket bits, so small first levels hit
    the clamp."""
    import paper_2111_03005_amd as gesmc
    n = 1 << 18
    E = graphgen.gnp(n, 8.0 / (n - 1), 31)
    rc, exp, _, _ = oracle_run(E, n, 123, 0, 2)
    assert rc == 0
    for l1 in (0, 1, 4, 10):
        c = gesmc.Context(0)
        try:
            c.set_option(gesmc.OPT_BUCKET_AVG, 64)
            c.set_option(gesmc.OPT_LEVEL1_BITS, l1)
            out, _ = c.run(to_dev(E), n, 123, r=2)
            assert np.array_equal(to_host(out), exp), l1
        finally:
            c.close()


def test_resume_equals_single_call(ctx):
    E, n = graphgen.workload_gnp_small()
    a, _ = ctx.run(to_dev(E), n, 5, t0=0, r=7)
    b1, _ = ctx.run(to_dev(E), n, 5, t0=0, r=3)
    b2, _ = ctx.run(b1, n, 5, t0=3, r=4)
    assert torch.equal(a, b2)


def test_unpermute_buckets_exact(ctx):
    """From 2^20 edges on, the write-back to input order goes through index
    buckets; sizes around the switch-over, an odd count and several bucket
    widths, against the oracle and against the one-pass write-back."""
    import paper_2111_03005_amd as gesmc
    for q, (n, m) in enumerate([(300000, (1 << 20) - 1), (300000, 1 << 20), (400000, (1 << 20) + 4097),
                                (1 << 21, 3000001)]):
        E = graphgen.class_graph(n, m, 0, 900 + q)
        check_run(ctx, E, n, 13 + q, q, 1, label="unpermute buckets m=%d" % m)
        ctx.set_option(gesmc.OPT_UNPERMUTE_BUCKETS, 0)
        try:
            one, _ = ctx.run(to_dev(E), n, 13 + q, t0=q, r=1)
        finally:
            ctx.set_option(gesmc.OPT_UNPERMUTE_BUCKETS, 1)
        two, _ = ctx.run(to_dev(E), n, 13 + q, t0=q, r=1)
        assert torch.equal(one, two)


def test_count_ahead_tile_edges(ctx):
    """A superstep's first radix level is counted by the previous superstep's
    first decision round, over tiles of 2048 positions.  Edge counts around
    tile ends (odd m puts the idle record alone in the last tile at 2049,
    4097 and 6145), several supersteps, a nonzero t0: exact against the oracle."""
    base = graphgen.gnp(3000, 0.0025, 21)
    assert len(base) >= 6145
    for m in (2049, 2050, 4095, 4096, 4097, 6144, 6145):
        check_run(ctx, base[:m].copy(), 3000, 70 + m, 5, 3, label="tile edge m=%d" % m)


def test_repeat_determinism(ctx):
    E = graphgen.powerlaw_graph(100000, 2.3, 2, 316, 4)
    outs = [to_host(ctx.run(to_dev(E), 100000, 8, r=3)[0]) for _ in range(3)]
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


# ---------------------------------------------------------------------------
# Full-size workloads (the benchmark's launch configuration)
# ---------------------------------------------------------------------------

def test_full_powerlaw_n2p20_20_supersteps(ctx):
    E, n = graphgen.workload_powerlaw_1m()
    st, steps = check_run(ctx, E, n, 42, 0, 20, label="pld_n2^20_g2.5")
    print("rounds per superstep:", [s["rounds"] for s in steps], flush=True)


def test_hub_heavy_powerlaw_exact(ctx):
    """gamma = 2.01 with degrees up to n^(1/(gamma-1)): hubs adjacent to a
    large share of the vertices make dependency chains hundreds of rounds
    long, which the finisher's in-order sweep decides.  Exact against the
    oracle, also at n = 2^20 (the hub benchmark workload)."""
    for n, seed in [(20000, 3), (100000, 4)]:
        E = graphgen.powerlaw_graph(n, 2.01, 1, int(n ** (1 / 1.01)), seed)
        st, steps = check_run(ctx, E, n, 7 + seed, 0, 3, label="hubs n=%d" % n)
        print("rounds per superstep:", [s["rounds"] for s in steps], flush=True)
    E, n = graphgen.workload_powerlaw_hubs()
    st, steps = check_run(ctx, E, n, 42, 0, 2, label="pld_n2^20_g2.01")
    print("rounds per superstep:", [s["rounds"] for s in steps], flush=True)


def test_adaptive_rounds_exact():
    """With GESMC_OPT_FAST_ROUNDS unset, a plain call after one that needed
    more than 16 decision rounds per superstep runs 64 multi-workgroup rounds
    (then a graph without hubs brings the context back to 2).  Every call is
    exact against the oracle whatever the schedule."""
    _require_gpu()
    import paper_2111_03005_amd as gesmc
    n = 20000
    E = graphgen.powerlaw_graph(n, 2.01, 1, int(n ** (1 / 1.01)), 3)
    G = graphgen.gnp(3000, 0.004, 9)
    c = gesmc.Context(0)
    try:
        _, steps = check_run(c, E, n, 11, 0, 3, label="hubs, first call")
        assert max(s["rounds"] for s in steps) > 16, "the hub graph must need long chains"
        check_run(c, E, n, 12, 3, 3, label="hubs, adapted rounds")
        check_run(c, G, 3000, 13, 0, 3, label="no hubs after hubs")
        check_run(c, E, n, 14, 0, 2, label="hubs again")
    finally:
        c.close()


def test_full_gnp_n2p22_one_superstep_exact(ctx):
    E, n = graphgen.workload_gnp_large()
    check_run(ctx, E, n, 42, 0, 1, label="gnp_n2^22_d32 r=1")


@pytest.mark.timeout(900)
def test_full_gnp_n2p22_ten_supersteps_exact(ctx):
    """The headline workload exactly as the benchmark runs it: 10 global
    switches on G(2^22, 32/(2^22-1)), the whole edge list and every
    superstep's counts against the oracle.

    The oracle's ten supersteps run as ten independent single-superstep
    calls, in parallel: superstep q starts from the GPU's state after q
    supersteps (s_q, computed by gesmc_run with t0 = q, r = 1) and must give
    s_{q+1} exactly.  The GPU's one 10-superstep call must equal s_10.  Since
    oracle.run(E, t0, a + b) = oracle.run(oracle.run(E, t0, a), t0 + a, b)
    (a pinned property of the oracle), this is the same as comparing the
    10-superstep call with oracle.run(E, 0, 10), in a tenth of the wall time."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    E, n = graphgen.workload_gnp_large()
    print("case gnp_n2^22_d32 r=10: m=%d" % len(E), flush=True)
    out, st, steps = ctx.run(to_dev(E), n, 42, t0=0, r=10, steps=True)
    full = to_host(out)
    states = [E]
    for q in range(10):
        o, _ = ctx.run(to_dev(states[-1]), n, 42, t0=q, r=1)
        states.append(to_host(o))
    assert np.array_equal(full, states[10]), "the 10-superstep call differs from its superstep-by-superstep chain"
    oracle._load()

    def one(q):
        rc, exp, counts, _ = oracle.run(states[q], n, 42, q, 1, 0)
        assert rc == 0
        ok = np.array_equal(exp, states[q + 1])
        print("oracle superstep %d: %s" % (q, "equal" if ok else "DIFFERS"), flush=True)
        return ok, counts[0]

    with ThreadPoolExecutor(max_workers=min(10, os.cpu_count() or 1)) as ex:
        res = list(ex.map(one, range(10)))
    bad = [q for q, (ok, _) in enumerate(res) if not ok]
    assert not bad, "supersteps %s differ from the oracle" % bad
    for q, (s, (_, c)) in enumerate(zip(steps, res)):
        for k in COUNT_KEYS:
            assert s[k] == c[k], (q, k, s, c)


def test_largest_size_gnp_one_superstep():
    """Close to the largest input (m < 2^30): G(n,p) with n = 2^25 and about
    6.5e8 edges, where the tuple pass has 2^30 slots and 21 partition bits.
    One global switch, checked on the device by what holds at any size (the
    oracle takes minutes here): degrees kept, every edge canonical and in
    range, no edge twice, outcome counts that add up, and a legal fraction
    near one for a graph this sparse."""
    _require_gpu()
    import paper_2111_03005_amd as gesmc
    n = 1 << 25
    E = graphgen.gnp(n, 38.7 / (n - 1), 41)
    m = len(E)
    print("largest-size case: n=%d m=%d" % (n, m), flush=True)
    assert (1 << 29) < m < (1 << 30)
    d_in = torch.from_numpy(E.view(np.int64)).to("cuda")
    del E

    def degrees(d):
        return (torch.bincount(d >> 32, minlength=n) + torch.bincount(d & 0xFFFFFFFF, minlength=n))

    deg_in = degrees(d_in)
    c = gesmc.Context(0)
    try:
        out, st = c.run(d_in, n, 7, r=1)
        torch.cuda.synchronize()
        print("largest-size case: stats", st, flush=True)
        assert torch.equal(degrees(out), deg_in)
        u, v = out >> 32, out & 0xFFFFFFFF
        assert bool((u < v).all()) and bool((v < n).all())
        del u, v
        srt, _ = torch.sort(out)
        assert bool((srt[1:] != srt[:-1]).all())
        del srt
        ell = m // 2
        assert st["attempts"] == ell
        assert st["legal"] + st["rej_loop"] + st["rej_exists"] + st["rej_pl"] == ell
        assert st["legal"] > 0.999 * ell
    finally:
        c.close()


def test_autotuned_context_computes_the_same():
    """The autotuner changes options only: the tuned context reproduces the oracle."""
    _require_gpu()
    import paper_2111_03005_amd as gesmc
    E = graphgen.powerlaw_graph(60000, 2.3, 2, 244, 31)
    n = 60000
    gesmc.tune_cache_clear()
    c = gesmc.Context(0)
    try:
        tu = c.autotune(to_dev(E), n, seed=5, supersteps=2)
        print("tuning:", tu, flush=True)
        assert tu["candidates"] == 8 and tu["best_ms"] <= tu["default_ms"] + 1e-9
        assert tu["fuse_emit"] in (0, 1) and tu["level1_bits"] in (0, 8)
        check_run(c, E, n, 77, 1, 4, label="autotuned")
    finally:
        c.close()
    choice = {k: tu[k] for k in ("bucket_avg", "level1_bits", "fuse_emit")}
    assert gesmc.tune_cache_size() == 1
    # a second context on the same device and shape class takes the kept choice without timing
    path = os.path.join(tempfile.mkdtemp(), "tune.json")
    gesmc.tune_cache_save(path)
    gesmc.tune_cache_clear()
    gesmc.tune_cache_load(path)
    E2 = graphgen.powerlaw_graph(61000, 2.3, 2, 246, 32)  # same log2 classes of m and n
    c = gesmc.Context(0)
    try:
        tu2 = c.autotune(to_dev(E2), 61000, seed=6, supersteps=2)
        assert tu2["candidates"] == 0 and {k: tu2[k] for k in choice} == choice
        check_run(c, E2, 61000, 78, 0, 3, label="cached tuning")
        c.set_option(gesmc.OPT_TUNE_CACHE, 0)
        tu3 = c.autotune(to_dev(E2), 61000, seed=6, supersteps=2)
        assert tu3["candidates"] == 8
    finally:
        c.close()


def test_round_limit_fails_the_call_and_leaves_output_untouched():
    """GESMC_OPT_ROUND_LIMIT: a superstep that needs more decision rounds than
    the limit fails the call with GESMC_E_ROUNDS and d_out untouched; with a
    limit it fits, the result is the oracle's."""
    _require_gpu()
    import paper_2111_03005_amd as gesmc
    E = graphgen.powerlaw_graph(20000, 2.05, 2, 141, 17)
    n = 20000
    c = gesmc.Context(0)
    try:
        _, st, steps = c.run(to_dev(E), n, 5, r=6, steps=True)
        need = max(s["rounds"] for s in steps)
        print("rounds per superstep:", [s["rounds"] for s in steps], flush=True)
        assert need >= 2
        c.set_option(gesmc.OPT_ROUND_LIMIT, need - 1)
        sentinel = torch.full((len(E),), 7, dtype=torch.int64, device="cuda")
        with pytest.raises(gesmc.GesmcError) as ei:
            c.run(to_dev(E), n, 5, r=6, out=sentinel)
        assert ei.value.status == gesmc.E_ROUNDS
        assert bool((sentinel == 7).all())
        c.set_option(gesmc.OPT_ROUND_LIMIT, need)
        check_run(c, E, n, 5, 0, 6, label="round limit met")
        c.set_option(gesmc.OPT_ROUND_LIMIT, 0)
    finally:
        c.close()


@pytest.mark.parametrize("pl", [0, 1 << 31])
def test_small_plain_path_exact(pl):
    """gesmc_run on graphs that fit one workgroup's LDS (at most 4096 edges,
    6144 with ids below 2^16) runs every superstep in LDS, with the
    permutations computed ahead in pieces of up to 32 supersteps: equal to
    the oracle and to the multi-kernel supersteps (GESMC_OPT_SMALL_GRAPHS 0)
    at every size limit, for long chains, with P_L, and over several pieces
    (r = 70: 32 + 32 + 6)."""
    _require_gpu()
    import paper_2111_03005_amd as gesmc
    cases = []
    for m in (2, 3, 1023, 1024, 1025, 4095, 4096, 4097, 6143, 6144, 6145):
        E = graphgen.gnp(900, 0.02, 100 + m)
        cases.append((np.sort(E[:m]), 900, "G(900, .02) cut to %d" % m))
    E, n = graphgen.workload_gnp_small()
    cases.append((E, n, "gnp_n1024_d10"))
    cases.append((graphgen.gnp(40, 0.9, 5), 40, "dense"))
    cases.append((keys([(0, v) for v in range(1, 300)]), 300, "star"))
    E = graphgen.gnp(900, 0.02, 7)[:5000]  # ids beyond 2^16: the compact class does not apply
    cases.append(((E + np.uint64((70000 << 32) | 70000)).astype(np.uint64), 71000, "ids above 2^16"))
    c_on, c_off = gesmc.Context(0), gesmc.Context(0)
    try:
        c_off.set_option(gesmc.OPT_SMALL_GRAPHS, 0)
        for q, (E, n, label) in enumerate(cases):
            st_on = check_run_plain(c_on, E, n, 11 + q, 5 * q, 30, pl, label)
            st_off = check_run_plain(c_off, E, n, 11 + q, 5 * q, 30, pl, label + " (multi-kernel)")
            for k in COUNT_KEYS:
                assert st_on[k] == st_off[k], (label, k)
        for E, n, label in (cases[3], cases[9], cases[11]):  # 1024, 6144 (compact) and gnp_n1024_d10 edges
            check_run_plain(c_on, E, n, 5, 3, 70, pl, label + ", 70 supersteps")
    finally:
        c_on.close()
        c_off.close()


def check_run_plain(ctx, E, n, seed, t0, r, pl, label):
    """gesmc_run without per-superstep records (the small-graph path applies)."""
    print("case %s: m=%d n=%d r=%d pl=%d" % (label, len(E), n, r, pl), flush=True)
    out, st = ctx.run(to_dev(E), n, seed, t0=t0, r=r, pl=pl)
    rc, exp, counts, _ = oracle_run(E, n, seed, t0, r, pl)
    assert rc == 0
    got = to_host(out)
    assert np.array_equal(got, exp), "%s: %d positions differ" % (label, int((got != exp).sum()))
    for k in COUNT_KEYS:
        assert st[k] == sum(c[k] for c in counts), (label, k, st)
    return st


def test_small_plain_path_invalid_inputs():
    """The small path checks its input as the multi-kernel path does (loop,
    id out of range, duplicate) and leaves d_out untouched, also when the
    call runs in several pieces (the later pieces see the error and stop)."""
    _require_gpu()
    import paper_2111_03005_amd as gesmc
    c = gesmc.Context(0)
    try:
        good = graphgen.gnp(900, 0.02, 3)[:5000]
        for bad, status in [(np.concatenate([good, good[:1]]), gesmc.E_NOT_SIMPLE),
                            (np.concatenate([good[:100], keys([(5, 5)])]), gesmc.E_NOT_SIMPLE),
                            (np.concatenate([good[:3000], keys([(1, 900)])]), gesmc.E_RANGE)]:
            sentinel = torch.full((len(bad),), 3, dtype=torch.int64, device="cuda")
            for r in (4, 40):
                with pytest.raises(gesmc.GesmcError) as ei:
                    c.run(to_dev(bad), 900, 1, r=r, out=sentinel)
                assert ei.value.status == status
                assert bool((sentinel == 3).all())
    finally:
        c.close()

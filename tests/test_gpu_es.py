"""ParES (Alg. 2): the ES-MC chain on the GPU through the C ABI, bit for bit
against the sequential ES-MC oracle (Def. 2.1 applied switch by switch).

Integer work throughout, so the bar is exact equality of the edge list in
position order, the outcome counts and (at small sizes) every switch's
outcome code.  The superstep cut is the GPU's own schedule and is not part
of parity; only its result is.
"""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

COUNTS = ("attempts", "legal", "rej_loop", "rej_exists")


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


def check_es(ctx, E, n, seed, k0, r, label="", outcomes=False):
    print("case %s: m=%d n=%d seed=%d k0=%d r=%d" % (label, len(E), n, seed, k0, r), flush=True)
    res = ctx.run_es(to_dev(E), n, seed, k0=k0, r=r, outcomes=outcomes)
    got = to_host(res[0])
    st = res[1]
    rc, exp, cnt, oc = oracle.es_run(E, n, seed, k0, r, outcomes=outcomes)
    assert rc == 0
    diff = np.flatnonzero(got != exp)
    assert diff.size == 0, "%s: %d positions differ, first %s" % (label, diff.size, diff[:5])
    for k in COUNTS:
        assert st[k] == cnt[k], (label, k, st, cnt)
    if outcomes:
        assert np.array_equal(res[2].cpu().numpy(), oc), label
    return st


@pytest.mark.parametrize("m,seed,k0", [(2, 1, 0), (3, 5, 2**32 - 7), (5209, 42, 0), (6654522, 2**63 + 11, 2**40)])
def test_es_draws(ctx, m, seed, k0):
    di, dj, dg = ctx.es_draws(m, seed, k0, 100000)
    i, j, g = oracle.es_draws(seed, k0, 100000, m)
    assert np.array_equal(di.cpu().numpy().view(np.uint64), i)
    assert np.array_equal(dj.cpu().numpy().view(np.uint64), j)
    assert np.array_equal(dg.cpu().numpy(), g)


def test_es_small_graphs_every_outcome(ctx):
    """Small graphs, many switches: tiny supersteps (indices collide often),
    dense graphs where most targets exist, a star (every switch rejected)."""
    cases = [(graphgen.gnp(30, 0.3, 1), 30), (graphgen.gnp(14, 0.8, 2), 14),
             (keys([(0, v) for v in range(1, 40)]), 40), (keys([(0, 1), (2, 3)]), 4),
             (keys([(0, 1), (2, 3), (4, 5)]), 6), (graphgen.powerlaw_graph(500, 2.1, 1, 22, 3), 500)]
    for q, (E, n) in enumerate(cases):
        check_es(ctx, E, n, 100 + q, 7 * q, 3000, label="small %d" % q, outcomes=True)


def test_es_gnp_small_and_powerlaw(ctx):
    E, n = graphgen.workload_gnp_small()
    st = check_es(ctx, E, n, 42, 0, 50000, label="gnp n=1024", outcomes=True)
    print("supersteps", st["supersteps"], "rounds_max", st["rounds_max"], flush=True)
    E = graphgen.powerlaw_graph(100000, 2.1, 2, 316, 5)
    check_es(ctx, E, 100000, 9, 12345, 400000, label="power-law n=1e5 gamma 2.1")
    E = graphgen.powerlaw_graph(20000, 2.01, 1, 2000, 6)  # hubs: many target dependencies
    check_es(ctx, E, 20000, 3, 0, 200000, label="power-law hubs gamma 2.01", outcomes=True)


def test_es_epochs_and_resume(ctx):
    """More switches than one epoch (the edge set is rebuilt between launches),
    and run(r1) followed by run(r2, k0 + r1) equals run(r1 + r2)."""
    E = graphgen.powerlaw_graph(3000, 2.3, 2, 54, 8)
    n = 3000
    st = check_es(ctx, E, n, 17, 5, 300000, label="several epochs")
    assert st["epochs"] >= 4
    a, _ = ctx.run_es(to_dev(E), n, 17, k0=5, r=120000)
    b, _ = ctx.run_es(a, n, 17, k0=120005, r=180000)
    full, _ = ctx.run_es(to_dev(E), n, 17, k0=5, r=300000)
    assert torch.equal(b, full)


def test_es_edge_cases_and_errors(ctx):
    import paper_2111_03005_amd as gesmc
    for E in (np.zeros(0, dtype=np.uint64), keys([(3, 1)])):
        out, st = ctx.run_es(to_dev(E), 5, 1, r=10) if len(E) else (None, None)
        if len(E):
            assert np.array_equal(to_host(out), keys([(1, 3)])) and st["attempts"] == 0
    E = keys([(0, 1), (2, 3), (4, 5), (6, 7)])
    out, st = ctx.run_es(to_dev(E), 8, 1, r=0)
    assert np.array_equal(to_host(out), E) and st["attempts"] == 0
    for bad, status in [(keys([(1, 2), (2, 1), (3, 4)]), gesmc.E_NOT_SIMPLE), (keys([(1, 9)]) , gesmc.E_RANGE),
                        (np.array([(2 << 32) | 2, key(0, 1)], dtype=np.uint64), gesmc.E_NOT_SIMPLE)]:
        sentinel = torch.full((len(bad),), 7, dtype=torch.int64, device="cuda")
        with pytest.raises(gesmc.GesmcError) as ei:
            ctx.run_es(to_dev(bad), 5, 1, r=100, out=sentinel)
        assert ei.value.status == status
        assert bool((sentinel == 7).all())
    E = keys([(1, 0), (3, 2), (5, 4), (7, 6)])  # (max, min) pairs are canonicalised
    check_es(ctx, E, 8, 4, 0, 1000, label="non-canonical input")


def test_es_full_size_powerlaw_n2p20(ctx):
    """The power-law n = 2^20 workload (m = 6.65e6) with m ES-MC switches:
    the result and counts exactly against the oracle."""
    E, n = graphgen.workload_powerlaw_1m()
    st = check_es(ctx, E, n, 42, 0, len(E), label="pld_n2^20_g2.5, r = m")
    print("ParES stats:", st, flush=True)

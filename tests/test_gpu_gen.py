"""Input realisation on the GPU (G(n,p), power-law degrees, Havel-Hakimi,
relabelling: the steps before the chain that build Sec. 6's synthetic
inputs) through the C ABI, bit for bit against the oracle's definitions
(``oracle/gen_oracle.cpp``).

Floating point decides integers here (the geometric skips, the degree
weights); both sides take those decisions with the same portable ln / exp
steps, so the bar is exact equality of every edge key and degree.
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


def host64(t):
    return t.cpu().numpy().view(np.uint64)


def dev32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32).copy()).to("cuda")


def dev64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64).copy()).to("cuda")


@pytest.mark.parametrize("n,p,seed", [(1024, 10.0 / 1023.0, 1), (5000, 0.3, 2), (3000, 0.002, 2**63 + 3),
                                      (2, 0.5, 4), (300, 1.0, 5), (200, 0.999, 6), (100000, 1e-7, 7),
                                      (1 << 20, 16.0 / ((1 << 20) - 1), 8)])
def test_gnp_exact(ctx, n, p, seed):
    print("case gnp n=%d p=%g seed=%d" % (n, p, seed), flush=True)
    got = host64(ctx.gen_gnp(n, p, seed))
    want = oracle.gen_gnp(n, p, seed)
    assert len(got) == len(want)
    assert np.array_equal(got, want)


def test_gnp_empty_cases(ctx):
    for n, p in [(0, 0.5), (1, 0.5), (100, 0.0), (100, -1.0)]:
        assert ctx.gen_gnp(n, p, 1).numel() == 0


def test_gnp_full_size_exact(ctx):
    """G(n = 2^22, p = 32/(2^22 - 1)): the benchmark's G(n,p) workload, every key."""
    n = 1 << 22
    p = 32.0 / (n - 1)
    print("case gnp n=2^22", flush=True)
    got = host64(ctx.gen_gnp(n, p, 3))
    want = oracle.gen_gnp(n, p, 3)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n,gamma,dmin,dmax,seed", [(1 << 20, 2.5, 5, 1024, 2), (1000, 2.01, 1, 31, 3),
                                                    (77777, 3.0, 2, 278, 2**40 + 9), (9, 2.0, 4, 4, 1),
                                                    (33, 0.0, 1, 7, 5)])
def test_pld_exact(ctx, n, gamma, dmin, dmax, seed):
    print("case pld n=%d gamma=%g [%d..%d]" % (n, gamma, dmin, dmax), flush=True)
    deg, s = ctx.gen_pld_degrees(n, gamma, dmin, dmax, seed)
    want = oracle.gen_pld(n, gamma, dmin, dmax, seed)
    assert want is not None
    assert np.array_equal(deg.cpu().numpy().view(np.uint32), want[0])
    assert s == want[1]


def test_pld_rejects(ctx):
    import paper_2111_03005_amd as gesmc
    for args in [(7, 2.0, 3, 3, 1), (0, 2.0, 1, 5, 1), (10, 2.0, 0, 5, 1), (10, 2.0, 6, 5, 1), (10, -1.0, 1, 5, 1)]:
        with pytest.raises(gesmc.GesmcError) as ei:
            ctx.gen_pld_degrees(*args)
        assert ei.value.status == gesmc.E_INVAL, args


def check_hh(ctx, deg, label):
    print("case hh %s n=%d" % (label, len(deg)), flush=True)
    want = oracle.gen_havel_hakimi(np.asarray(deg, dtype=np.uint32))
    import paper_2111_03005_amd as gesmc
    if want is None:
        with pytest.raises(gesmc.GesmcError) as ei:
            ctx.gen_havel_hakimi(dev32(deg))
        assert ei.value.status == gesmc.E_NOT_GRAPHICAL, label
        return None
    got = host64(ctx.gen_havel_hakimi(dev32(deg)))
    assert np.array_equal(got, want), label
    return got


def test_havel_hakimi_small_sequences(ctx):
    rng = np.random.default_rng(11)
    graphical = 0
    for q in range(150):
        n = int(rng.integers(1, 200))
        deg = rng.integers(0, max(1, min(n, 90)), n).astype(np.uint32)
        if deg.sum() % 2:
            deg[0] = deg[0] + 1 if deg[0] + 1 < n else max(int(deg[0]) - 1, 0)
        if deg.sum() % 2:
            continue
        graphical += check_hh(ctx, deg, "random %d" % q) is not None
    assert graphical > 20
    for deg, label in [([0] * 10, "zeros"), ([3] * 8, "cubic"), ([9] + [1] * 9, "star"),
                       ([5, 5, 5, 5, 5, 5], "K6"), ([6, 1, 1, 1, 1, 1, 1], "star of 7"), ([2, 2], "2 on 2"),
                       ([1, 1], "one edge"), ([70] * 71 + [0], "K71 plus isolated")]:
        if sum(deg) % 2 == 0:
            check_hh(ctx, np.array(deg, dtype=np.uint32), label)


@pytest.mark.parametrize("n,gamma,dmin,dmax,seed", [(1 << 20, 2.5, 5, 1024, 2), (100000, 2.01, 1, 316, 4),
                                                    (50000, 2.2, 2, 7000, 5), (4000, 2.1, 1, 3999, 6)])
def test_havel_hakimi_powerlaw_exact(ctx, n, gamma, dmin, dmax, seed):
    deg = oracle.gen_pld(n, gamma, dmin, dmax, seed)[0]
    check_hh(ctx, deg, "pld gamma=%g" % gamma)


def test_relabel_exact(ctx):
    E = graphgen.gnp(5000, 0.003, 3)
    got = host64(ctx.gen_relabel(dev64(E), 5000, 77))
    assert np.array_equal(got, oracle.gen_relabel(E, 5000, 77))
    import paper_2111_03005_amd as gesmc
    with pytest.raises(gesmc.GesmcError) as ei:
        ctx.gen_relabel(dev64(np.array([(1 << 32) | 7], dtype=np.uint64)), 5, 1)
    assert ei.value.status == gesmc.E_RANGE


def test_powerlaw_pipeline_full_size(ctx):
    """Degrees, Havel-Hakimi and relabelling at n = 2^20, gamma = 2.5,
    [5..1024] (the power-law benchmark input's recipe), against the oracle."""
    n, seed = 1 << 20, 2
    print("case pipeline n=2^20", flush=True)
    got = host64(ctx.gen_powerlaw_graph(n, 2.5, 5, 1024, seed))
    deg = oracle.gen_pld(n, 2.5, 5, 1024, seed)[0]
    want = oracle.gen_relabel(oracle.gen_havel_hakimi(deg), n, seed)
    assert np.array_equal(got, want)

"""Mixing diagnostic (Sec. 6.1) on the GPU through the C ABI against its
oracle (every state kept, the definition applied directly).

The chain, the thinned series and the transition counts are integer work:
edges tracked and the summed counts must be equal.  G^2 is float64 on both
sides; an edge's decision may differ only where |G^2 - ln N| is within
rounding (the oracle counts those as borderline).
"""
import numpy as np
import pytest

import graphgen
from oracle import mixing

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


def check(ctx, E, n, seed, K, thin, chain, pl=0, label=""):
    print("case %s: m=%d n=%d K=%d chain=%d" % (label, len(E), n, K, chain), flush=True)
    d = to_dev(E)
    got, ms = ctx.mixing(d, n, seed, K, thin, chain=chain, pl=pl)
    assert np.array_equal(d.cpu().numpy().view(np.uint64), E)  # input left as it was
    exp = mixing.diagnostic(E, n, seed, K, thin, chain="global" if chain == 0 else "es", pl=pl)
    for g, x in zip(got, exp):
        assert g["k"] == x["k"] and g["transitions"] == x["N"], (label, g, x)
        assert g["tracked"] == x["tracked"], (label, g, x)
        tot = x["counts_total"]
        assert [g["n00"], g["n01"], g["n10"], g["n11"]] == [tot[0][0], tot[0][1], tot[1][0], tot[1][1]], (label, g, x)
        assert abs(g["non_independent"] - x["non_independent"]) <= x["borderline"], (label, g, x)
    print("  fractions:", [round(x["fraction"], 4) for x in exp], "%.1f ms" % ms, flush=True)
    return got


@pytest.mark.parametrize("chain", [0, 1])
def test_mixing_powerlaw_small(ctx, chain):
    E = graphgen.powerlaw_graph(128, 2.2, 1, 11, 4)
    check(ctx, E, 128, 9, 200, [1, 2, 3, 5, 8, 16, 250], chain, label="n=2^7 gamma=2.2")


@pytest.mark.parametrize("chain", [0, 1])
def test_mixing_powerlaw_hubs(ctx, chain):
    """(n, gamma) = (2^10, 2.01) with d_max = n^(1/(gamma-1)): the skewed end of Sec. 6.1's grid."""
    n = 1 << 10
    E = graphgen.powerlaw_graph(n, 2.01, 1, int(n ** (1 / 1.01)), 6)
    check(ctx, E, n, 3, 120, [1, 4, 16], chain, label="n=2^10 gamma=2.01")


def test_mixing_pl_and_star(ctx):
    E = graphgen.gnp(200, 0.05, 2)
    check(ctx, E, 200, 5, 60, [1, 7], 0, pl=1 << 30, label="gnp with P_L")
    star = np.array([v for v in range(1, 50)], dtype=np.uint64)  # (0, v): every switch rejected
    got = check(ctx, star, 50, 1, 40, [1, 2], 0, label="star")
    assert all(g["non_independent"] == 0 and g["tracked"] == 49 for g in got)


def test_mixing_argument_checks(ctx):
    import paper_2111_03005_amd as gesmc
    E = graphgen.gnp(100, 0.05, 1)
    for kw, status in [(dict(n=(1 << 14) + 1), gesmc.E_RANGE), (dict(thin=[0]), gesmc.E_INVAL),
                       (dict(chain=2), gesmc.E_INVAL)]:
        args = dict(n=100, thin=[1], chain=0)
        args.update(kw)
        with pytest.raises(gesmc.GesmcError) as ei:
            ctx.mixing(to_dev(E), args["n"], 1, 10, args["thin"], chain=args["chain"])
        assert ei.value.status == status
    bad = np.array([(1 << 32) | 2, (1 << 32) | 2], dtype=np.uint64)
    with pytest.raises(gesmc.GesmcError) as ei:
        ctx.mixing(to_dev(bad), 10, 1, 10, [1])
    assert ei.value.status == gesmc.E_NOT_SIMPLE

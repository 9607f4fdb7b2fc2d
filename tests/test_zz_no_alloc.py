"""gesmc_run_noalloc (the entry point that allocates nothing) through the C ABI.

Its output and counts must equal gesmc_run's on the same input, bit for bit,
and the oracle's; two calls in a row, the second on a smaller input, so that
what the first left in the shared device array cannot leak into the second.
"""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

COUNT_KEYS = ("attempts", "legal", "rej_loop", "rej_exists", "rej_pl")


def _gesmc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_03005_amd as gesmc
    return gesmc


def to_dev(E):
    return torch.from_numpy(np.ascontiguousarray(E, dtype=np.uint64).view(np.int64).copy()).to("cuda")


def to_host(t):
    return t.cpu().numpy().view(np.uint64)


def check_same(gesmc, ctx, E, n, seed, t0, r, pl=0, label=""):
    print("case %s: m=%d n=%d r=%d pl=%d" % (label, len(E), n, r, pl), flush=True)
    d = to_dev(E)
    got, st = ctx.run_noalloc(d, n, seed, t0=t0, r=r, pl=pl)
    ref, st_ref = ctx.run(d, n, seed, t0=t0, r=r, pl=pl)
    got_h, ref_h = to_host(got), to_host(ref)
    assert np.array_equal(got_h, ref_h), "%s: %d positions differ from gesmc_run" % (label, int((got_h != ref_h).sum()))
    for k in COUNT_KEYS + ("supersteps",):
        assert st[k] == st_ref[k], (label, k, st, st_ref)
    rc, exp, counts, _ = oracle.run(E, n, seed, t0, r, pl)
    assert rc == 0 and np.array_equal(got_h, exp), label
    for k in COUNT_KEYS:
        assert st[k] == sum(c[k] for c in counts), (label, k)


def test_noalloc_equals_run_two_calls_second_smaller():
    gesmc = _gesmc()
    c = gesmc.Context(0)
    try:
        E1 = graphgen.powerlaw_graph(300000, 2.2, 2, 547, 3)
        assert len(E1) <= gesmc.NOALLOC_MAX_EDGES
        check_same(gesmc, c, E1, 300000, 42, 0, 5, label="power-law n=3e5")
        E2, n2 = graphgen.workload_gnp_small()
        check_same(gesmc, c, E2, n2, 7, 3, 70, label="gnp n=1024, 70 supersteps (two pieces)")
        check_same(gesmc, c, E2[:777], n2, 9, 0, 4, pl=1 << 30, label="gnp cut to 777 edges, P_L")
    finally:
        c.close()


def test_noalloc_fresh_context_first_call():
    """The entry point as the very first call of a context (nothing sized yet)."""
    gesmc = _gesmc()
    c = gesmc.Context(0)
    try:
        E = graphgen.powerlaw_graph(50000, 2.5, 2, 223, 8)
        check_same(gesmc, c, E, 50000, 11, 0, 3, label="fresh context")
    finally:
        c.close()


def test_noalloc_limits_and_errors():
    gesmc = _gesmc()
    c = gesmc.Context(0)
    try:
        big = torch.zeros(gesmc.NOALLOC_MAX_EDGES + 1, dtype=torch.int64, device="cuda")
        with pytest.raises(gesmc.GesmcError) as ei:
            c.run_noalloc(big, 1 << 20, 1, r=1)
        assert ei.value.status == gesmc.E_RANGE and "no-allocation limit" in str(ei.value)
        del big
        # an input error leaves d_out untouched
        E = np.array([(1 << 32) | 2, (1 << 32) | 2, (3 << 32) | 4], dtype=np.uint64)
        out = torch.full((3,), 5, dtype=torch.int64, device="cuda")
        with pytest.raises(gesmc.GesmcError) as ei:
            c.run_noalloc(to_dev(E), 10, 1, r=2, out=out)
        assert ei.value.status == gesmc.E_NOT_SIMPLE
        assert bool((out == 5).all())
        c.set_option(gesmc.OPT_STRATEGY, 1)
        with pytest.raises(gesmc.GesmcError) as ei:
            c.run_noalloc(to_dev(E), 10, 1, r=2)
        assert ei.value.status == gesmc.E_INVAL
        c.set_option(gesmc.OPT_STRATEGY, 0)
        # the context's own buffers still work after the no-allocation calls
        E2, n2 = graphgen.workload_gnp_small()
        check_same(gesmc, c, E2, n2, 3, 0, 2, label="after errors")
    finally:
        c.close()

"""The caller-supplied allocator (gesmc_set_allocator): results identical to
the context's own hipMalloc buffers, every buffer returned to the allocator
that made it, and an allocation failure injected through the hook fails the
call cleanly (GESMC_E_NOMEM, output untouched, context usable afterwards)."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_03005_amd as gesmc
    return gesmc


def to_dev(E):
    return torch.from_numpy(np.ascontiguousarray(E, dtype=np.uint64).view(np.int64).copy()).to("cuda")


class Counting:
    """PyTorch's caching allocator with counts; fail_after = n makes the
    (n+1)-th allocation return no memory."""

    def __init__(self, fail_after=None):
        self.live, self.allocs, self.frees, self.fail_after = {}, 0, 0, fail_after

    def alloc(self, n):
        if self.fail_after is not None and self.allocs >= self.fail_after:
            return 0
        p = torch.cuda.caching_allocator_alloc(n, device=0)
        self.live[p] = n
        self.allocs += 1
        return p

    def free(self, p):
        assert p in self.live, "freed a buffer this allocator did not make"
        del self.live[p]
        self.frees += 1
        torch.cuda.caching_allocator_delete(p)


def test_torch_allocator_same_results_and_all_returned():
    gesmc = _gpu()
    E, n = graphgen.workload_powerlaw_1m()
    a = Counting()
    ctx = gesmc.Context(0)
    ctx.set_allocator(a.alloc, a.free)
    out, st = ctx.run(to_dev(E), n, 42, t0=0, r=2)
    ref = gesmc.Context(0)
    want, _ = ref.run(to_dev(E), n, 42, t0=0, r=2)
    assert torch.equal(out, want)
    assert a.allocs > 0 and len(a.live) == a.allocs - a.frees
    # batched and the generators allocate through it too
    g = graphgen.batch_graphs(8, 3, 1e2, 1e4)
    Eb, offs, ns = graphgen.concat(g)
    got_b, _, _ = ctx.run_batch(to_dev(Eb), offs, ns, [5 + q for q in range(8)], [3] * 8)
    want_b, _, _ = ref.run_batch(to_dev(Eb), offs, ns, [5 + q for q in range(8)], [3] * 8)
    assert torch.equal(got_b, want_b)
    G = ctx.gen_gnp(3000, 0.01, 7)
    assert np.array_equal(G.cpu().numpy().view(np.uint64), oracle.gen_gnp(3000, 0.01, 7))
    ctx.close()
    ref.close()
    assert a.live == {} and a.frees == a.allocs


def test_allocation_failure_through_the_hook():
    gesmc = _gpu()
    E, n = graphgen.gnp(20000, 0.001, 4), 20000
    a = Counting(fail_after=2)
    ctx = gesmc.Context(0)
    ctx.set_option(gesmc.OPT_SMALL_GRAPHS, 0)
    ctx.set_allocator(a.alloc, a.free)
    out = torch.full((len(E),), -1, dtype=torch.int64, device="cuda")
    with pytest.raises(gesmc.GesmcError) as ei:
        ctx.run(to_dev(E), n, 1, r=2, out=out)
    assert ei.value.status == gesmc.E_NOMEM
    assert (out == -1).all()
    a.fail_after = None  # the allocator recovers: the same context works
    got, _ = ctx.run(to_dev(E), n, 1, r=2, out=out)
    rc, want, _, _ = oracle.run(E, n, 1, 0, 2)
    assert np.array_equal(got.cpu().numpy().view(np.uint64), want)
    ctx.set_allocator(None, None)  # back to hipMalloc; earlier buffers keep their allocator
    got2, _ = ctx.run(to_dev(E), n, 1, r=2)
    assert torch.equal(got, got2)
    ctx.close()
    assert a.live == {}


def test_allocator_argument_checks():
    gesmc = _gpu()
    ctx = gesmc.Context(0)
    lib = gesmc._binding.load_library()
    from paper_2111_03005_amd._binding import ALLOC_FN, FREE_FN
    st = lib.gesmc_set_allocator(ctx._h, ALLOC_FN(lambda n, u: 0), FREE_FN(), None)
    assert st == gesmc.E_INVAL
    srv = gesmc.Server(ctx, hbm_budget_bytes=1 << 26)
    a = Counting()
    with pytest.raises(gesmc.GesmcError) as ei:
        ctx.set_allocator(a.alloc, a.free)  # not while a server uses the context
    assert ei.value.status == gesmc.E_INVAL
    srv.close()
    ctx.set_allocator(a.alloc, a.free)
    ctx.close()

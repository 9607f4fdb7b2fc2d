"""Serving form (gesmc_server_*) through the C ABI: continuous batching.

Requests submitted while others are on the GPU join the running supersteps;
every result must equal the oracle and gesmc_run on that graph alone, bit for
bit (tolerance 0), whatever else was resident.
"""
import time

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gesmc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_03005_amd as gesmc
    return gesmc


def key(a, b):
    return (min(a, b) << 32) | max(a, b)


def keys(pairs):
    return np.array([key(a, b) for a, b in pairs], dtype=np.uint64).reshape(-1)


def requests(seed, count, n_lo, n_hi):
    graphs = graphgen.batch_graphs(count, seed, n_lo, n_hi)
    rng = np.random.default_rng(seed)
    out = []
    for g, (E, n) in enumerate(graphs):
        out.append(dict(E=E, n=n, seed=int(rng.integers(0, 2**63)), r=int(rng.integers(1, 9)),
                        t0=int(rng.integers(0, 100)), pl=int(rng.choice([0, 1 << 29]))))
    return out


def alone(ctx, q):
    d = torch.from_numpy(q["E"].view(np.int64).copy()).to("cuda")
    out, _ = ctx.run(d, q["n"], q["seed"], t0=q["t0"], r=q["r"], pl=q["pl"])
    return out.cpu().numpy().view(np.uint64)


def test_serve_staggered_equals_alone_and_oracle():
    gesmc = _gesmc()
    qs = requests(3, 36, 1e2, 2e4)
    c = gesmc.Context(0)
    ref = gesmc.Context(0)
    srv = gesmc.Server(c, hbm_budget_bytes=1 << 30)
    try:
        tickets = []
        for i, q in enumerate(qs):
            tickets.append(srv.submit(q["E"], q["n"], q["seed"], q["r"], t0=q["t0"], pl=q["pl"]))
            if i % 6 == 5:
                time.sleep(0.003)  # later requests arrive while earlier ones run
        results = [srv.wait(t) for t in tickets]
        info = srv.info()
        print("server info:", info, flush=True)
        assert info["completed"] == len(qs)
        for q, res in zip(qs, results):
            assert res["status"] == gesmc.OK
            rc, exp, counts, _ = oracle.run(q["E"], q["n"], q["seed"], q["t0"], q["r"], q["pl"])
            assert rc == 0
            assert np.array_equal(res["edges"], exp)
            assert np.array_equal(res["edges"], alone(ref, q))
            s = res["stats"]
            for k in ("attempts", "legal", "rej_loop", "rej_exists", "rej_pl"):
                assert s[k] == sum(cn[k] for cn in counts), k
            assert res["t_submit"] <= res["t_admit"] <= res["t_done"]
    finally:
        srv.close()
        ref.close()
        c.close()


def test_serve_admission_by_budget():
    """A budget for about 12k resident edges: requests wait in the queue for
    memory, and each still gets its exact result."""
    gesmc = _gesmc()
    qs = requests(5, 20, 1e3, 3e3)
    c = gesmc.Context(0)
    srv = gesmc.Server(c, hbm_budget_bytes=136 * 12000, max_graphs=8)
    try:
        tickets = [srv.submit(q["E"], q["n"], q["seed"], q["r"], t0=q["t0"], pl=q["pl"]) for q in qs]
        peak = 0
        while srv.info()["completed"] < len(qs):
            inf = srv.info()
            peak = max(peak, inf["resident_edges"])
            assert inf["resident_edges"] <= 12000 and inf["resident"] <= 8
            time.sleep(0.0005)
        for q, t in zip(qs, tickets):
            res = srv.wait(t)
            assert res["status"] == gesmc.OK
            rc, exp, _, _ = oracle.run(q["E"], q["n"], q["seed"], q["t0"], q["r"], q["pl"])
            assert np.array_equal(res["edges"], exp)
        with pytest.raises(gesmc.GesmcError) as ei:  # can never fit
            srv.submit(graphgen.gnp(2000, 0.01, 1), 2000, 1, 1)
        assert ei.value.status == gesmc.E_RANGE
    finally:
        srv.close()
        c.close()


def test_serve_bad_and_trivial_requests_do_not_disturb_others():
    gesmc = _gesmc()
    qs = requests(7, 10, 1e2, 5e3)
    bad = [
        (keys([(0, 1), (1, 2), (0, 1)]), 3, 2, gesmc.E_NOT_SIMPLE),                        # duplicate
        (np.array([(2 << 32) | 2, key(0, 1), key(1, 2)], dtype=np.uint64), 3, 3, gesmc.E_NOT_SIMPLE),  # loop
        (keys([(0, 1), (1, 7), (2, 3)]), 5, 1, gesmc.E_RANGE),                              # id >= n
        (keys([(0, 1), (0, 1)]), 2, 0, gesmc.E_NOT_SIMPLE),                                 # r = 0, duplicate
    ]
    trivial = [(keys([(3, 1)]), 4, 5), (np.zeros(0, dtype=np.uint64), 2, 3), (keys([(0, 1), (2, 3)]), 4, 0)]
    c = gesmc.Context(0)
    srv = gesmc.Server(c, hbm_budget_bytes=1 << 28)
    try:
        good_t = []
        bad_t = []
        triv_t = []
        for i, q in enumerate(qs):
            good_t.append(srv.submit(q["E"], q["n"], q["seed"], q["r"], t0=q["t0"], pl=q["pl"]))
            if i < len(bad):
                E, n, r, code = bad[i]
                bad_t.append((srv.submit(E, n, 1, r), code))
            if i < len(trivial):
                E, n, r = trivial[i]
                triv_t.append((srv.submit(E, n, 9, r), E, n, r))
        for (t, code) in bad_t:
            res = srv.wait(t)
            assert res["status"] == code and res["edges"] is None
        for (t, E, n, r) in triv_t:
            res = srv.wait(t)
            assert res["status"] == gesmc.OK
            rc, exp, _, _ = oracle.run(E, n, 9, 0, r)
            assert np.array_equal(res["edges"], exp)
        for q, t in zip(qs, good_t):
            res = srv.wait(t)
            assert res["status"] == gesmc.OK
            rc, exp, _, _ = oracle.run(q["E"], q["n"], q["seed"], q["t0"], q["r"], q["pl"])
            assert np.array_equal(res["edges"], exp)
    finally:
        srv.close()
        c.close()


def test_serve_cancel_and_poll():
    gesmc = _gesmc()
    E, n = graphgen.workload_powerlaw_1m()
    small = requests(9, 4, 1e2, 1e3)
    c = gesmc.Context(0)
    srv = gesmc.Server(c, hbm_budget_bytes=4 << 30)
    try:
        long_t = srv.submit(E, n, 5, 50)
        t_small = [srv.submit(q["E"], q["n"], q["seed"], q["r"], t0=q["t0"], pl=q["pl"]) for q in small]
        assert srv.poll(long_t) is None  # still running (50 supersteps of 6.6M edges)
        srv.cancel(long_t)
        res = srv.wait(long_t)
        assert res["status"] == gesmc.E_CANCELED and res["edges"] is None
        for q, t in zip(small, t_small):
            res = srv.wait(t)
            rc, exp, _, _ = oracle.run(q["E"], q["n"], q["seed"], q["t0"], q["r"], q["pl"])
            assert res["status"] == gesmc.OK and np.array_equal(res["edges"], exp)
        with pytest.raises(gesmc.GesmcError) as ei:  # ticket already taken
            srv.poll(long_t)
        assert ei.value.status == gesmc.E_INVAL
    finally:
        srv.close()
        c.close()


def test_serve_stream_with_cancels_bad_inputs_and_bursts():
    """A budget and graph limit that keep the queue blocked (long bursts of
    supersteps between completions), requests with 1..200 switches, bad
    inputs among them, cancels at random moments (queued, resident, done)
    and results taken by polling while others run.  Every request that was
    not cancelled returns the oracle's result and counts; a cancelled one
    returns E_CANCELED or, if it had already finished, its exact result."""
    gesmc = _gesmc()
    qs = requests(11, 48, 1e2, 5e3)
    rng = np.random.default_rng(11)
    for q in qs:
        if rng.random() < 0.3:
            q["r"] = int(rng.integers(40, 200))
    bad = [(keys([(0, 1), (1, 2), (0, 1), (2, 3)]), 4), (keys([(0, 5), (1, 2), (2, 3), (1, 2), (3, 4)]), 6)]
    c = gesmc.Context(0)
    srv = gesmc.Server(c, hbm_budget_bytes=136 * 40000, max_graphs=10)
    try:
        entries = []  # (ticket, query or None, expected bad status)
        early = set(int(x) for x in rng.choice(len(qs), 6, replace=False))  # cancelled right after submission
        for i, q in enumerate(qs):
            entries.append((srv.submit(q["E"], q["n"], q["seed"], q["r"], t0=q["t0"], pl=q["pl"]), q, None))
            if i in early:
                srv.cancel(entries[-1][0])
            if i % 16 == 7:
                E, n = bad[(i // 16) % len(bad)]
                entries.append((srv.submit(E, n, 3, 5), None, gesmc.E_NOT_SIMPLE))
            if i % 8 == 3:
                time.sleep(0.002)
        cancel = set(int(x) for x in rng.choice(len(qs), 12, replace=False))
        results = {}
        good_idx = [j for j, e in enumerate(entries) if e[1] is not None]
        for step, j in enumerate(good_idx):
            if step in cancel and j not in results:  # a taken ticket is unknown to the server
                srv.cancel(entries[j][0])
            if step % 5 == 0:  # take whatever is already done
                for jj, (t, _, _) in enumerate(entries):
                    if jj not in results:
                        res = srv.poll(t)
                        if res is not None:
                            results[jj] = res
            time.sleep(0.0005)
        for jj, (t, _, _) in enumerate(entries):
            if jj not in results:
                results[jj] = srv.wait(t)
        info = srv.info()
        print("server info:", info, flush=True)
        assert info["completed"] == len(entries)
        cancelled_steps = {good_idx[s] for s in cancel} | {good_idx[i] for i in early}
        n_cancelled = 0
        for jj, (t, q, bad_status) in enumerate(entries):
            res = results[jj]
            if q is None:
                assert res["status"] == bad_status and res["edges"] is None
                continue
            if jj in cancelled_steps and res["status"] == gesmc.E_CANCELED:
                assert res["edges"] is None
                n_cancelled += 1
                continue
            assert res["status"] == gesmc.OK, (jj, res["status"])
            rc, exp, counts, _ = oracle.run(q["E"], q["n"], q["seed"], q["t0"], q["r"], q["pl"])
            assert np.array_equal(res["edges"], exp), jj
            s = res["stats"]
            for k in ("attempts", "legal", "rej_loop", "rej_exists", "rej_pl"):
                assert s[k] == sum(cn[k] for cn in counts), (jj, k)
        print("cancelled before finishing:", n_cancelled, flush=True)
    finally:
        srv.close()
        c.close()


def test_serve_recipe_stream_exact():
    """Requests drawn as the benchmark's served stream draws them: power-law
    graphs with n log-uniform in [1e3, 1e6] (gamma in [2.1, 3.0], d_min 2,
    d_max floor(sqrt(n))), r uniform in 10..50, own seeds, Poisson arrivals
    at 300 requests/s.  Every result is checked exactly against the oracle
    (run on a thread pool), and a sample against gesmc_run alone."""
    import os
    import threading
    from concurrent.futures import ThreadPoolExecutor
    gesmc = _gesmc()
    pool = graphgen.batch_graphs(32, 5, 1e3, 1e6)
    rng = np.random.default_rng(1300)
    nreq = 40
    picks = rng.integers(0, len(pool), nreq)
    rs = rng.integers(10, 51, nreq)
    seeds = rng.integers(0, 2**63, nreq)
    gaps = rng.exponential(1.0 / 300.0, nreq)
    print("served recipe: %d requests, m up to %d" % (nreq, max(len(pool[p][0]) for p in picks)), flush=True)
    c = gesmc.Context(0)
    srv = gesmc.Server(c)
    tickets = [None] * nreq
    try:
        def producer():
            t_next = time.perf_counter()
            for i in range(nreq):
                t_next += gaps[i]
                d = t_next - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                E, n = pool[picks[i]]
                tickets[i] = srv.submit(E, n, int(seeds[i]), int(rs[i]))

        th = threading.Thread(target=producer)
        th.start()
        oracle._load()

        def one(i):
            E, n = pool[picks[i]]
            return oracle.run(E, n, int(seeds[i]), 0, int(rs[i]), 0)

        with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
            exp = list(ex.map(one, range(nreq)))
        th.join()
        results = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
        c.close()
    ref = gesmc.Context(0)
    try:
        for i, (res, (rc, e, counts, _)) in enumerate(zip(results, exp)):
            assert rc == 0 and res["status"] == gesmc.OK, i
            assert np.array_equal(res["edges"], e), "request %d (m=%d, r=%d)" % (i, len(e), rs[i])
            for k in ("attempts", "legal", "rej_loop", "rej_exists", "rej_pl"):
                assert res["stats"][k] == sum(cn[k] for cn in counts), (i, k)
        for i in range(0, nreq, 8):
            E, n = pool[picks[i]]
            q = dict(E=E, n=n, seed=int(seeds[i]), t0=0, r=int(rs[i]), pl=0)
            assert np.array_equal(results[i]["edges"], alone(ref, q)), i
    finally:
        ref.close()


def test_serve_destroy_while_a_thread_waits():
    """gesmc_server_destroy with threads blocked in gesmc_wait: they return
    (their requests cancelled, or finished if they got that far) before the
    server is freed, and destroy returns."""
    import threading
    gesmc = _gesmc()
    E = graphgen.powerlaw_graph(400000, 2.3, 2, 632, 9)
    c = gesmc.Context(0)
    srv = gesmc.Server(c)
    got = {}
    try:
        tickets = [srv.submit(E, 400000, s, 2000) for s in range(4)]  # about a second of work

        def waiter(t):
            got[t] = srv.wait(t)

        ths = [threading.Thread(target=waiter, args=(t,)) for t in tickets]
        for th in ths:
            th.start()
        time.sleep(0.2)  # the waiters are blocked inside gesmc_wait by now
        srv.close()  # destroy while they block
        for th in ths:
            th.join(timeout=60)
            assert not th.is_alive()
    finally:
        srv.close()
        c.close()
    assert sorted(got) == sorted(tickets)
    for t, res in got.items():
        assert res["status"] in (gesmc.OK, gesmc.E_CANCELED), res["status"]

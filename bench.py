"""Benchmark of the G-ES-MC global switch on one MI355X.

Headline (value): the plain form on G(n,p) with n=2^22 and average degree 32
(m = 67,125,011, 10 global switches per step), the HBM-bound instance.  A
step is one call of the library: input edges resident in HBM -> load and
validation -> r global switches (permutation, dependency resolution, rounds
of decisions) -> edges back in position order.  The value is switch attempts
per second over the timed steps (floor(m/2) attempts per superstep, rejected
ones included), the convention of the paper's runtime table (init +
supersteps).  The same line carries the other plain workloads (power-law
n=2^20, G(1024, 10/1023)) under plain_<name>, the batched form (4096 graphs
in one call, beside the plain form looping over the same graphs) and the
served form (Poisson request streams: p50 / p99 latency and attempts/s).

Prints ONE JSON line on stdout; diagnostics go to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "edge-switch attempts/sec (1 GPU), batched/served vs plain; p50/p99 latency"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per work item of each kernel (item = the unit the library
# counts for that kernel: edges m, switches ell, or table slots).  Random table
# touches count the 16-byte slot read and written back; records are 12 bytes
# (4-byte index + 8-byte key).
def kernel_bytes(name: str, m: int, ell: int, tb: int = 12) -> float | None:
    """Algorithmic HBM bytes of one launch over m records / ell switches;
    tb is the dependency tuple size the call reported (12, or 8 packed)."""
    return {
        "k_counts1": 4.0 * m,                            # index of every record (keys recomputed)
        "k_scatter1": 24.0 * m,                          # read + write one 12-byte record per edge
        "k_counts2": 4.0 * m,
        "k_scatter2": 24.0 * m,
        "k_sort_buckets": 24.0 * m,
        "k_build": 24.0 * ell + 8.0 * ell + 4 * 32.0 * ell,  # table strategy: pair records, slot ids, 4 slot RMWs
        "k_decide_first": 24.0 * ell + 8.0 * ell + 2 * 8.0 * ell + 24.0 * ell + 2.0 * ell,
        "k_unpermute": 12.0 * m + 8.0 * m,
        "k_load": 8.0 * m + 12.0 * m,
        # sorted-tuples dependency resolution: 4 tuples of tb bytes per switch
        "k_emit": 24.0 * ell + 16.0 * ell + 1.0 * ell,   # pair records in, free target records + statuses out
        "k_tcounts1": 24.0 * ell + 16.0 * ell + 1.0 * ell,  # the emit fused in: as k_emit
        "k_tscatter1": 24.0 * ell + 4.0 * tb * ell,      # pair records in, partitioned tuples out
        "k_tcounts2": 32.0 * ell,                        # the 8-byte key (or packed) word of each tuple
        "k_tscatter2": 8.0 * tb * ell,
        "k_resolve": 4.0 * tb * ell,                     # tuples in (records out are rare)
        "k_decide_chain1": 16.0 * ell + 24.0 * ell + 24.0 * ell + 2.0 * ell,
    }.get(name)


def switch_roofline(value: float, legal_fraction: float, G: float | None):
    """Attempts/s against the HBM bound of the method's own traffic: per
    attempt 2 source reads and 2 target probes, and for an accepted switch 2
    edge writes plus 2 erases and 2 inserts in the edge set (2 touches each),
    every random touch one G-byte DRAM transaction, plus 16 streaming bytes of
    the permutation: B_txn = G (4 + 10 a) + 16; B_alg = 48 + 48 a at byte
    level.  G is the transaction size measured for isolated random 8-byte
    reads (profiles/gather_calibration.json); None if it was never measured."""
    a = legal_fraction
    b_alg = 48 + 48 * a
    bound_alg = HBM_PEAK_GBS * 1e9 / b_alg  # byte-level lower bound on the traffic: an upper bound on attempts/s
    out = {"bytes_per_attempt_alg": round(b_alg, 1), "bound_attempts_per_s_alg": round(bound_alg, 1),
           "frac_alg": round(value / bound_alg, 4), "G_bytes": None}
    if G:
        b_txn = G * (4 + 10 * a) + 16
        bound = HBM_PEAK_GBS * 1e9 / b_txn
        out.update({"G_bytes": round(G, 1), "G_source": "profiles/gather_calibration.json",
                    "bytes_per_attempt_txn": round(b_txn, 1), "bound_attempts_per_s": round(bound, 1),
                    "frac": round(value / bound, 4)})
    return out


# The kernel sources of the plain path's supersteps: HBM counters taken on
# them stay valid while these files are unchanged.
PLAIN_KERNEL_SOURCES = ("device_common.h", "perm_kernels.h", "resolve_kernels.h", "switch_kernels.h", "tuple_pack.h")


def source_digest() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2111_03005_amd", "csrc")
    for f in PLAIN_KERNEL_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def _profile_json(name: str):
    try:
        with open(os.path.join(ROOT, "profiles", name)) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return None


def load_traffic(workload: str):
    """Per-kernel HBM bytes per launch from committed rocprofv3 counter runs
    (read and write request counts by size), if they were taken on the
    current kernel sources; else None."""
    d = _profile_json("traffic.json")
    if not d or d.get("source_digest") != source_digest():
        return None
    return d.get("kernels", {}).get(workload)


def measured_G():
    """DRAM transaction bytes per isolated random 8-byte read, measured with
    the request-size counters on a random gather (bench.py --gather-calibration)."""
    d = _profile_json("gather_calibration.json")
    return d.get("G_bytes") if d else None


def host_cpu():
    """(CPU model, logical CPUs) of the host running the bench."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline_batch(graphs, seeds, r, stride, threads):
    """The oracle on every stride-th graph of a batch, one graph per task on
    a thread pool (the oracle's C calls release the GIL)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    oracle._load()
    sample = list(range(0, len(graphs), stride))

    def one(g):
        E, n = graphs[g]
        rc, _, counts, _ = oracle.run(E, n, seeds[g], 0, r, 0)
        return sum(c["attempts"] for c in counts)

    t = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        att = sum(ex.map(one, sample))
    dt = time.perf_counter() - t
    return att / dt, dt, len(sample)


def cpu_baseline(E, n, r_sample, seed):
    import oracle
    oracle._load()
    t = time.perf_counter()
    rc, _, counts, _ = oracle.run(E, n, seed, 0, r_sample, 0)
    dt = time.perf_counter() - t
    att = sum(c["attempts"] for c in counts)
    return att / dt, dt


def bench_batched(gesmc, torch, args, plain_value):
    """The 4096-graph batch: one gesmc_run_batch call (20 global switches of
    every graph) per step, beside the plain path looping over the same graphs."""
    import graphgen
    t = time.perf_counter()
    graphs = graphgen.workload_batch_4096()
    E, offs, ns = graphgen.concat(graphs)
    print("batched: %d graphs, %d edges generated in %.1f s" % (len(graphs), offs[-1], time.perf_counter() - t),
          file=sys.stderr)
    G = len(graphs)
    seeds = [args.seed + g for g in range(G)]
    rs = [20] * G
    attempts = sum(20 * (int(m) // 2) for m in np.diff(offs))
    ctx = gesmc.Context(0)
    d_in = torch.from_numpy(E.view(np.int64).copy()).to("cuda")
    d_out = torch.empty_like(d_in)
    tuning = ctx.autotune_batch(d_in, offs, ns, seeds, supersteps=2)  # options only; results never change
    print("batched: autotuner chose %s" % tuning, file=sys.stderr)
    ctx.run_batch(d_in, offs, ns, seeds, rs, out=d_out, stats=False)  # warm-up
    torch.cuda.synchronize()
    times = []
    for _ in range(args.batch_steps):
        t = time.perf_counter()
        ctx.run_batch(d_in, offs, ns, seeds, rs, out=d_out, stats=False)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    wall = sum(times)
    value = attempts * len(times) / wall
    # the outcome counts of one more call (untimed) for the roofline's legal fraction
    _, _, tot = ctx.run_batch(d_in, offs, ns, seeds, rs, out=d_out, stats=True)
    legal_fraction = tot["legal"] / max(tot["attempts"], 1)
    # the same calls replayed from a hipGraph (captured on the second call of this shape)
    ctx.set_option(gesmc.OPT_GRAPH, 1)
    for _ in range(2):
        ctx.run_batch(d_in, offs, ns, seeds, rs, out=d_out, stats=False)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.batch_steps):
        ctx.run_batch(d_in, offs, ns, seeds, rs, out=d_out, stats=False)
    torch.cuda.synchronize()
    gwall = time.perf_counter() - t
    ctx.set_option(gesmc.OPT_GRAPH, 0)
    graph_rec = {"value": round(attempts * args.batch_steps / gwall, 1), "unit": "attempts/s",
                 "ms_per_step": round(1e3 * gwall / args.batch_steps, 3), "vs_eager": round(wall / gwall, 3)}
    print("batched: hipGraph replay %s" % graph_rec, file=sys.stderr)
    # the plain path (one gesmc_run per graph) on a sample of the same graphs
    sample = list(range(0, G, args.plain_sample_stride))
    dev_graphs = [(torch.from_numpy(graphs[g][0].view(np.int64).copy()).to("cuda"), graphs[g][1]) for g in sample]
    for d, n in dev_graphs[:4]:
        ctx.run(d, n, 1, 0, 20)
    torch.cuda.synchronize()
    t = time.perf_counter()
    att_plain = 0
    for g, (d, n) in zip(sample, dev_graphs):
        ctx.run(d, n, seeds[g], 0, 20)
        att_plain += 20 * (d.numel() // 2)
    torch.cuda.synchronize()
    plain_same = att_plain / (time.perf_counter() - t)
    ctx.close()
    print("batched: %.3e attempts/s (%.1f ms per batch); plain loop on every %dth graph: %.3e attempts/s" % (
        value, 1e3 * wall / len(times), args.plain_sample_stride, plain_same), file=sys.stderr)
    cpu_b = None
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)  # the machine's CPU share per GPU
        v, dt, ns_ = cpu_baseline_batch(graphs, seeds, 20, 16, threads)
        cpu_b = {"value": round(v, 1), "unit": "attempts/s", "cores": threads, "kind": "oracle",
                 "sample": "every 16th graph (%d graphs), 20 supersteps each, one graph per task on %d threads "
                           "(%.1f s)" % (ns_, threads, dt)}
        print("batched: oracle %s" % cpu_b, file=sys.stderr)
    small = bench_small_batches(gesmc, torch, args)
    return {"value": round(value, 1), "unit": "attempts/s", "steps": len(times),
            "ms_per_step": round(1e3 * wall / len(times), 3), "graphs": G, "edges": int(offs[-1]),
            "supersteps_per_graph": 20, "attempts_per_step": attempts,
            "workload": "4096 power-law graphs, n log-uniform [1e2,1e5], gamma U[2.1,3.0], d_min 2, "
                        "d_max floor(sqrt(n)), Havel-Hakimi, generator seed 4, Philox seeds 42+g",
            "plain_same_graphs": {"value": round(plain_same, 1), "unit": "attempts/s",
                                  "sample": "gesmc_run per graph on every %dth graph (%d graphs)" % (
                                      args.plain_sample_stride, len(sample))},
            "vs_plain_same_graphs": round(value / plain_same, 2),
            "autotuner": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in tuning.items()},
            "vs_plain_headline": round(value / plain_value, 3) if plain_value else None,
            "legal_fraction": round(legal_fraction, 5),
            "switch_roofline": switch_roofline(value, legal_fraction, measured_G()),
            "cpu_baseline": cpu_b,
            "hipgraph_replay": graph_rec,
            "small_batches_hipgraph": small}


def bench_small_batches(gesmc, torch, args):
    """Launch-bound shapes, eager vs replayed from a hipGraph (GESMC_OPT_GRAPH):
    64 small power-law graphs (n log-uniform [1e2, 1e3]) with 20 switches each,
    and the G(1024, 10/1023) graph alone (a batch of one) with 10."""
    import graphgen
    out = {}
    shapes = {"64 graphs n in [1e2,1e3], r=20": (graphgen.batch_graphs(64, 6, 1e2, 1e3), 20),
              "gnp_n1024_d10 as a batch of one, r=10": ([graphgen.workload_gnp_small()], 10)}
    stream = torch.cuda.Stream()
    for name, (graphs, r) in shapes.items():
        E, offs, ns = graphgen.concat(graphs)
        G = len(graphs)
        attempts = sum(r * (int(m) // 2) for m in np.diff(offs))
        res = {}
        for mode in (0, 1):
            ctx = gesmc.Context(0)
            ctx.set_option(gesmc.OPT_GRAPH, mode)
            d_in = torch.from_numpy(E.view(np.int64).copy()).to("cuda")
            d_out = torch.empty_like(d_in)
            with torch.cuda.stream(stream):
                for w in range(3):  # eager, capture, first replay
                    ctx.run_batch(d_in, offs, ns, [args.seed + g + w for g in range(G)], [r] * G, out=d_out,
                                  stream=stream, stats=False)
                stream.synchronize()
                calls = 20
                t = time.perf_counter()
                for i in range(calls):
                    ctx.run_batch(d_in, offs, ns, [args.seed + g + i for g in range(G)], [r] * G, out=d_out,
                                  stream=stream, stats=False)
                stream.synchronize()
                dt = (time.perf_counter() - t) / calls
            ctx.close()
            res["graph" if mode else "eager"] = {"ms_per_call": round(1e3 * dt, 3),
                                                "attempts_per_s": round(attempts / dt, 1)}
        res["speedup"] = round(res["eager"]["ms_per_call"] / res["graph"]["ms_per_call"], 2)
        print("small batch %s: %s" % (name, res), file=sys.stderr)
        out[name] = res
    return out


def bench_served(gesmc, torch, args):
    """Open-loop Poisson request stream against the serving loop, per rate:
    p50 / p99 latency (completion - submission, server clock) and attempts/s."""
    import threading

    import graphgen
    t = time.perf_counter()
    pool = graphgen.batch_graphs(args.serve_pool, 5, 1e3, 1e6)
    print("served: pool of %d graphs generated in %.1f s" % (len(pool), time.perf_counter() - t), file=sys.stderr)
    out = []
    for rate, budget in [(x, args.serve_budget) for x in args.serve_rates] + [(args.serve_rates[-1], 1 << 30)]:
        rng = np.random.default_rng(1000 + int(rate))
        # at low rates, about serve_window seconds of arrivals (at least 40 requests)
        nreq = min(args.serve_requests, max(40, int(rate * args.serve_window)))
        picks = rng.integers(0, len(pool), nreq)
        rs = rng.integers(10, 51, nreq)
        seeds = rng.integers(0, 2**63, nreq)
        gaps = rng.exponential(1.0 / rate, nreq)
        ctx = gesmc.Context(0)
        srv = gesmc.Server(ctx, hbm_budget_bytes=budget)
        tickets = [None] * nreq

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
        th.join()
        res = [srv.wait(tk) for tk in tickets]
        info = srv.info()
        srv.close()
        ctx.close()
        bad = sum(1 for x in res if x["status"] != gesmc.OK)
        lat = np.array([x["t_done"] - x["t_submit"] for x in res]) * 1e3
        att = sum(x["stats"]["attempts"] for x in res)
        span = max(x["t_done"] for x in res) - min(x["t_submit"] for x in res)
        rec = {"rate_req_per_s": rate, "requests": nreq, "hbm_budget_bytes": budget, "failed": bad,
               "p50_ms": round(float(np.percentile(lat, 50)), 2), "p99_ms": round(float(np.percentile(lat, 99)), 2),
               "attempts_per_s": round(att / span, 1),
               "attempts_per_busy_s": round(info["attempts"] / max(info["busy_s"], 1e-9), 1),
               "iterations": info["iterations"],
               "busy_fraction": round(info["busy_s"] / max(info["now_s"], 1e-9), 3),
               "host_copy_fraction": round(info["copy_s"] / max(info["busy_s"], 1e-9), 3),
               "device_wait_fraction": round(info["wait_s"] / max(info["busy_s"], 1e-9), 3)}
        print("served: %s" % rec, file=sys.stderr)
        out.append(rec)
    # the plain form on the same kind of stream: gesmc_run on the requests one after
    # another (a bounded sample of the highest rate's requests, no arrival gaps)
    rng = np.random.default_rng(1000 + int(args.serve_rates[-1]))
    picks = rng.integers(0, len(pool), args.serve_requests)
    rs = rng.integers(10, 51, args.serve_requests)
    seeds = rng.integers(0, 2**63, args.serve_requests)
    ctx = gesmc.Context(0)
    sample = list(range(0, args.serve_requests, 4))
    devs = [torch.from_numpy(pool[picks[i]][0].view(np.int64).copy()).to("cuda") for i in sample]
    for d, i in list(zip(devs, sample))[:4]:
        ctx.run(d, pool[picks[i]][1], 1, 0, 2)
    torch.cuda.synchronize()
    t = time.perf_counter()
    att = 0
    for d, i in zip(devs, sample):
        ctx.run(d, pool[picks[i]][1], int(seeds[i]), 0, int(rs[i]))
        att += int(rs[i]) * (d.numel() // 2)
    torch.cuda.synchronize()
    plain = att / (time.perf_counter() - t)
    ctx.close()
    del devs
    best = max(x["attempts_per_s"] for x in out)
    print("served: plain gesmc_run on every 4th request of the %g req/s stream: %.3e attempts/s" % (
        args.serve_rates[-1], plain), file=sys.stderr)
    return {"unit": "attempts/s", "per_rate": out,
            "plain_same_requests": {"value": round(plain, 1), "unit": "attempts/s",
                                    "sample": "gesmc_run one request after another, every 4th request of the "
                                              "%g req/s stream (%d requests)" % (args.serve_rates[-1], len(sample))},
            "vs_plain_same_requests": round(best / plain, 3),
            "workload": "Poisson arrivals; requests drawn from a pool of %d power-law graphs (n log-uniform "
                        "[1e3,1e6], gamma U[2.1,3.0], d_min 2, d_max floor(sqrt(n)), generator seed 5), "
                        "r uniform in 10..50, own Philox seed" % len(pool)}


def bench_plain(gesmc, torch, args, workload: str, steps: int, warmup: int, host_api: bool = False):
    """The plain form on one named workload: whole gesmc_run calls (r global
    switches each) with the input resident in HBM.  Returns the record and
    the input (for the CPU baseline)."""
    import graphgen
    make, r = graphgen.WORKLOADS[workload]
    E, n = make()
    m = len(E)
    ell = m // 2
    dev = torch.device("cuda", 0)
    ctx = gesmc.Context(0)
    for opt in args.option:
        name, val = opt.split("=")
        ctx.set_option(getattr(gesmc, "OPT_" + name.upper()), int(val))
    d_in = torch.from_numpy(E.view(np.int64).copy()).to(dev)
    d_out = torch.empty_like(d_in)
    stream = torch.cuda.current_stream()

    # Warm-up: the first pass times every kernel (events between all launches)
    # to find the dominant one; the timed steps then carry events around that
    # kernel only, on the launch stream, so the clock around them is barely
    # disturbed.
    ctx.set_option(gesmc.OPT_PROFILE, 0 if args.no_profile else 1)
    ctx.set_option(gesmc.OPT_PROFILE_ONLY, -1)
    ctx.profile_reset()
    wst = None
    for w in range(max(warmup, 1)):
        _, wst = ctx.run(d_in, n, args.seed, 0, r, 0, out=d_out, stream=stream)
        if w == 0:
            torch.cuda.synchronize()
            ctx.set_option(gesmc.OPT_PROFILE, 0)
    torch.cuda.synchronize()
    warm_prof = ctx.profile()
    tb = int(wst["tuple_bytes"]) or 12
    dominant = None
    for name, (ms, launches, items) in sorted(warm_prof.items(), key=lambda kv: -kv[1][0]):
        print("%s warm-up kernel %-16s total %9.3f ms  launches %5d" % (workload, name, ms, launches),
              file=sys.stderr)
        if dominant is None and kernel_bytes(name, m, ell, tb) is not None:
            dominant = name
    warm_total = sum(v[0] for v in warm_prof.values())

    if dominant is not None:
        ctx.set_option(gesmc.OPT_PROFILE, 1)
        ctx.set_option(gesmc.OPT_PROFILE_ONLY, gesmc.Context.kernel_names().index(dominant))
    ctx.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    step_ms = []
    for _ in range(steps):
        _, stats = ctx.run(d_in, n, args.seed, 0, r, 0, out=d_out, stream=stream)
        step_ms.append(stats["ms_device"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.set_option(gesmc.OPT_PROFILE, 0)
    ctx.set_option(gesmc.OPT_PROFILE_ONLY, -1)
    prof = ctx.profile()
    # per-superstep records of one more call (outside the timed region): the
    # exact slow paths taken (partitions over the LDS capacity) and the rounds
    _, _, step_recs = ctx.run(d_in, n, args.seed, 0, r, 0, out=d_out, stream=stream, steps=True)
    torch.cuda.synchronize()

    value = steps * r * ell / wall
    a = stats["legal"] / max(stats["attempts"], 1)
    traffic = load_traffic(workload) or {}
    roofline = None
    if dominant is not None and dominant in prof:
        ms, launches, items = prof[dominant]
        b = kernel_bytes(dominant, m, ell, tb)
        avg_s = ms / launches / 1e3
        achieved = b / avg_s / 1e9
        print("%s timed kernel %s: %d launches, avg %.4f ms, %.0f GB/s" % (
            workload, dominant, launches, avg_s * 1e3, achieved), file=sys.stderr)
        tr = traffic.get(dominant)
        roofline = {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": tr["bytes_per_launch"] if tr else None,
                    "traffic_over_alg": round(tr["bytes_per_launch"] / b, 3) if tr else None,
                    "bytes_per_launch": b, "avg_launch_ms": round(avg_s * 1e3, 4),
                    "share_of_step": round(ms / (wall * 1e3), 3)}
    # whole-superstep HBM traffic from the counter runs (every kernel of a
    # superstep), over the measured time per superstep
    step_traffic = None
    if traffic:
        per_step = sum(v["bytes_per_launch"] * v.get("launches_per_superstep", 1) for v in traffic.values())
        s_per_superstep = wall / (steps * r)
        step_traffic = {"bytes_per_superstep": round(per_step), "bytes_per_attempt": round(per_step / ell, 1),
                        "achieved_GBs": round(per_step / s_per_superstep / 1e9, 1),
                        "frac": round(per_step / s_per_superstep / 1e9 / HBM_PEAK_GBS, 4)}
    rec = {"workload": workload, "value": round(value, 1), "unit": "attempts/s", "n": n, "m": m,
           "supersteps_per_step": r, "attempts_per_step": r * ell, "steps": steps,
           "ms_per_step": round(1000.0 * wall / steps, 3),
           "step_ms_device_p50": round(float(np.median(step_ms)), 3) if step_ms else None,
           "legal_fraction": round(a, 5), "rounds_max": stats["rounds_max"],
           "tuple_bytes": int(stats["tuple_bytes"]), "timed_kernel_events": dominant,
           "kernel_share_warmup": {k: round(v[0] / warm_total, 3) for k, v in warm_prof.items()} if warm_total else None,
           "fallback_buckets_per_superstep": round(sum(q["fallback_buckets"] for q in step_recs) / max(r, 1), 2),
           "rounds_mean": round(sum(q["rounds"] for q in step_recs) / max(r, 1), 2),
           "roofline": roofline, "superstep_traffic": step_traffic,
           "switch_roofline": switch_roofline(value, a, measured_G())}
    if host_api:
        # the host entry point on the same workload: edges in and out of host
        # memory, so both PCIe copies are inside the time (never the headline)
        uv = np.stack([(E >> np.uint64(32)).astype(np.uint32), (E & np.uint64(0xFFFFFFFF)).astype(np.uint32)], 1)
        ctx.run_host(uv, n, args.seed, 0, r)  # sizes its staging
        t = time.perf_counter()
        ctx.run_host(uv, n, args.seed, 0, r)
        dt_host = time.perf_counter() - t
        rec["host_api"] = {"value": round(r * ell / dt_host, 1), "unit": "attempts/s",
                           "ms_per_call": round(1e3 * dt_host, 3),
                           "note": "gesmc_run_host, %d supersteps per call, incl. host->device and device->host "
                                   "copies" % r}
    ctx.close()
    del d_in, d_out
    torch.cuda.empty_cache()
    print("%s: %.3e attempts/s (%.3f ms per %d-superstep call)" % (workload, value, rec["ms_per_step"], r),
          file=sys.stderr)
    return rec, E, n, r


def bench_es(gesmc, torch, args):
    """ParES (Alg. 2): the ES-MC chain on the power-law n=2^20 graph, r = m
    switches per call (input resident in HBM), beside the ES-MC oracle on a
    bounded sample of the same chain."""
    import graphgen
    E, n = graphgen.workload_powerlaw_1m()
    m = len(E)
    r = m
    ctx = gesmc.Context(0)
    d_in = torch.from_numpy(E.view(np.int64).copy()).to("cuda")
    d_out = torch.empty_like(d_in)
    ctx.run_es(d_in, n, args.seed, 0, r, out=d_out)  # warm-up (sizes the buffers)
    torch.cuda.synchronize()
    times, st = [], None
    for _ in range(args.es_steps):
        t = time.perf_counter()
        _, st = ctx.run_es(d_in, n, args.seed, 0, r, out=d_out)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    ctx.close()
    wall = sum(times)
    value = r * len(times) / wall
    rec = {"value": round(value, 1), "unit": "attempts/s", "workload": "pld_n2^20_g2.5", "m": m,
           "switches_per_step": r, "steps": len(times), "ms_per_step": round(1e3 * wall / len(times), 3),
           "supersteps": st["supersteps"], "mean_superstep": round(r / max(st["supersteps"], 1), 1),
           "rounds_max": st["rounds_max"], "legal_fraction": round(st["legal"] / max(st["attempts"], 1), 5),
           "epochs": st["epochs"]}
    if not args.no_cpu_baseline:
        import oracle
        oracle._load()
        sample = min(r, 4000000)
        t = time.perf_counter()
        oracle.es_run(E, n, args.seed, 0, sample)
        dt = time.perf_counter() - t
        rec["cpu_baseline"] = {"value": round(sample / dt, 1), "unit": "attempts/s", "cores": 1, "kind": "oracle",
                               "sample": "ES-MC oracle, first %d of the %d switches incl. validation and set build "
                                         "(%.1f s)" % (sample, r, dt)}
    print("ParES: %s" % rec, file=sys.stderr)
    return rec


def bench_mixing(gesmc, torch, args):
    """The mixing diagnostic of Sec. 6.1 on a point of its SynPld grid: a
    power-law graph with n = 2^13, gamma = 2.2, degrees in [1, n^(1/(gamma-1))],
    Havel-Hakimi; K supersteps of each chain with the thinned series of
    k = 1, 2, 4, ..., 64 aggregated on the device; beside the oracle (every
    state kept) on a bounded sample of the same run."""
    import graphgen
    n, gamma = 1 << 13, 2.2
    E = graphgen.powerlaw_graph(n, gamma, 1, int(n ** (1.0 / (gamma - 1.0))), 7)
    m = len(E)
    thin = [1, 2, 4, 8, 16, 32, 64]
    K = args.mixing_supersteps
    ctx = gesmc.Context(0)
    d = torch.from_numpy(E.view(np.int64).copy()).to("cuda")
    rec = {"workload": "SynPld n=2^13 gamma=2.2 d in [1, n^(1/(gamma-1))], Havel-Hakimi, generator seed 7",
           "m": m, "supersteps": K, "thinning": thin}
    for chain, name in ((0, "G-ES-MC"), (1, "ES-MC")):
        ctx.mixing(d, n, args.seed, 2, [1], chain=chain)  # warm-up
        t = time.perf_counter()
        res, ms = ctx.mixing(d, n, args.seed, K, thin, chain=chain)
        dt = time.perf_counter() - t
        rec[name] = {"ms": round(1e3 * dt, 1), "attempts_per_s": round(K * (m // 2) / dt, 1),
                     "fraction_not_independent": {r["k"]: round(r["non_independent"] / max(r["tracked"], 1), 5)
                                                  for r in res}}
    ctx.close()
    if not args.no_cpu_baseline:
        from oracle import mixing
        Ks = min(K, 50)
        t = time.perf_counter()
        mixing.diagnostic(E, n, args.seed, Ks, thin, chain="global")
        dt = time.perf_counter() - t
        rec["cpu_baseline"] = {"value": round(Ks * (m // 2) / dt, 1), "unit": "attempts/s", "cores": 1,
                               "kind": "oracle", "sample": "G-ES-MC, first %d of the %d supersteps with every state "
                                                           "kept and the same thinning values (%.1f s)" % (Ks, K, dt)}
    print("mixing: %s" % rec, file=sys.stderr)
    return rec


def bench_generation(gesmc, torch, args):
    """Input realisation on the device (Sec. 6's synthetic families): G(n,p)
    at n = 2^22, p = 32/(n-1) (the G(n,p) benchmark input), and the power-law
    pipeline -- degrees, Havel-Hakimi, relabelling -- at n = 2^20, gamma =
    2.5, degrees in [5..1024]; beside the oracle's definitions on the CPU."""
    ctx = gesmc.Context(0)
    n, p, seed = 1 << 22, 32.0 / ((1 << 22) - 1), 3
    E = ctx.gen_gnp(n, p, seed)  # warm-up; sizes the output
    out = torch.empty(E.numel() + 1024, dtype=torch.int64, device="cuda")
    del E
    torch.cuda.synchronize()
    times = []
    for _ in range(3):
        t = time.perf_counter()
        E = ctx.gen_gnp(n, p, seed, out=out)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    m = E.numel()
    dt = float(np.median(times))
    rec = {"gnp": {"workload": "G(n=2^22, p=32/(2^22-1)), seed 3", "m": m, "ms": round(1e3 * dt, 3),
                   "edges_per_s": round(m / dt, 1), "written_GBs": round(8 * m / dt / 1e9, 1),
                   "note": "counting pass, scan and writing pass; Philox and a portable ln per draw"}}
    del out, E
    pn, gamma, dmin, dmax, pseed = 1 << 20, 2.5, 5, 1024, 2
    ctx.gen_powerlaw_graph(pn, gamma, dmin, dmax, pseed)  # warm-up
    torch.cuda.synchronize()
    ph = {}
    t = time.perf_counter()
    deg, _ = ctx.gen_pld_degrees(pn, gamma, dmin, dmax, pseed)
    torch.cuda.synchronize()
    ph["degrees_ms"] = 1e3 * (time.perf_counter() - t)
    ctx.set_option(gesmc.OPT_PROFILE, 1)
    ctx.profile_reset()
    t = time.perf_counter()
    H = ctx.gen_havel_hakimi(deg)
    torch.cuda.synchronize()
    ph["havel_hakimi_ms"] = 1e3 * (time.perf_counter() - t)
    prof = ctx.profile()
    ctx.set_option(gesmc.OPT_PROFILE, 0)
    t = time.perf_counter()
    ctx.gen_relabel(H, pn, pseed)
    torch.cuda.synchronize()
    ph["relabel_ms"] = 1e3 * (time.perf_counter() - t)
    pm = H.numel()
    total = sum(ph.values())
    rec["powerlaw"] = {"workload": "Pld([5..1024], 2.5) on n=2^20, Havel-Hakimi, relabelled, seed 2", "m": pm,
                       **{k: round(v, 3) for k, v in ph.items()}, "ms": round(total, 3),
                       "edges_per_s": round(pm / total * 1e3, 1),
                       "hh_steps_kernel_ms": round(prof.get("k_hh_steps", (0.0,))[0], 3)}
    del H, deg
    ctx.close()
    if not args.no_cpu_baseline:
        import oracle
        oracle._load()
        t = time.perf_counter()
        Eo = oracle.gen_gnp(1 << 20, 32.0 / ((1 << 20) - 1), seed)
        dg = time.perf_counter() - t
        t = time.perf_counter()
        d0 = oracle.gen_pld(pn, gamma, dmin, dmax, pseed)[0]
        Ho = oracle.gen_havel_hakimi(d0)
        oracle.gen_relabel(Ho, pn, pseed)
        dp = time.perf_counter() - t
        rec["cpu_baseline"] = {"gnp_edges_per_s": round(len(Eo) / dg, 1), "powerlaw_edges_per_s": round(len(Ho) / dp, 1),
                               "cores": 1, "kind": "oracle",
                               "sample": "G(n=2^20, p=32/(2^20-1)) (%.1f s); the whole power-law pipeline (%.1f s)"
                                         % (dg, dp)}
    print("generation: %s" % rec, file=sys.stderr)
    return rec


def bench_classes(gesmc, torch, args):
    """G-ES-MC on other graph classes (Sec. 1): random graphs with n = 2^20
    and m = 2^22 of the classes with loops, directed, and with loops and
    multi-edges, 5 supersteps per call with the input resident in HBM."""
    import graphgen
    ctx = gesmc.Context(0)
    n, m, r = 1 << 20, 1 << 22, 5
    rec = {"workload": "class_graph(n=2^20, m=2^22), 5 supersteps per call", "n": n, "m": m}
    for cls, name in ((1, "loops"), (4, "directed"), (3, "loops_multi")):
        E = graphgen.class_graph(n, m, cls, 60 + cls)
        d_in = torch.from_numpy(E.view(np.int64).copy()).to("cuda")
        d_out = torch.empty_like(d_in)
        ctx.run_class(d_in, n, args.seed, cls, r=r, out=d_out)  # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        steps = 3
        st = None
        for _ in range(steps):
            _, st, _, _ = ctx.run_class(d_in, n, args.seed, cls, r=r, out=d_out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        rec[name] = {"cls": cls, "value": round(steps * r * (m // 2) / dt, 1), "unit": "attempts/s",
                     "legal_fraction": round(st["legal"] / max(st["attempts"], 1), 5)}
        del d_in, d_out
    ctx.close()
    print("classes: %s" % rec, file=sys.stderr)
    return rec


def gather_calibration(mib: int, count: int):
    """Isolated random 8-byte reads: index_select of `count` random int64
    words from a `mib` MiB buffer, three times.  Under rocprofv3's read
    request-size counters this gives the DRAM bytes moved per random 8-byte
    read (the gather kernel also streams its index array and output)."""
    import torch
    words = (mib << 20) // 8
    src = torch.arange(words, dtype=torch.int64, device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    idx = torch.randint(0, words, (count,), dtype=torch.int64, device="cuda", generator=g)
    out = None
    for _ in range(3):
        out = torch.index_select(src, 0, idx)
    torch.cuda.synchronize()
    assert int(out[0]) == int(idx[0])
    print(json.dumps({"gather_calibration_buffer_bytes": words * 8, "gathers": count, "repeats": 3,
                      "streamed_bytes_per_gather": 16}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="gnp_n2^22_d32", help="the headline workload (plain form)")
    ap.add_argument("--extra-workloads", nargs="*", default=["pld_n2^20_g2.5", "gnp_n1024_d10", "pld_n2^20_g2.01"],
                    help="further plain workloads reported under plain_<name>")
    ap.add_argument("--seed", type=int, default=42)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-supersteps", type=int, default=1)
    ap.add_argument("--no-profile", action="store_true", help="no kernel events at all (no roofline)")
    ap.add_argument("--option", action="append", default=[], metavar="NAME=VALUE",
                    help="library option (e.g. PERSIST=2, STRATEGY=1); results never depend on options")
    ap.add_argument("--no-batched", action="store_true", help="skip the 4096-graph batch")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--plain-sample-stride", type=int, default=8)
    ap.add_argument("--no-served", action="store_true", help="skip the serving sweep")
    ap.add_argument("--serve-rates", type=float, nargs="+", default=[10.0, 30.0, 100.0, 300.0, 1000.0, 3000.0])
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests per rate (at most)")
    ap.add_argument("--serve-window", type=float, default=4.0,
                    help="seconds of arrivals per rate at low rates (at least 40 requests)")
    ap.add_argument("--serve-pool", type=int, default=128)
    ap.add_argument("--serve-budget", type=int, default=32 << 30, help="HBM budget of the server, bytes")
    ap.add_argument("--no-es", action="store_true", help="skip ParES (the ES-MC chain)")
    ap.add_argument("--no-mixing", action="store_true", help="skip the mixing diagnostic")
    ap.add_argument("--mixing-supersteps", type=int, default=400)
    ap.add_argument("--es-steps", type=int, default=3)
    ap.add_argument("--no-generation", action="store_true", help="skip the input realisation on the device")
    ap.add_argument("--no-classes", action="store_true", help="skip the graph classes")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 times): the reference for HBM counters")
    ap.add_argument("--gather-calibration", type=int, default=0, metavar="MIB",
                    help="only run 2^26 random 8-byte gathers from a MIB MiB buffer (3 times): the DRAM "
                         "transaction size of isolated random reads, from the request-size counters")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 3}))
        return
    if args.gather_calibration:
        gather_calibration(args.gather_calibration, 1 << 26)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(independent graphs would shard across GPUs without communication).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2111_03005_amd as gesmc

    head, E, n, r = bench_plain(gesmc, torch, args, args.workload, args.steps, args.warmup, host_api=True)
    extra = {}
    for w in args.extra_workloads:
        if w != args.workload:
            rec, _, _, _ = bench_plain(gesmc, torch, args, w, args.steps, args.warmup)
            extra["plain_" + w] = rec

    cpu = None
    if not args.no_cpu_baseline:
        rs = min(args.cpu_sample_supersteps, r)
        v, dt = cpu_baseline(E, n, rs, args.seed)
        model, nproc = host_cpu()
        cpu = {"value": round(v, 1), "unit": "attempts/s", "cores": 1, "kind": "oracle",
               "sample": "%s, first %d of %d supersteps incl. validation and set build (%.1f s)" % (
                   args.workload, rs, r, dt), "host_cpu": model, "host_logical_cpus": nproc}
        print("oracle: %s" % cpu, file=sys.stderr)
    del E

    es = None if args.no_es else bench_es(gesmc, torch, args)
    mix = None if args.no_mixing else bench_mixing(gesmc, torch, args)
    gen = None if args.no_generation else bench_generation(gesmc, torch, args)
    classes = None if args.no_classes else bench_classes(gesmc, torch, args)
    batched = None if args.no_batched else bench_batched(gesmc, torch, args, head["value"])
    served = None if args.no_served else bench_served(gesmc, torch, args)

    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(args.warmup, 1),
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": head["n"], "m": head["m"],
                   "supersteps_per_step": head["supersteps_per_step"],
                   "attempts_per_step": head["attempts_per_step"], "seed": args.seed, "pl": 0, "mode": "plain",
                   "legal_fraction": head["legal_fraction"], "rounds_max": head["rounds_max"],
                   "tuple_bytes": head["tuple_bytes"], "step_ms_device_p50": head["step_ms_device_p50"],
                   "timed_kernel_events": head["timed_kernel_events"] if not args.no_profile else None,
                   "options": args.option},
        "roofline": head["roofline"],
        "superstep_traffic": head["superstep_traffic"],
        "switch_roofline": head["switch_roofline"],
        "kernel_share_warmup": head["kernel_share_warmup"],
        "host_api": head.get("host_api"),
        "cpu_baseline": cpu,
    }
    out.update(extra)
    out["es_pares"] = es
    out["mixing"] = mix
    out["generation"] = gen
    out["classes"] = classes
    out["batched"] = batched
    out["served"] = served
    print(json.dumps(out))


if __name__ == "__main__":
    main()

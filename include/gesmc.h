/*
 * gesmc -- Global Edge Switching Markov Chain (G-ES-MC) on AMD MI355X (gfx950).
 *
 * C ABI of libgesmc.so.  The method is that of Allendorf, Meyer, Penschuck and
 * Tran, "Parallel Global Edge Switching for the Uniform Sampling of Simple
 * Graphs with Prescribed Degrees" (arXiv 2111.03005):
 *   - an edge switch (Def. 2.1) turns edges e1 = E[i], e2 = E[j] (canonical
 *     orientation) into tau(e1, e2, g) and is rejected if a new edge is a loop
 *     or already present;
 *   - a global switch (Def. 3.2) permutes the m edge indices uniformly and
 *     runs the floor(m/2) switches (pi[2k], pi[2k+1], [pi[2k] < pi[2k+1]]) in
 *     sequence, each one skipped independently with probability P_L (Sec. 3);
 *   - the driver (Alg. 3) applies r global switches; the result equals the
 *     sequential execution (Sec. 4), whatever the parallel schedule.
 *
 * Random choices are defined exactly with Philox4x32-10 (Salmon et al., SC'11)
 * keyed by (seed_lo, seed_hi): in superstep t the permutation sorts edge
 * indices by (K_i, i) with K_i = (x0 << 32) | x1 at counter (i, 0, t, 0), and
 * switch k is skipped iff x0 at counter (k, 0, t, 1) is below pl.  The output
 * is a deterministic function of (input edge order, n, seed, t0, r, pl).
 *
 * Edges are 64-bit keys (min << 32) | max (Sec. 5.1).  Vertex ids must be < n
 * and < 0xFFFFFFFF; m must be below 2^30.
 *
 * Threading: a context serves one host thread at a time.  Every call below
 * enqueues its work on `stream` (a hipStream_t passed as void*; NULL = the
 * default stream) and returns after the work has completed.
 */
#ifndef GESMC_H
#define GESMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gesmc_status;

#define GESMC_OK 0
#define GESMC_E_INVAL (-1)      /* bad pointer or argument                         */
#define GESMC_E_NOT_SIMPLE (-2) /* the input edge list has a loop or a duplicate   */
#define GESMC_E_RANGE (-3)      /* vertex id >= n or 0xFFFFFFFF, or m >= 2^30      */
#define GESMC_E_NOMEM (-4)      /* device allocation failed                        */
#define GESMC_E_DEVICE (-5)     /* HIP runtime error                               */
#define GESMC_E_AGAIN (-6)      /* server: queue full (submit) / not done (poll)   */
#define GESMC_E_CANCELED (-7)   /* server: the request was cancelled               */
#define GESMC_E_ROUNDS (-8)     /* a superstep exceeded GESMC_OPT_ROUND_LIMIT      */
#define GESMC_E_INTERNAL (-9)   /* an internal consistency check failed            */
#define GESMC_E_NOT_GRAPHICAL (-10) /* a degree sequence no simple graph realises  */

typedef struct gesmc_ctx gesmc_ctx;

/* Totals over one call. */
typedef struct gesmc_stats {
    uint64_t attempts;   /* floor(m/2) per superstep, rejected ones included   */
    uint64_t legal;      /* accepted switches                                   */
    uint64_t rej_loop;   /* rejected: a target is a loop                        */
    uint64_t rej_exists; /* rejected: a target is present when the switch runs  */
    uint64_t rej_pl;     /* skipped with probability P_L                        */
    uint64_t rounds_sum; /* dependency-resolution rounds summed over supersteps */
    uint32_t rounds_max; /* most rounds in one superstep                        */
    uint32_t supersteps; /* r                                                   */
    double ms_device;    /* device time of the whole call (HIP events)          */
    uint32_t tuple_bytes; /* bytes per dependency tuple in the call's last
                             superstep: 8 (packed words, GESMC_OPT_PACK_TUPLES),
                             12, or 0 if no superstep ran the tuple passes     */
    uint32_t reserved;   /* 0                                                   */
} gesmc_stats;

/* Per superstep (same meaning as above; `rounds` counts the decision rounds of
 * Alg. 1 as scheduled here: 1 + the rounds needed for delayed switches). */
typedef struct gesmc_step_stats {
    uint64_t attempts, legal, rej_loop, rej_exists, rej_pl;
    uint64_t rounds;
    uint64_t undecided_after_round1;
    uint64_t fallback_buckets; /* permutation buckets sorted by the slow exact path */
} gesmc_step_stats;

/* Creates a context on HIP device `hip_device`.  Device memory is allocated
 * lazily and kept for later calls (about 136 bytes per edge).  *out receives
 * the context; release it with gesmc_destroy. */
gesmc_status gesmc_create(int hip_device, gesmc_ctx **out);
void gesmc_destroy(gesmc_ctx *ctx);

/* Message of the last failing call on this host thread ("" if none). */
const char *gesmc_last_error(void);

/*
 * r global switches (Alg. 3) on the m edges at d_in (device memory, uint64
 * keys; a key (max << 32) | min is accepted and canonicalised).  The result,
 * canonical keys in position order, goes to d_out (device memory, m words; may
 * equal d_in).  Supersteps t0 .. t0+r-1 are run, so run(r1) followed by
 * run(r2, t0 = r1) equals run(r1 + r2).  pl: P_L = pl / 2^32 (0 = never skip).
 * flags: reserved, pass 0.  stats (host, nullable): totals; steps (host,
 * nullable): r records.  On any error d_out is left untouched and a negative
 * status is returned; GESMC_E_NOT_SIMPLE / GESMC_E_RANGE report invalid input.
 * m < 2 copies the canonicalised input.  A graph of at most 4096 edges (6144
 * with every vertex id below 2^16) runs its supersteps in one workgroup's LDS
 * (Sec. 7's base case for small graphs) when steps is NULL and
 * GESMC_OPT_SMALL_GRAPHS is on: per piece of up to 32 supersteps, one launch
 * computes their permutations and one runs the chain; its stats then count
 * no rounds.
 */
gesmc_status gesmc_run(gesmc_ctx *ctx, void *stream, const uint64_t *d_in, uint64_t *d_out, uint64_t m, uint32_t n,
                       uint64_t seed, uint32_t t0, uint32_t r, uint32_t pl, uint32_t flags, gesmc_stats *stats,
                       gesmc_step_stats *steps);

/*
 * Host convenience form of gesmc_run (Alg. 3 on an edge list in host memory):
 * uv holds the m input edges as 2m vertex ids (u0, v0, u1, v1, ...; either
 * orientation), uv_out (host, 2m ids, may equal uv) receives the result as
 * (min, max) pairs in position order.  Runs on the default stream of the
 * context's device and returns when the result is in uv_out; the edges go
 * through pinned staging and device buffers owned by the context, so the
 * time includes both PCIe copies.  Limits, flags, pl, stats and errors as in
 * gesmc_run; on error uv_out is left untouched.
 */
gesmc_status gesmc_run_host(gesmc_ctx *ctx, const uint32_t *uv, uint32_t *uv_out, uint64_t m, uint32_t n,
                            uint64_t seed, uint32_t t0, uint32_t r, uint32_t pl, uint32_t flags, gesmc_stats *stats);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): gesmc_run
 * with every per-call device buffer -- state records, dependency tuples,
 * radix counts, statuses, undecided lists, error words and counters -- taken
 * from one fixed device array of GESMC_NOALLOC_SCRATCH_MIB MiB that the
 * library holds on each device from the first gesmc_create on it until the
 * process ends.  This call allocates nothing (no hipMalloc, hipFree or
 * pinned host memory); the context's own buffers are left as they are.
 * Arguments, result, stats and errors as in gesmc_run (no per-superstep
 * records); m at most GESMC_NOALLOC_MAX_EDGES (else GESMC_E_RANGE and d_out
 * untouched); needs GESMC_OPT_STRATEGY 0.  Runs of more than 64 supersteps
 * go in pieces of 64 that resume one another (run(r1) then run(r2, t0 = r1)
 * equals run(r1 + r2)), so only an internal error or GESMC_E_ROUNDS in a
 * later piece can leave d_out holding the earlier pieces' result; input
 * errors leave it untouched.  Every call on a device shares that device's
 * array and keeps nothing in it between calls: calls that overlap on one
 * device (from any context or thread) race and must not be made.
 */
#define GESMC_NOALLOC_SCRATCH_MIB 256u
#define GESMC_NOALLOC_MAX_EDGES 2000000ull
gesmc_status gesmc_run_noalloc(gesmc_ctx *ctx, void *stream, const uint64_t *d_in, uint64_t *d_out, uint64_t m,
                               uint32_t n, uint64_t seed, uint32_t t0, uint32_t r, uint32_t pl, uint32_t flags,
                               gesmc_stats *stats);

/*
 * G independent graphs in one call: the batched form of gesmc_run.  Graph g
 * is d_in[offsets[g] .. offsets[g+1]) (device memory, uint64 keys of local
 * vertex ids < n[g]); it runs r[g] global switches from superstep t0[g] with
 * seed seed[g], and its result goes to the same range of d_out (device; may
 * equal d_in).  Every graph's result equals gesmc_run on that graph alone
 * with the same (n, seed, t0, r, pl) -- bit for bit, whatever the rest of the
 * batch holds.  Host arrays: offsets (G + 1 entries, offsets[0] = 0,
 * non-decreasing), n, seed and r (G each), t0 (G, nullable: all 0).
 * stats (host, nullable): G records, one per graph (attempts and outcome
 * counts of that graph; rounds_* count the batch's rounds of the supersteps
 * the graph took part in; ms_device is the whole call's).  total (host,
 * nullable): the batch's sums.  Limits: offsets[G] + G < 2^30, the sum of n
 * below 2^32 - 1, G <= 2^21, and at most 2^21 permutation buckets (about
 * offsets[G] / GESMC_OPT_BUCKET_AVG + G).  Needs GESMC_OPT_STRATEGY 0.  Any
 * invalid graph fails the whole call with d_out untouched; the message names
 * the graph.  flags: reserved, pass 0.
 */
gesmc_status gesmc_run_batch(gesmc_ctx *ctx, void *stream, uint32_t G, const uint64_t *d_in, uint64_t *d_out,
                             const uint64_t *offsets, const uint32_t *n, const uint64_t *seed, const uint32_t *t0,
                             const uint32_t *r, uint32_t pl, uint32_t flags, gesmc_stats *stats, gesmc_stats *total);

/*
 * One superstep t (as gesmc_run with t0 = t, r = 1) that also writes the
 * outcome of every switch k < floor(m/2) to d_outcome (device memory, one byte
 * per switch): 1 accepted, 2 rejected loop, 3 rejected target present,
 * 4 skipped (P_L).  Parity hook for the per-switch decisions (Def. 2.1).
 */
gesmc_status gesmc_superstep_outcomes(gesmc_ctx *ctx, void *stream, const uint64_t *d_in, uint64_t *d_out, uint64_t m,
                                      uint32_t n, uint64_t seed, uint32_t t, uint32_t pl, uint8_t *d_outcome,
                                      gesmc_step_stats *step);

/*
 * G-ES-MC on another graph class (Sec. 1 names directed graphs and graphs
 * with loops or multi-edges as classes the switch carries over to).  cls is
 * a set of bits: GESMC_CLASS_LOOPS (loops allowed), GESMC_CLASS_MULTI
 * (multi-edges allowed), GESMC_CLASS_DIRECTED; 0 is gesmc_run's simple
 * undirected graph.  The permutation, the pairs, P_L and g = [i < j] are as
 * for gesmc_run; the switch of a pair is:
 *   undirected: tau of Def. 2.1 on the canonical keys (smaller id high);
 *   directed: keys stay (tail << 32) | head as given and the switch
 *     exchanges the heads, (u->v), (x->y) -> (u->y), (x->v), for either g,
 *     keeping every out- and in-degree;
 *   rejected as a loop (code 2): a loop target where loops are not allowed;
 *     and, undirected with loops but no multi-edges, a switch with g = 1
 *     and a loop among its sources (its two g give the same targets, its
 *     reverse move only one; rejecting one keeps the chain symmetric, so
 *     the class's uniform distribution is stationary);
 *   rejected as present (code 3), without multi-edges only: a target that
 *     is an edge (Def. 2.1's rule, the switch's own sources included), or
 *     two equal targets.
 * With multi-edges every switch is decided from its own two edges, and the
 * chain balances the configuration model's weights (1 / the product of the
 * multiplicities' factorials, times 2^-loops undirected).  Input: ids < n,
 * loops only with GESMC_CLASS_LOOPS (else GESMC_E_NOT_SIMPLE), duplicates
 * (equal keys; directed (a,b) and (b,a) differ) only with GESMC_CLASS_MULTI
 * (else GESMC_E_NOT_SIMPLE).  Output: undirected canonical, directed as
 * stored, at the input positions.  d_outcome (device, nullable, floor(m/2)
 * bytes): the last superstep's codes as for gesmc_superstep_outcomes.
 * Other arguments, statistics and errors as for gesmc_run (no LDS small-
 * graph path; GESMC_E_INVAL for cls > 7).
 */
#define GESMC_CLASS_LOOPS 1u
#define GESMC_CLASS_MULTI 2u
#define GESMC_CLASS_DIRECTED 4u
gesmc_status gesmc_run_class(gesmc_ctx *ctx, void *stream, const uint64_t *d_in, uint64_t *d_out, uint64_t m,
                             uint32_t n, uint64_t seed, uint32_t t0, uint32_t r, uint32_t pl, uint32_t cls,
                             gesmc_stats *stats, gesmc_step_stats *steps, uint8_t *d_outcome);

/*
 * Input realisation on the device: the steps before the chain that build the
 * synthetic inputs of Sec. 6, G(n,p) graphs (SynGnp) and Havel-Hakimi
 * realisations of i.i.d. Pld([a..b], gamma) degree sequences (SynPld, Sec.
 * 2.1's notation), plus a random relabelling.  Each result is a function of
 * the arguments alone (any device, any launch shape):
 *
 *   Draws: Philox4x32-10 with key (seed_lo, seed_hi), counter tag 3 for
 *   G(n,p) and 4 for degrees (tags 0 .. 2 belong to the chain).  Where
 *   floating point decides an integer it goes through ln_p / exp_p, made of
 *   correctly rounded IEEE double steps in a fixed order, never fused:
 *     ln_p(x): x = 2^e m, m in [1, 2), if m > sqrt(2) then m /= 2, e += 1;
 *       f = m - 1, s = f / (2 + f), z = s s, P = 1/23 then P = P z + 1/(2j+1)
 *       for j = 10 .. 1, t = 2 s; ln_p = e LN2_HI + (e LN2_LO + (t + t (z P)))
 *       with fdlibm's LN2_HI = 6.93147180369123816490e-01 and LN2_LO =
 *       1.90821492927058770002e-10 (2 atanh(s) by its power series);
 *     exp_p(x), -700 <= x <= 0: k = floor(x 1.4426950408889634 + 0.5),
 *       r = (x - k LN2_HI) - k LN2_LO, p = 1/13! then p = p r + 1/j! for
 *       j = 12 .. 0; exp_p = p 2^k.
 *
 *   gesmc_gen_gnp: each pair w < v < n an edge with probability p.  Pairs
 *   are indexed q = v(v-1)/2 + w; [0, N) is cut into chunks of L pairs, L
 *   the smallest power of two >= 64 with L p >= 64 (at most 2^40).  Chunk
 *   j = [jL, min(jL+L, N)) walks a cursor c from jL: draw t takes (x0, x1)
 *   of Philox(ctr = (j_lo, j_hi, t, 3)), U = (((x0 << 32 | x1) >> 11) + 1)
 *   / 2^53, G = ln_p(U) / ln_p(1 - p); if G >= end - c the chunk ends, else
 *   pair c + floor(G) is an edge and c moves past it (geometric skipping,
 *   Batagelj and Brandes 2005; restarting at chunk starts is exact).  p >= 1:
 *   every pair; p <= 0 or n < 2: none.  Output (w << 32) | v in q order.
 *   *m = the edge count; d_out (device, cap keys) NULL only counts, and a
 *   count above cap is GESMC_E_RANGE (d_out untouched).
 *
 *   gesmc_gen_pld_degrees: W_i = floor(exp_p(-(gamma (ln_p(a+i) - ln_p(a))))
 *   2^43) for i = 0 .. b-a, C_i = W_0 + .. + W_i, T = C_{b-a}; vertex v's
 *   draw r takes R = x0 << 32 | x1 of Philox(ctr = (v, r, 0, 4)), u =
 *   floor(R T / 2^64), degree a + min{i : C_i > u}.  All vertices take draw
 *   0; while the sum is odd vertex 0 takes draws 1, 2, ... (at most 65535).
 *   d_deg (device, n words); *sum the even degree sum.  GESMC_E_INVAL for
 *   n = 0, a < 1, b < a, b - a >= 2^20, gamma < 0, (b/a)^gamma >= e^690, or
 *   no even sum (a = b odd with n odd).
 *
 *   gesmc_gen_havel_hakimi: vertices placed at positions 0 .. n-1 by (degree
 *   descending, id ascending), residuals starting at the degrees; while a
 *   residual is positive, the position v of largest residual d (smallest
 *   position among ties) is joined to the d other positions of positive
 *   residual with the largest (residual, position), v's residual becomes 0
 *   and theirs drop by one; edges (v, partner) by ascending partner
 *   position (Havel 1955, Hakimi 1962: this succeeds iff the sequence is
 *   graphical).  d_deg (device, n words); d_out (device, cap keys, (min <<
 *   32) | max); *m = sum / 2 (NULL d_out: only *m).  GESMC_E_NOT_GRAPHICAL
 *   for an odd sum, a degree >= n, or a sequence that runs out of partners
 *   (d_out then holds nothing defined); GESMC_E_RANGE for a degree above
 *   16000, m >= 2^32 or m > cap.  The steps run in one wavefront (the
 *   construction is sequential); the placement and edge writing are parallel.
 *
 *   gesmc_gen_relabel: pi = gesmc_permutation(n, seed ^ 0x9E3779B97F4A7C15,
 *   t = 0); vertex pi[r] becomes r; each of the m keys of d_edges (device,
 *   in place) is rewritten and made canonical.  1 <= n < 2^30;
 *   GESMC_E_RANGE for an id >= n (keys then partly rewritten).
 */
gesmc_status gesmc_gen_gnp(gesmc_ctx *ctx, void *stream, uint32_t n, double p, uint64_t seed, uint64_t *d_out,
                           uint64_t cap, uint64_t *m);
gesmc_status gesmc_gen_pld_degrees(gesmc_ctx *ctx, void *stream, uint32_t n, double gamma, uint32_t dmin,
                                   uint32_t dmax, uint64_t seed, uint32_t *d_deg, uint64_t *sum);
gesmc_status gesmc_gen_havel_hakimi(gesmc_ctx *ctx, void *stream, uint32_t n, const uint32_t *d_deg,
                                    uint64_t *d_out, uint64_t cap, uint64_t *m);
gesmc_status gesmc_gen_relabel(gesmc_ctx *ctx, void *stream, uint64_t *d_edges, uint64_t m, uint32_t n,
                               uint64_t seed);

/* Permutation keys K_i (see above) for i < m, to d_keys (device, m words). */
gesmc_status gesmc_perm_keys(gesmc_ctx *ctx, void *stream, uint64_t m, uint64_t seed, uint32_t t, uint64_t *d_keys);

/* The permutation pi of superstep t (Def. 3.2): d_pi[r] (device, m words) is
 * the edge index of rank r in (K_i, i) order. */
gesmc_status gesmc_permutation(gesmc_ctx *ctx, void *stream, uint64_t m, uint64_t seed, uint32_t t, uint32_t *d_pi);

/*
 * Serving: a request loop with continuous batching.  A worker thread owns the
 * context; every iteration it admits queued requests in arrival order while
 * their device footprint fits the HBM budget and the resident-graph limit,
 * runs one superstep of every resident graph together (the batched form,
 * each graph at its own superstep), and hands back every graph that has
 * finished its r supersteps.  Requests that arrive while others run join at
 * the next iteration; a graph's records stay resident on the device between
 * its supersteps.  Every result equals gesmc_run on that graph alone.
 * While a server exists, its context must not be used by other calls.
 */
typedef struct gesmc_server gesmc_server;

typedef struct gesmc_server_cfg {
    uint64_t hbm_budget_bytes; /* device memory for resident graphs (0: 16 GiB); about 136 bytes per
                                  edge, so at most budget / 136 edges are resident at once; copy
                                  buffers beside it grow to the largest admission and completion
                                  (8 bytes per edge each, three of them)                              */
    uint32_t max_graphs;       /* resident graphs at most (0: 4096)                                   */
    uint32_t max_queue;        /* queued requests at most; submit then returns GESMC_E_AGAIN (0: 2^16) */
} gesmc_server_cfg;

typedef struct gesmc_request {
    const uint64_t *edges; /* host memory, m keys as for gesmc_run; copied by gesmc_submit */
    uint64_t m;
    uint32_t n;
    uint32_t t0;
    uint32_t r;
    uint32_t pl;
    uint64_t seed;
} gesmc_request;

typedef struct gesmc_result {
    gesmc_status status; /* GESMC_OK, an input error, GESMC_E_CANCELED or GESMC_E_INTERNAL      */
    uint64_t m;
    uint64_t *edges;     /* host memory owned by the caller after poll / wait: m keys in position
                            order (NULL unless status is GESMC_OK); release with gesmc_result_free */
    gesmc_stats stats;   /* rounds_* are those of the shared supersteps                          */
    double t_submit, t_admit, t_done; /* seconds on the server's steady clock                      */
} gesmc_result;

typedef struct gesmc_server_info {
    uint64_t submitted, completed, iterations, attempts, legal;
    uint64_t resident_edges;
    uint32_t queued, resident;
    double busy_s; /* wall time of the worker's iterations             */
    double now_s;  /* the server clock                                  */
    double copy_s; /* of busy_s: host copies of edges in and results out */
    double wait_s; /* of busy_s: waiting for the device                  */
} gesmc_server_info;

/* Starts the worker (cfg nullable: defaults).  Fails with GESMC_E_NOMEM if
 * the budget cannot be allocated.  *out receives the server. */
gesmc_status gesmc_server_create(gesmc_ctx *ctx, const gesmc_server_cfg *cfg, gesmc_server **out);
/* Stops the worker; requests still queued or resident are dropped.  Threads
 * blocked in gesmc_wait on this server return first, with a result whose
 * status is GESMC_E_CANCELED (unless their request had finished); destroy
 * waits for them to leave before it frees anything.  No other call on the
 * server may start once destroy has been entered. */
void gesmc_server_destroy(gesmc_server *srv);
/* Queues a request (edges copied; thread-safe).  GESMC_E_AGAIN if the queue is
 * full, GESMC_E_RANGE if the graph can never fit the budget, GESMC_E_INVAL for
 * bad arguments.  Input errors of the graph itself are reported in its result. */
gesmc_status gesmc_submit(gesmc_server *srv, const gesmc_request *req, uint64_t *ticket);
/* Non-blocking: fills *out and forgets the ticket if the request is done,
 * else returns GESMC_E_AGAIN.  GESMC_E_INVAL for an unknown ticket.  A ticket
 * is taken by one thread: two threads must not poll or wait on the same one. */
gesmc_status gesmc_poll(gesmc_server *srv, uint64_t ticket, gesmc_result *out);
/* As gesmc_poll, but blocks until the request is done. */
gesmc_status gesmc_wait(gesmc_server *srv, uint64_t ticket, gesmc_result *out);
/* Cancels a queued or resident request; its result then has GESMC_E_CANCELED. */
gesmc_status gesmc_cancel(gesmc_server *srv, uint64_t ticket);
void gesmc_result_free(gesmc_result *res);
gesmc_status gesmc_server_info_get(gesmc_server *srv, gesmc_server_info *out);

/*
 * ParES (Alg. 2, Sec. 4): the Edge Switching Markov Chain of Def. 2.1, run
 * exactly in supersteps without source dependencies.  r edge switches with
 * switch counters k0 .. k0+r-1 are applied in sequence to the m edges at d_in
 * (device memory, uint64 keys as for gesmc_run); the result, in position
 * order, goes to d_out (device, m words, may equal d_in).  Switch k draws,
 * with (x0, x1, x2, x3) = Philox4x32-10 at counter (k_lo, k_hi, 0, 2) and key
 * (seed_lo, seed_hi):
 *   i = floor(((x0 << 32) | x1) * m / 2^64),
 *   j = j' + [j' >= i] with j' = floor(((x2 << 32) | x3) * (m - 1) / 2^64),
 *   g = x1 & 1,
 * so i != j (as Alg. 2 samples them) and the triple is uniform up to a bias
 * below m / 2^64; the switch is rejected on a loop or a present target, else
 * E[i] <- canon(e3), E[j] <- canon(e4).  run_es(r1) then run_es(r2, k0 + r1)
 * equals run_es(r1 + r2).  d_outcome (device, nullable, r bytes): the outcome
 * code of switch k0 + q at d_outcome[q] (1 accepted, 2 loop, 3 target
 * present).  stats (host, nullable).  m < 2 copies the canonicalised input
 * (no two distinct indices exist).  Errors as for gesmc_run, d_out untouched.
 * Runs on one workgroup of the device per call: ES-MC has supersteps of
 * about sqrt(m) switches (Sec. 3), a latency-bound chain.
 */
typedef struct gesmc_es_stats {
    uint64_t attempts, legal, rej_loop, rej_exists;
    uint64_t supersteps;  /* ParES supersteps: runs of switches without a shared edge index, at
                             most 1024 switches each                                          */
    uint64_t rounds_sum;  /* decision rounds over all supersteps                              */
    uint32_t rounds_max;  /* most rounds in one superstep                                     */
    uint32_t epochs;      /* launches (the edge set is rebuilt between them)                  */
    double ms_device;
} gesmc_es_stats;

gesmc_status gesmc_run_es(gesmc_ctx *ctx, void *stream, const uint64_t *d_in, uint64_t *d_out, uint64_t m, uint32_t n,
                          uint64_t seed, uint64_t k0, uint64_t r, uint32_t flags, uint8_t *d_outcome,
                          gesmc_es_stats *stats);

/* The draws (i, j, g) of ES-MC switches k0 .. k0+count-1 on m edges (2 <= m
 * < 2^30), defined as for gesmc_run_es: d_i, d_j (device, count uint64 each),
 * d_g (device, count bytes).  Parity hook for the random choices of ParES. */
gesmc_status gesmc_es_draws(gesmc_ctx *ctx, void *stream, uint64_t m, uint64_t seed, uint64_t k0, uint64_t count,
                            uint64_t *d_i, uint64_t *d_j, uint8_t *d_g);

/*
 * Mixing diagnostic (Sec. 6.1): the autocorrelation analysis of a chain's
 * edge series, aggregated on the device while the chain runs.  The chain
 * runs K supersteps from the m edges at d_in (device, keys as for gesmc_run,
 * left unchanged): chain 0 = G-ES-MC (superstep t is gesmc_run's superstep t
 * with this seed and pl), chain 1 = ES-MC (superstep t is floor(m/2) edge
 * switches of gesmc_run_es, counters t*floor(m/2) ..).  For each thinning
 * value k = thin[q] the k-thinned series samples the states X_0, X_k, ...,
 * X_{Nk}, N = floor(K / k); every edge present in some sample is tracked
 * with the counts n_ab of its transitions a -> b between consecutive
 * samples; G^2 = 2 sum n_ab ln(n_ab N / (n_a. n_.b)) (float64) and the
 * Bayesian information criterion (the Markov model has one parameter more)
 * deem it not independent iff G^2 > ln N.  out[q] (host, nthin records)
 * receives k, N, the edges tracked, those not independent and the counts
 * summed over tracked edges (exact integers).  ms_chain (host, nullable):
 * wall time of the chain and its sampling.  Limits: 2 <= n <= 2^14 (dense
 * pair counters: 12 bytes per vertex pair and thinning value), 1 <= nthin
 * <= 16, every k >= 1.  Device memory is allocated for the call and freed.
 */
typedef struct gesmc_mixing_result {
    uint32_t k;            /* thinning value                                */
    uint32_t transitions;  /* N = floor(K / k)                              */
    uint64_t tracked;      /* edges present in at least one sample          */
    uint64_t non_independent;
    uint64_t n00, n01, n10, n11; /* transitions summed over tracked edges   */
} gesmc_mixing_result;

#define GESMC_CHAIN_GLOBAL 0u
#define GESMC_CHAIN_ES 1u

gesmc_status gesmc_mixing(gesmc_ctx *ctx, void *stream, const uint64_t *d_in, uint64_t m, uint32_t n, uint64_t seed,
                          uint32_t chain, uint32_t pl, uint32_t K, const uint32_t *thin, uint32_t nthin,
                          gesmc_mixing_result *out, double *ms_chain);

/* Result of an autotuning run: the options chosen and the measured times. */
typedef struct gesmc_tuning {
    uint32_t bucket_avg;  /* GESMC_OPT_BUCKET_AVG chosen          */
    uint32_t level1_bits; /* GESMC_OPT_LEVEL1_BITS chosen         */
    uint32_t fuse_emit;   /* GESMC_OPT_FUSE_EMIT chosen           */
    uint32_t candidates;  /* settings timed                       */
    double best_ms;       /* device time of the chosen setting    */
    double default_ms;    /* device time of the default setting   */
} gesmc_tuning;

/*
 * Autotuner: times `supersteps` global switches (from superstep 0 with the
 * given seed, results discarded) of the plain form on d_in (device, m keys,
 * ids < n) under each candidate setting of the options above, and leaves the
 * fastest set on the context.  Results never depend on the options, so a
 * tuned context computes exactly what an untuned one does.  out (host,
 * nullable) receives the choice.  Needs GESMC_OPT_STRATEGY 0.  Allocates a
 * scratch output of m words for the duration of the call.
 */
gesmc_status gesmc_autotune(gesmc_ctx *ctx, void *stream, const uint64_t *d_in, uint64_t m, uint32_t n,
                            uint64_t seed, uint32_t supersteps, gesmc_tuning *out);

/* The same for batches: candidates are timed on gesmc_run_batch over the
 * given graphs (arguments as for gesmc_run_batch; every graph runs
 * `supersteps` switches from t0 = 0). */
gesmc_status gesmc_autotune_batch(gesmc_ctx *ctx, void *stream, uint32_t G, const uint64_t *d_in,
                                  const uint64_t *offsets, const uint32_t *n, const uint64_t *seed,
                                  uint32_t supersteps, gesmc_tuning *out);

/*
 * Tuning cache.  With GESMC_OPT_TUNE_CACHE on (the default), the autotuner
 * keeps each choice per device (architecture and PCI address) and shape
 * class (plain or batch; log2 of the edge count, of the largest vertex count
 * and of the graph count), shared by every context of the process, and a
 * later autotune of the same device and class sets the kept choice without
 * timing anything (out->candidates = 0).  save writes the cache as a JSON
 * array, one entry per line; load merges such a file into the cache
 * (GESMC_E_INVAL if it cannot be read or is not in that form, cache
 * unchanged).  Thread-safe; no device is needed.
 */
gesmc_status gesmc_tune_cache_save(const char *path);
gesmc_status gesmc_tune_cache_load(const char *path);
void gesmc_tune_cache_clear(void);
uint32_t gesmc_tune_cache_size(void);

/* Tuning knobs (values are validated; results never depend on them, except
 * that GESMC_OPT_ROUND_LIMIT can make a call fail). */
#define GESMC_OPT_BUCKET_AVG 1  /* largest mean records per sort bucket (64 .. 1152, default 1152)  */
#define GESMC_OPT_SORT_CAP 2    /* records sorted in LDS per bucket (64 .. 1536, default 1536)     */
#define GESMC_OPT_FAST_ROUNDS 3 /* multi-workgroup rounds before the 1-workgroup finisher (0 .. 64);
                                   unset: 2, or 128 for a plain call after one on this context whose
                                   supersteps needed more than 16 decision rounds (hub edges)      */
#define GESMC_OPT_PROFILE 4     /* 1: time every kernel launch with HIP events                      */
#define GESMC_OPT_STRATEGY 5    /* dependency resolution: 0 = tuples sorted by edge key per hash
                                   partition in LDS (default); 1 = one open-addressing table in HBM
                                   rebuilt every superstep with device-scope atomics               */
#define GESMC_OPT_PERSIST 6     /* workgroups of the tile/bucket kernels: resident count x value;
                                   0 = one workgroup per tile or bucket (default 0)                */
#define GESMC_OPT_LEVEL1_BITS 8  /* digit bits of the first radix level (1 .. 10); 0 = half of the
                                    bucket bits, rounded up (default)                              */
#define GESMC_OPT_FUSE_EMIT 9      /* 1: the first tuple partition pass computes the switches' tuples from
                                      their pair records, and its count kernel also writes each
                                      switch's status and records (default); 0: a separate emit
                                      kernel, and the tuples are written out first                   */
#define GESMC_OPT_GRAPH 10         /* 1: gesmc_run_batch captures its device work into a hipGraph on the
                                      second call of the same shape (pointers, sizes, offsets, r, pl,
                                      options) and replays it for later calls of that shape -- seeds,
                                      t0 and n may change; needs a non-NULL stream (default 0)         */
#define GESMC_OPT_SMALL_GRAPHS 11  /* 1: graphs of at most 4096 edges, or 6144 with every vertex id below
                                      2^16, run all their supersteps in one workgroup's LDS -- in
                                      gesmc_run_batch one launch per size class (up to 1024 edges on
                                      256 threads, up to 4096 on 1024, up to 6144 with 32-bit keys on
                                      1024), in gesmc_run two launches per 32 supersteps (their
                                      permutations, then the chain) when steps is NULL; 0: every
                                      graph takes the multi-kernel supersteps (default 1)            */
#define GESMC_OPT_PACK_TUPLES 12   /* 1: dependency tuples travel as one 8-byte word (a bijective hash of
                                      the edge key on 2 x the vertex id bits, minus the bits the first
                                      partition pass implies, over a coded tag) wherever those bits and
                                      the tag fit 64 -- in a batch too large for batch-wide switch ids,
                                      with tags local to each graph; 0: always (tag u32, key hash u64);
                                      2: as 1, with graph-local tags in every batch (default 1)        */
#define GESMC_OPT_PROFILE_ONLY 7 /* kernel id whose launches are timed while profiling; -1 = every
                                    kernel (default).  Events between launches cost time, so timing
                                    one kernel disturbs the rest least                              */
#define GESMC_OPT_ROUND_LIMIT 13  /* decision rounds a superstep may take (Alg. 1's loop, counted as in
                                     gesmc_step_stats.rounds) before the call fails with GESMC_E_ROUNDS
                                     and d_out untouched; 0 = no limit (default).  A debugging cap for
                                     the multi-kernel supersteps of GESMC_OPT_STRATEGY 0 (plain and
                                     batched); the LDS small-graph kernels do not count against it,
                                     and a context serving a gesmc_server must keep it 0.  The only
                                     option that can change a call's outcome                        */
#define GESMC_OPT_UNPERMUTE_BUCKETS 14 /* 1 (default): from 2^20 edges on, the final write-back to input
                                          order first gathers the records into buckets of consecutive
                                          indices, then writes each bucket's window of d_out XCD by XCD;
                                          0: one scattered write per edge over all of d_out          */
#define GESMC_OPT_TUNE_CACHE 15  /* 1 (default): the autotuner reuses and keeps its choices per device and
                                    shape class (see gesmc_tune_cache_save); 0: it always times       */
gesmc_status gesmc_set_option(gesmc_ctx *ctx, int option, int64_t value);

/*
 * Caller-supplied device memory (for instance PyTorch's caching allocator).
 * After the call the context takes every device buffer it allocates from
 * alloc(bytes, user), which must return memory of the context's device,
 * aligned to 256 bytes, or NULL (the call that needed it then fails with
 * GESMC_E_NOMEM and leaves its output untouched; the context stays usable).
 * Each buffer goes back to the allocator that made it: free_fn(ptr, user) of
 * the pair in force when it was allocated, called only after the device has
 * finished all queued work (hipMalloc buffers from before stay hipMalloc
 * buffers).  Both NULL: back to hipMalloc.  The functions run on the thread
 * of the library call that allocates (a context's buffers grow on demand)
 * and must not call into the library.  GESMC_E_INVAL for one function given
 * without the other, or while a gesmc_server uses the context.  The small
 * fixed area of gesmc_create and gesmc_run_noalloc's array are never taken
 * from it.
 */
typedef void *(*gesmc_alloc_fn)(size_t bytes, void *user);
typedef void (*gesmc_free_fn)(void *ptr, void *user);
gesmc_status gesmc_set_allocator(gesmc_ctx *ctx, gesmc_alloc_fn alloc, gesmc_free_fn free_fn, void *user);

/* Kernel timing collected while GESMC_OPT_PROFILE is on.  Kernel ids run from 0
 * to gesmc_kernel_count() - 1; gesmc_kernel_name gives the name.  *ms is the
 * summed device duration of all launches of that kernel, *launches their
 * count, *items the work items they covered (edges, switches or slots, per
 * kernel). */
int gesmc_kernel_count(void);
const char *gesmc_kernel_name(int kernel_id);
gesmc_status gesmc_profile_get(gesmc_ctx *ctx, int kernel_id, double *ms, uint64_t *launches, uint64_t *items);
gesmc_status gesmc_profile_reset(gesmc_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* GESMC_H */

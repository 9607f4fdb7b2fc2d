// Serving runtime (gesmc_server_*): a worker thread with continuous batching
// over the batched superstep.  Included at the end of gesmc.hip (it drives
// the context's buffers and the superstep pipeline directly).
//
// Layout between iterations: buffer 0 of the context holds the records of
// the resident graphs in rank order (segments as in a batch, BatchGraph);
// every graph keeps its index labels (local index + a fixed base) and is
// re-shifted to a new vertex base whenever the layout is rebuilt.
#pragma once

#include <chrono>
#include <condition_variable>
#include <memory>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "copy_pool.h"

namespace {

constexpr uint64_t kServeBytesPerEdge = 136;  // context buffers per resident record (see ensure_capacity)
// Supersteps per iteration (one host round trip): never beyond the next
// completion; at most kServeBurstIdle while no request waits, so arrivals
// are admitted within that many supersteps, and up to kServeBurstMax while
// the queue is blocked (nothing can be admitted before a completion).
constexpr uint32_t kServeBurstIdle = 4, kServeBurstMax = 64;

struct ServeReq {
    uint64_t ticket = 0;
    std::vector<uint64_t> edges;
    uint64_t m = 0;
    uint32_t n = 0, t0 = 0, r = 0, pl = 0;
    uint64_t seed = 0;
    uint32_t done = 0;  // supersteps queued (the worker's view, ahead of the device)
    uint32_t goff = 0;  // index label base, fixed at admission
    uint32_t poff = 0, vbase = 0;  // segment and vertex base in the current layout
    bool cancel = false, finished = false;
    uint32_t flights = 0;                   // queued iterations holding the graph (worker only)
    bool leaving = false;                   // out of the resident set; finished when flights == 0
    gesmc_status final_status = GESMC_OK;   // what it finishes with
    gesmc_status status = GESMC_OK;
    gesmc_stats stats{};
    uint64_t *result = nullptr;
    double t_submit = 0, t_admit = -1, t_done = 0;
};

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// One queued iteration of the worker: its rank order, result offsets, and
// the pinned host buffers its results and counts come back to.
struct ServeFlight {
    std::vector<ServeReq *> ranks;
    std::vector<uint64_t> rb;  // result offset (words) per rank, ~0: not finishing
    uint32_t nsurv = 0, k = 0;
    uint32_t tuple_bytes = 0;  // tuple size of the iteration's supersteps
    bool live = false;
    hipEvent_t done = nullptr;  // on the compute stream, after the iteration's last copy
    uint64_t *h_res = nullptr;  // results of the finishing graphs
    uint64_t res_cap = 0;       // words
    uint64_t *d_res = nullptr;  // the same on the device (filled by the compute stream)
    uint64_t d_res_cap = 0;     // words
    hipEvent_t ext = nullptr;     // on the compute stream, after the results are extracted
    hipEvent_t res_ev = nullptr;  // on the download stream, after the results' copy
    bool res_pending = false;
    unsigned long long *h_gacc = nullptr;  // 4 per rank (max_graphs)
    uint32_t *h_gerr = nullptr;            // per rank
    StepCounters *h_ctr = nullptr;         // per superstep (kServeBurstMax)
    uint32_t *h_err = nullptr;             // error words
};

}  // namespace

struct gesmc_server {
    gesmc_ctx *c = nullptr;
    hipStream_t s = nullptr;
    uint64_t cap_edges = 0;
    uint32_t max_graphs = 0, max_queue = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<ServeReq *> queue;
    std::unordered_map<uint64_t, ServeReq *> reqs;
    std::vector<ServeReq *> resident;  // worker only: rank order of the layout in buffer 0
    bool stop = false;
    uint32_t waiters = 0;  // threads blocked in gesmc_wait (under mu); destroy waits for them to leave
    std::thread worker;
    std::chrono::steady_clock::time_point t0;
    uint64_t next_ticket = 1;
    // info (under mu)
    uint64_t submitted = 0, completed = 0, iterations = 0, attempts = 0, legal = 0, resident_edges = 0;
    uint32_t resident_count = 0;
    double busy_s = 0, copy_s = 0, wait_s = 0;  // under mu
    double w_copy = 0, w_wait = 0;              // the worker's, folded into the above under mu
    // worker-side staging
    std::vector<BatchGraph> h_gr;
    std::vector<uint2> h_mv;
    std::vector<uint64_t> h_stage_off;
    std::vector<uint32_t> h_stage_rank;
    uint64_t *h_pin = nullptr;  // pinned staging of admitted edges
    uint64_t pin_cap = 0;       // words
    uint64_t *d_stage = nullptr;  // device staging of admitted edges (the upload's target)
    uint64_t d_stage_cap = 0;     // words
    // Copies of edges and results run on streams of their own, so that they
    // overlap the supersteps of the neighbouring iteration.  Every wait below
    // is on an event recorded earlier in host order.
    hipStream_t up = nullptr, down = nullptr;
    hipEvent_t stage_ev = nullptr;  // on `up`, after the last upload from h_pin into d_stage
    bool stage_pending = false;
    hipEvent_t load_ev = nullptr;   // on the compute stream, after the last load from d_stage
    bool load_recorded = false;
    ServeFlight fl[2];          // two iterations in flight at most
    uint2 *d_mv = nullptr;
    uint64_t *d_stage_off = nullptr;
    uint32_t *d_stage_rank = nullptr;
    std::unique_ptr<gesmc::CopyPool> copier;  // worker only
    std::vector<gesmc::CopyPool::Seg> segs;
};

namespace {

void serve_finish_locked(gesmc_server *S, ServeReq *q, gesmc_status st) {
    if (st != GESMC_OK && q->result) {
        free(q->result);
        q->result = nullptr;
    }
    q->status = st;
    q->finished = true;
    q->t_done = seconds_since(S->t0);
    q->edges.clear();
    q->edges.shrink_to_fit();
    ++S->completed;
    S->cv_done.notify_all();
}

// Requests without switches (r = 0 or m < 2): validated and canonicalised on
// the host, with the checks and status precedence of gesmc_run.
gesmc_status serve_trivial(ServeReq *q) {
    bool loop = false, range = false;
    std::vector<uint64_t> canon(q->m);
    for (uint64_t i = 0; i < q->m; ++i) {
        const uint32_t a = (uint32_t)(q->edges[i] >> 32), b = (uint32_t)q->edges[i];
        loop |= a == b;
        range |= a >= q->n || b >= q->n || a == 0xFFFFFFFFu || b == 0xFFFFFFFFu;
        canon[i] = a < b ? ((uint64_t)a << 32) | b : ((uint64_t)b << 32) | a;
    }
    std::vector<uint64_t> sorted = canon;
    std::sort(sorted.begin(), sorted.end());
    const bool dup = std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end();
    if (loop || dup) return GESMC_E_NOT_SIMPLE;
    if (range) return GESMC_E_RANGE;
    q->result = (uint64_t *)malloc(std::max<uint64_t>(q->m, 1) * 8);
    if (!q->result) return GESMC_E_NOMEM;
    memcpy(q->result, canon.data(), q->m * 8);
    return GESMC_OK;
}

gesmc_status serve_map_gerr(uint32_t e) {
    if (e & (ERR_LOOP | ERR_DUP)) return GESMC_E_NOT_SIMPLE;
    if (e & ERR_RANGE) return GESMC_E_RANGE;
    return GESMC_E_INTERNAL;
}

// Grows the pinned staging of admitted edges to at least `words` words
// (after the previous upload from it has left).
gesmc_status serve_stage(gesmc_server *S, uint64_t words) {
    if (S->stage_pending) {
        GESMC_TRY(check_hip(hipEventSynchronize(S->stage_ev), "hipEventSynchronize"));
        S->stage_pending = false;
    }
    if (words <= S->pin_cap) return GESMC_OK;
    if (S->h_pin) (void)hipHostFree(S->h_pin);
    S->h_pin = nullptr;
    S->pin_cap = 0;
    const uint64_t cap = std::max<uint64_t>(words + words / 4, 8ull << 20);
    if (hipHostMalloc((void **)&S->h_pin, cap * 8, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        S->h_pin = nullptr;
        set_error("hipHostMalloc of the serving staging buffer failed");
        return GESMC_E_NOMEM;
    }
    S->pin_cap = cap;
    return GESMC_OK;
}

// Grows the device staging of admitted edges to at least `words` words,
// once no upload into it and no load from it is queued any more.
gesmc_status serve_dev_stage(gesmc_server *S, uint64_t words) {
    if (words <= S->d_stage_cap) return GESMC_OK;
    if (S->d_stage) {
        if (S->stage_pending) GESMC_TRY(check_hip(hipEventSynchronize(S->stage_ev), "hipEventSynchronize"));
        if (S->load_recorded) GESMC_TRY(check_hip(hipEventSynchronize(S->load_ev), "hipEventSynchronize"));
        dev_free(S->c, S->d_stage);
    }
    S->d_stage = nullptr;
    S->d_stage_cap = 0;
    const uint64_t cap = std::max(words, std::min<uint64_t>(std::max<uint64_t>(words + words / 4, 1ull << 20),
                                                            S->cap_edges + 64));
    GESMC_TRY(dev_alloc(S->c, (void **)&S->d_stage, cap * 8));
    S->d_stage_cap = cap;
    return GESMC_OK;
}

// Grows a flight's device result buffer (the flight is not in use: its last
// download was waited for when it completed).
gesmc_status serve_flight_dres(gesmc_server *S, ServeFlight &F, uint64_t words) {
    if (words <= F.d_res_cap) return GESMC_OK;
    if (F.d_res) dev_free(S->c, F.d_res);
    F.d_res = nullptr;
    F.d_res_cap = 0;
    const uint64_t cap = std::max(words, std::min<uint64_t>(std::max<uint64_t>(words + words / 4, 1ull << 20),
                                                            S->cap_edges + 64));
    GESMC_TRY(dev_alloc(S->c, (void **)&F.d_res, cap * 8));
    F.d_res_cap = cap;
    return GESMC_OK;
}

// Grows a flight's pinned result buffer (the flight is not in use).
gesmc_status serve_flight_res(ServeFlight &F, uint64_t words) {
    if (words <= F.res_cap) return GESMC_OK;
    if (F.h_res) (void)hipHostFree(F.h_res);
    F.h_res = nullptr;
    F.res_cap = 0;
    const uint64_t cap = std::max<uint64_t>(words + words / 4, 8ull << 20);
    if (hipHostMalloc((void **)&F.h_res, cap * 8, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        F.h_res = nullptr;
        set_error("hipHostMalloc of a serving result buffer failed");
        return GESMC_E_NOMEM;
    }
    F.res_cap = cap;
    return GESMC_OK;
}

// Queues one iteration into flight F: new layout (survivors `next` + the
// admitted), k supersteps of every resident graph (each at its own superstep
// t0 + done + step), the results of the graphs that finish, the outcome
// counts; nothing waits for the device.  The requests' host state advances
// as if the iteration had run (done += k); its outcome is read in
// serve_complete.
gesmc_status serve_enqueue(gesmc_server *S, ServeFlight &F, const std::vector<ServeReq *> &next,
                           const std::vector<ServeReq *> &admit, bool relayout, uint32_t k) {
    gesmc_ctx *c = S->c;
    hipStream_t s = S->s;
    const uint32_t nsurv = (uint32_t)next.size();
    F.ranks = next;
    F.ranks.insert(F.ranks.end(), admit.begin(), admit.end());
    F.nsurv = nsurv;
    F.k = k;
    const std::vector<ServeReq *> &ranks = F.ranks;
    const uint32_t G = (uint32_t)ranks.size();
    S->h_gr.assign(G, BatchGraph{});
    S->h_mv.assign(G, make_uint2(0xFFFFFFFFu, 0));
    uint64_t poff = 0, vbase = 0, bbase = 0, stage = 0, nmax = 0, mmax = 0;
    uint32_t pl_any = 0;
    S->h_stage_off.clear();
    S->h_stage_rank.clear();
    for (uint32_t q = 0; q < G; ++q) {
        ServeReq *R = ranks[q];
        BatchGraph &b = S->h_gr[q];
        if (q >= nsurv) {  // admitted now: loaded from the staging buffer, labels = staging positions
            R->goff = (uint32_t)stage;
            S->h_stage_off.push_back(stage);
            S->h_stage_rank.push_back(q);
            stage += R->m;
        } else if (relayout) {
            S->h_mv[q] = make_uint2(R->poff, R->vbase);
        }
        b.poff = (uint32_t)poff;
        b.mpad = (uint32_t)(R->m + (R->m & 1));
        b.goff = R->goff;
        b.vbase = (uint32_t)vbase;
        b.k0 = (uint32_t)R->seed;
        b.k1 = (uint32_t)(R->seed >> 32);
        b.t0 = R->t0 + R->done;
        b.nb = (uint32_t)std::max<uint64_t>(1, ceil_div(b.mpad, c->bucket_avg));
        b.bbase = (uint32_t)bbase;
        b.m = (uint32_t)R->m;
        b.n = R->n;
        b.pl = R->pl;
        pl_any |= R->pl;
        R->poff = b.poff;
        R->vbase = b.vbase;
        poff += b.mpad;
        vbase += R->n;
        nmax = std::max<uint64_t>(nmax, R->n);
        mmax = std::max<uint64_t>(mmax, b.mpad);
        bbase += b.nb;
    }
    S->h_stage_off.push_back(stage);
    const uint32_t npos = (uint32_t)poff;
    // graphs that finish in this iteration, and their result offsets
    F.rb.assign(G, ~0ull);
    uint64_t rpos = 0;
    for (uint32_t q = 0; q < G; ++q) {
        if (ranks[q]->done + k == ranks[q]->r) {
            F.rb[q] = rpos;
            rpos += ranks[q]->m;
        }
    }
    // position chunks: every rank (pg) and the staying ranks (relayout) if the
    // layout is rebuilt, then the finishing ranks with their result offsets
    c->h_chunks.clear();
    if (relayout)
        for (uint32_t q = 0; q < G; ++q) add_chunks(c->h_chunks, q, S->h_gr[q].poff, S->h_gr[q].mpad);
    const uint32_t n_fill = (uint32_t)c->h_chunks.size();
    if (relayout)
        for (uint32_t q = 0; q < nsurv; ++q) add_chunks(c->h_chunks, q, S->h_gr[q].poff, S->h_gr[q].mpad);
    const uint32_t n_move = (uint32_t)c->h_chunks.size() - n_fill;
    for (uint32_t q = 0; q < G; ++q)
        if (F.rb[q] != ~0ull) add_chunks(c->h_chunks, q, S->h_gr[q].poff, S->h_gr[q].mpad, (uint32_t)F.rb[q]);
    const uint32_t n_out = (uint32_t)c->h_chunks.size() - n_fill - n_move;
    if (bbase > (1ull << kMaxFineBits) || npos > c->cap_pos || G > S->max_graphs || k > kServeBurstMax) {
        set_error("serving layout exceeds the context's capacity");
        return GESMC_E_INTERNAL;
    }
    {  // pinned buffers sized before any copy is queued (growing them is part of the copies' cost)
        const auto a0 = std::chrono::steady_clock::now();
        GESMC_TRY(serve_stage(S, stage));
        GESMC_TRY(serve_flight_res(F, rpos));
        GESMC_TRY(serve_dev_stage(S, stage));
        GESMC_TRY(serve_flight_dres(S, F, rpos));
        S->w_copy += seconds_since(a0);
    }
    // small uploads through the context's pinned arena (records, chunks, moves, staging map)
    const uint32_t nadm = (uint32_t)admit.size();
    GESMC_TRY(ensure_chunks(c));
    GESMC_TRY(up_begin(c,
                       G * (sizeof(BatchGraph) + sizeof(uint2)) + (uint64_t)c->h_chunks.size() * sizeof(uint4) +
                           (nadm + 1) * 8ull + nadm * 4ull,
                       5));
    GESMC_TRY(up_copy(c, s, c->gr, S->h_gr.data(), G * sizeof(BatchGraph)));
    GESMC_TRY(up_copy(c, s, c->chunks, c->h_chunks.data(), (uint64_t)c->h_chunks.size() * sizeof(uint4)));
    GESMC_TRY(ensure_counters(c, k));
    GESMC_TRY(launch(c, s, KID_MISC, 0, k_zero_words, dim3(4), dim3(256), 0, c->err, (uint64_t)64));
    GESMC_TRY(launch(c, s, KID_MISC, 0, k_zero_words, dim3(1), dim3(256), 0, (uint32_t *)c->ctr,
                     (uint64_t)k * (sizeof(StepCounters) / 4)));
    GESMC_TRY(launch(c, s, KID_MISC, 0, k_zero_words, dim3(16), dim3(256), 0, c->gerr, (uint64_t)G));
    GESMC_TRY(launch(c, s, KID_MISC, 0, k_zero_words, dim3(16), dim3(256), 0, (uint32_t *)c->gacc,
                     (uint64_t)G * 8));
    if (relayout) {
        if (n_fill)
            GESMC_TRY(launch(c, s, KID_MISC, 0, k_fill_pg, dim3(n_fill), dim3(kBlock), 0, (const uint4 *)c->chunks,
                             c->pg));
        if (n_move) {
            GESMC_TRY(up_copy(c, s, S->d_mv, S->h_mv.data(), G * sizeof(uint2)));
            GESMC_TRY(launch(c, s, KID_MISC, 0, k_relayout, dim3(n_move), dim3(kBlock), 0,
                             (const uint4 *)c->chunks + n_fill, (const BatchGraph *)c->gr, (const uint2 *)S->d_mv,
                             (const uint32_t *)c->idx[0], (const unsigned long long *)c->key[0], c->idx[1],
                             c->key[1]));
        }
        if (!admit.empty()) {
            // raw edges of the admitted requests -> pinned staging -> one copy to the
            // device staging (on the upload stream, once the previous load from it
            // is done), then load on the compute stream after that copy
            const unsigned long long *stg = (const unsigned long long *)S->d_stage;
            const auto c0 = std::chrono::steady_clock::now();
            S->segs.clear();
            for (size_t j = 0; j < admit.size(); ++j)
                if (admit[j]->m) S->segs.push_back({S->h_pin + S->h_stage_off[j], admit[j]->edges.data(), admit[j]->m * 8});
            S->copier->copy(S->segs);
            S->w_copy += seconds_since(c0);
            if (stage) {
                if (S->load_recorded)
                    GESMC_TRY(check_hip(hipStreamWaitEvent(S->up, S->load_ev, 0), "hipStreamWaitEvent"));
                GESMC_TRY(check_hip(hipMemcpyAsync(S->d_stage, S->h_pin, stage * 8, hipMemcpyHostToDevice, S->up),
                                    "hipMemcpyAsync"));
                GESMC_TRY(check_hip(hipEventRecord(S->stage_ev, S->up), "hipEventRecord"));
                S->stage_pending = true;
                GESMC_TRY(check_hip(hipStreamWaitEvent(s, S->stage_ev, 0), "hipStreamWaitEvent"));
            }
            GESMC_TRY(up_copy(c, s, S->d_stage_off, S->h_stage_off.data(), (nadm + 1) * 8ull));
            GESMC_TRY(up_copy(c, s, S->d_stage_rank, S->h_stage_rank.data(), nadm * 4ull));
            if (stage > 0)
                GESMC_TRY(launch(c, s, KID_LOAD, stage, k_load_batch, dim3(grid_stride_blocks(c, stage)),
                                 dim3(kBlock), 0, stg, (uint32_t)stage,
                                 (const uint64_t *)S->d_stage_off, nadm, (const uint32_t *)S->d_stage_rank,
                                 (const BatchGraph *)c->gr, c->idx[1], c->key[1], c->err + 8, c->err + 9, c->gerr));
            if (stage) {
                GESMC_TRY(check_hip(hipEventRecord(S->load_ev, s), "hipEventRecord"));
                S->load_recorded = true;
            }
        }
        std::swap(c->idx[0], c->idx[1]);
        std::swap(c->key[0], c->key[1]);
        ++g_alloc_epoch;  // buffer roles moved: no captured graph may be replayed
    }
    GESMC_TRY(up_end(c, s));
    const Plan p = batch_plan(c, npos, bbase);
    for (uint32_t st = 0; st < k; ++st) {
        BatchStep bs{c->gr, G, st, c->pg, c->bk, c->gacc, GraphErr{c->gr, G, c->gerr}, vbase, nmax, mmax};
        c->ctr_step = c->ctr + st;
        GESMC_TRY(superstep_partitioned(c, s, p, 0u, 0u, 0u, pl_any, 0u, &bs));
    }
    F.tuple_bytes = c->tuple_bytes;
    // results of the graphs finishing now (discarded on the host if flagged),
    // downloaded on the download stream while the next iteration computes
    if (n_out) {
        GESMC_TRY(launch(c, s, KID_UNPERMUTE, rpos, k_extract, dim3(n_out), dim3(kBlock), 0,
                         (const uint4 *)c->chunks + n_fill + n_move, (const uint32_t *)c->idx[0],
                         (const unsigned long long *)c->key[0], (const BatchGraph *)c->gr,
                         (unsigned long long *)F.d_res));
        GESMC_TRY(check_hip(hipEventRecord(F.ext, s), "hipEventRecord"));
        GESMC_TRY(check_hip(hipStreamWaitEvent(S->down, F.ext, 0), "hipStreamWaitEvent"));
        GESMC_TRY(check_hip(hipMemcpyAsync(F.h_res, F.d_res, rpos * 8, hipMemcpyDeviceToHost, S->down),
                            "hipMemcpyAsync"));
        GESMC_TRY(check_hip(hipEventRecord(F.res_ev, S->down), "hipEventRecord"));
        F.res_pending = true;
    }
    GESMC_TRY(check_hip(hipMemcpyAsync(F.h_err, c->err, 32, hipMemcpyDeviceToHost, s), "hipMemcpyAsync"));
    GESMC_TRY(check_hip(hipMemcpyAsync(F.h_ctr, c->ctr, k * sizeof(StepCounters), hipMemcpyDeviceToHost, s),
                        "hipMemcpyAsync"));
    GESMC_TRY(check_hip(hipMemcpyAsync(F.h_gacc, c->gacc, G * 32ull, hipMemcpyDeviceToHost, s), "hipMemcpyAsync"));
    GESMC_TRY(check_hip(hipMemcpyAsync(F.h_gerr, c->gerr, G * 4ull, hipMemcpyDeviceToHost, s), "hipMemcpyAsync"));
    GESMC_TRY(check_hip(hipEventRecord(F.done, s), "hipEventRecord"));
    F.live = true;
    for (ServeReq *R : ranks) {
        ++R->flights;
        R->done += k;
        if (R->done == R->r) {  // leaves the resident set; finished when this flight completes
            R->leaving = true;
            R->final_status = GESMC_OK;
        }
    }
    return GESMC_OK;
}

// Releases flight F's hold on R and finishes R if it is leaving and no live
// flight holds it any more.
void serve_release_locked(gesmc_server *S, ServeReq *R) {
    if (R->flights > 0) --R->flights;
    if (R->leaving && R->flights == 0 && !R->finished) serve_finish_locked(S, R, R->final_status);
}

// Waits for flight F and takes its outcome: results of the finishing graphs,
// outcome counts, input errors (a graph with one leaves the resident set and
// fails once no live flight holds it).
gesmc_status serve_complete(gesmc_server *S, ServeFlight &F) {
    const auto w0 = std::chrono::steady_clock::now();
    GESMC_TRY(check_hip(hipEventSynchronize(F.done), "hipEventSynchronize"));
    if (F.res_pending) {
        GESMC_TRY(check_hip(hipEventSynchronize(F.res_ev), "hipEventSynchronize"));
        F.res_pending = false;
    }
    const auto c0 = std::chrono::steady_clock::now();
    S->w_wait += std::chrono::duration<double>(c0 - w0).count();
    if (F.h_err[0] != 0) {
        set_error("internal consistency check failed (error bits 0x%x)", F.h_err[0]);
        return GESMC_E_INTERNAL;
    }
    const uint32_t G = (uint32_t)F.ranks.size();
    S->segs.clear();
    for (uint32_t q = 0; q < G; ++q) {
        ServeReq *R = F.ranks[q];
        if (F.rb[q] == ~0ull || F.h_gerr[q] || R->final_status != GESMC_OK) continue;
        R->result = (uint64_t *)malloc(std::max<uint64_t>(R->m, 1) * 8);
        if (!R->result) return GESMC_E_NOMEM;
        S->segs.push_back({R->result, F.h_res + F.rb[q], R->m * 8});
    }
    S->copier->copy(S->segs);
    S->w_copy += seconds_since(c0);
    uint64_t rounds = 0, rounds_max = 0;
    for (uint32_t st = 0; st < F.k; ++st) {
        rounds += F.h_ctr[st].rounds;
        rounds_max = std::max<uint64_t>(rounds_max, F.h_ctr[st].rounds);
    }
    std::lock_guard<std::mutex> lk(S->mu);
    ++S->iterations;
    for (uint32_t q = 0; q < G; ++q) {
        ServeReq *R = F.ranks[q];
        gesmc_stats &o = R->stats;
        o.attempts += (uint64_t)F.k * (R->m / 2);
        o.legal += F.h_gacc[4 * (size_t)q + 0];
        o.rej_loop += F.h_gacc[4 * (size_t)q + 1];
        o.rej_exists += F.h_gacc[4 * (size_t)q + 2];
        o.rej_pl += F.h_gacc[4 * (size_t)q + 3];
        o.rounds_sum += rounds;
        o.rounds_max = std::max<uint32_t>(o.rounds_max, (uint32_t)rounds_max);
        if (F.k) o.tuple_bytes = F.tuple_bytes;
        S->attempts += (uint64_t)F.k * (R->m / 2);
        S->legal += F.h_gacc[4 * (size_t)q + 0];
        const uint32_t ge = F.h_gerr[q];
        if (ge && R->final_status == GESMC_OK) {
            R->leaving = true;  // excluded from the next layouts
            R->final_status = q >= F.nsurv ? serve_map_gerr(ge) : GESMC_E_INTERNAL;
        }
        if (R->leaving && R->final_status == GESMC_OK) {
            o.supersteps = R->r;
            o.ms_device = 0;
        }
        serve_release_locked(S, R);
    }
    F.live = false;
    F.ranks.clear();
    return GESMC_OK;
}

// After a failed call: waits for the stream and fails every request that a
// flight holds or that is resident.
void serve_drain_locked(gesmc_server *S, gesmc_status st) {
    (void)hipStreamSynchronize(S->s);
    (void)hipStreamSynchronize(S->up);
    (void)hipStreamSynchronize(S->down);
    (void)hipGetLastError();
    S->stage_pending = false;
    S->load_recorded = false;
    for (ServeFlight &F : S->fl) {
        F.res_pending = false;
        for (ServeReq *R : F.ranks) R->flights = 0;
        for (ServeReq *R : F.ranks)
            if (!R->finished) serve_finish_locked(S, R, st);
        F.ranks.clear();
        F.live = false;
    }
    for (ServeReq *R : S->resident) {
        R->flights = 0;
        if (!R->finished) serve_finish_locked(S, R, st);
    }
    S->resident.clear();
    S->resident_edges = 0;
    S->resident_count = 0;
}

// The worker: a depth-one pipeline.  Each pass queues the next iteration
// (the layout and the graphs that finish are known on the host in advance)
// while the device still runs the previous one, then completes the previous
// one.  A cancelled graph, or one whose input turns out to be bad, leaves
// the resident set at the next pass and is finished once no queued
// iteration holds it.
void serve_loop(gesmc_server *S) {
    gesmc_ctx *c = S->c;
    (void)hipSetDevice(c->device);
    std::vector<ServeReq *> admit, trivial, next;
    bool dirty = true;  // the layout in buffer 0 differs from `resident`
    int cur = 0;        // flight slot of the next iteration; 1 - cur may be live
    for (;;) {
        admit.clear();
        trivial.clear();
        next.clear();
        uint32_t burst = 1;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] {
                return S->stop || !S->queue.empty() || !S->resident.empty() || S->fl[1 - cur].live;
            });
            if (S->stop) return;
            for (ServeReq *R : S->resident) {
                if (R->cancel && !R->leaving) {
                    R->leaving = true;
                    R->final_status = GESMC_E_CANCELED;
                }
                if (R->leaving) {
                    dirty = true;
                    if (R->flights == 0 && !R->finished) serve_finish_locked(S, R, R->final_status);
                } else {
                    next.push_back(R);
                }
            }
            uint64_t edges = 0, verts = 0;
            for (ServeReq *R : next) {
                edges += R->m + (R->m & 1);
                verts += R->n;
            }
            while (!S->queue.empty()) {
                ServeReq *R = S->queue.front();
                if (R->cancel) {
                    S->queue.pop_front();
                    serve_finish_locked(S, R, GESMC_E_CANCELED);
                    continue;
                }
                if (R->r == 0 || R->m < 2) {
                    S->queue.pop_front();
                    R->t_admit = seconds_since(S->t0);
                    trivial.push_back(R);
                    continue;
                }
                const uint64_t need = R->m + (R->m & 1);
                if (next.size() + admit.size() >= S->max_graphs || edges + need > S->cap_edges ||
                    verts + R->n > 0xFFFFFFFEull)
                    break;
                S->queue.pop_front();
                R->t_admit = seconds_since(S->t0);
                admit.push_back(R);
                edges += need;
                verts += R->n;
            }
            uint32_t rem = kServeBurstMax;
            for (ServeReq *R : next) rem = std::min(rem, R->r - R->done);
            for (ServeReq *R : admit) rem = std::min(rem, R->r - R->done);
            burst = std::max(1u, std::min(rem, S->queue.empty() ? kServeBurstIdle : kServeBurstMax));
        }
        const auto it0 = std::chrono::steady_clock::now();
        for (ServeReq *R : trivial) {
            const gesmc_status st = serve_trivial(R);
            std::lock_guard<std::mutex> lk(S->mu);
            serve_finish_locked(S, R, st);
        }
        bool queued = false;
        if (!next.empty() || !admit.empty()) {
            const bool relayout = dirty || !admit.empty();
            const gesmc_status st = serve_enqueue(S, S->fl[cur], next, admit, relayout, burst);
            std::lock_guard<std::mutex> lk(S->mu);
            if (st != GESMC_OK) {
                for (ServeReq *R : admit) S->resident.push_back(R);  // fail them with the others
                serve_drain_locked(S, st);
                dirty = true;
                S->busy_s += seconds_since(it0);
                continue;
            }
            queued = true;
            dirty = false;
            S->resident.clear();
            uint64_t edges = 0;
            for (ServeReq *R : S->fl[cur].ranks) {
                if (R->leaving) {
                    dirty = true;  // finishes with this flight: the next layout differs
                } else {
                    S->resident.push_back(R);
                    edges += R->m + (R->m & 1);
                }
            }
            S->resident_edges = edges;
            S->resident_count = (uint32_t)S->resident.size();
        } else {
            std::lock_guard<std::mutex> lk(S->mu);
            S->resident.clear();
            S->resident_edges = 0;
            S->resident_count = 0;
        }
        if (S->fl[1 - cur].live) {
            const gesmc_status st = serve_complete(S, S->fl[1 - cur]);
            std::lock_guard<std::mutex> lk(S->mu);
            if (st != GESMC_OK) {
                serve_drain_locked(S, st);
                dirty = true;
                queued = false;
            }
        }
        if (queued) cur = 1 - cur;
        std::lock_guard<std::mutex> lk(S->mu);
        S->busy_s += seconds_since(it0);
        S->copy_s += S->w_copy;
        S->wait_s += S->w_wait;
        S->w_copy = S->w_wait = 0;
    }
}

}  // namespace

extern "C" {

gesmc_status gesmc_server_create(gesmc_ctx *c, const gesmc_server_cfg *cfg, gesmc_server **out) {
    if (!c || !out) {
        set_error("null argument");
        return GESMC_E_INVAL;
    }
    *out = nullptr;
    if (c->strategy != 0) {
        set_error("serving needs the sorted-tuples strategy (GESMC_OPT_STRATEGY 0)");
        return GESMC_E_INVAL;
    }
    const uint64_t budget = (cfg && cfg->hbm_budget_bytes) ? cfg->hbm_budget_bytes : (16ull << 30);
    const uint32_t max_graphs = (cfg && cfg->max_graphs) ? cfg->max_graphs : 4096u;
    const uint32_t max_queue = (cfg && cfg->max_queue) ? cfg->max_queue : 65536u;
    const uint64_t cap_edges = std::min<uint64_t>(budget / kServeBytesPerEdge, kMaxEdges - 1 - max_graphs);
    if (cap_edges < 16 || max_graphs > (1u << kMaxFineBits)) {
        set_error("server budget too small or too many graphs");
        return GESMC_E_INVAL;
    }
    GESMC_TRY(check_hip(hipSetDevice(c->device), "hipSetDevice"));
    GESMC_TRY(ensure_capacity(c, cap_edges + 64));
    GESMC_TRY(ensure_counters(c, kServeBurstMax));
    GESMC_TRY(ensure_batch(c, max_graphs, cap_edges + 64));
    gesmc_server *S = new gesmc_server();
    S->c = c;
    c->serving = true;
    S->cap_edges = cap_edges;
    S->max_graphs = max_graphs;
    S->max_queue = max_queue;
    S->t0 = std::chrono::steady_clock::now();
    gesmc_status st = GESMC_OK;
    if (st == GESMC_OK) st = dev_alloc(c, (void **)&S->d_mv, max_graphs * sizeof(uint2));
    if (st == GESMC_OK) st = dev_alloc(c, (void **)&S->d_stage_off, (max_graphs + 1) * 8ull);
    if (st == GESMC_OK) st = dev_alloc(c, (void **)&S->d_stage_rank, max_graphs * 4ull);
    if (st == GESMC_OK && (hipEventCreateWithFlags(&S->stage_ev, hipEventDisableTiming) != hipSuccess ||
                           hipEventCreateWithFlags(&S->load_ev, hipEventDisableTiming) != hipSuccess)) {
        (void)hipGetLastError();
        set_error("hipEventCreate failed");
        st = GESMC_E_DEVICE;
    }
    for (ServeFlight &F : S->fl) {
        if (st != GESMC_OK) break;
        if (hipEventCreateWithFlags(&F.done, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&F.ext, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&F.res_ev, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void **)&F.h_gacc, max_graphs * 32ull, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&F.h_gerr, max_graphs * 4ull, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&F.h_ctr, kServeBurstMax * sizeof(StepCounters), hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc((void **)&F.h_err, 64, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            set_error("serving buffers could not be allocated");
            st = GESMC_E_NOMEM;
        }
    }
    if (st == GESMC_OK && (hipStreamCreateWithFlags(&S->s, hipStreamNonBlocking) != hipSuccess ||
                           hipStreamCreateWithFlags(&S->up, hipStreamNonBlocking) != hipSuccess ||
                           hipStreamCreateWithFlags(&S->down, hipStreamNonBlocking) != hipSuccess)) {
        (void)hipGetLastError();
        set_error("hipStreamCreate failed");
        st = GESMC_E_DEVICE;
    }
    if (st == GESMC_OK) {
        try {  // 7 copy threads beside the worker (the copies are memory-bound)
            const unsigned hc = std::max(2u, std::thread::hardware_concurrency());
            S->copier.reset(new gesmc::CopyPool(std::min(7u, hc - 1)));
        } catch (...) {
            set_error("cannot start the copy threads");
            st = GESMC_E_NOMEM;
        }
    }
    if (st != GESMC_OK) {
        gesmc_server_destroy(S);
        return st;
    }
    S->worker = std::thread(serve_loop, S);
    *out = S;
    return GESMC_OK;
}

void gesmc_server_destroy(gesmc_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    {
        std::unique_lock<std::mutex> lk(S->mu);
        for (auto &kv : S->reqs)
            if (!kv.second->finished) serve_finish_locked(S, kv.second, GESMC_E_CANCELED);
        S->cv_done.notify_all();
        // threads blocked in gesmc_wait take their (cancelled) results and
        // leave before any request or the server itself is freed
        S->cv_done.wait(lk, [&] { return S->waiters == 0; });
        for (auto &kv : S->reqs) {
            free(kv.second->result);
            delete kv.second;
        }
        S->reqs.clear();
    }
    for (hipStream_t q : {S->s, S->up, S->down})
        if (q) {
            (void)hipStreamSynchronize(q);
            (void)hipStreamDestroy(q);
        }
    for (void *p : {(void *)S->d_mv, (void *)S->d_stage_off, (void *)S->d_stage_rank, (void *)S->d_stage,
                    (void *)S->fl[0].d_res, (void *)S->fl[1].d_res})
        if (p) dev_free(S->c, p);
    S->c->serving = false;
    if (S->h_pin) (void)hipHostFree(S->h_pin);
    for (hipEvent_t e : {S->stage_ev, S->load_ev})
        if (e) (void)hipEventDestroy(e);
    for (ServeFlight &F : S->fl) {
        for (void *p : {(void *)F.h_res, (void *)F.h_gacc, (void *)F.h_gerr, (void *)F.h_ctr, (void *)F.h_err})
            if (p) (void)hipHostFree(p);
        for (hipEvent_t e : {F.done, F.ext, F.res_ev})
            if (e) (void)hipEventDestroy(e);
    }
    delete S;
}

gesmc_status gesmc_submit(gesmc_server *S, const gesmc_request *req, uint64_t *ticket) {
    if (!S || !req || !ticket || (req->m > 0 && !req->edges)) {
        set_error("null argument");
        return GESMC_E_INVAL;
    }
    if (req->m >= kMaxEdges || req->m + (req->m & 1) > S->cap_edges || req->n > 0xFFFFFFFEu) {
        set_error("request of m = %llu, n = %u can never fit the server", (unsigned long long)req->m, req->n);
        return GESMC_E_RANGE;
    }
    if ((uint64_t)req->t0 + req->r > 0x100000000ull) {
        set_error("superstep counter t0 + r overflows 32 bits");
        return GESMC_E_INVAL;
    }
    ServeReq *R = new ServeReq();
    R->edges.assign(req->edges, req->edges + req->m);
    R->m = req->m;
    R->n = req->n;
    R->t0 = req->t0;
    R->r = req->r;
    R->pl = req->pl;
    R->seed = req->seed;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->queue.size() >= S->max_queue) {
            delete R;
            set_error("queue full");
            return GESMC_E_AGAIN;
        }
        R->ticket = S->next_ticket++;
        R->t_submit = seconds_since(S->t0);
        S->reqs[R->ticket] = R;
        S->queue.push_back(R);
        ++S->submitted;
        *ticket = R->ticket;
    }
    S->cv_work.notify_one();
    return GESMC_OK;
}

static gesmc_status serve_take_locked(gesmc_server *S, std::unordered_map<uint64_t, ServeReq *>::iterator it,
                                      gesmc_result *out) {
    ServeReq *R = it->second;
    out->status = R->status;
    out->m = R->m;
    out->edges = R->status == GESMC_OK ? R->result : nullptr;
    if (R->status != GESMC_OK) free(R->result);
    out->stats = R->stats;
    out->t_submit = R->t_submit;
    out->t_admit = R->t_admit;
    out->t_done = R->t_done;
    S->reqs.erase(it);
    delete R;
    return GESMC_OK;
}

gesmc_status gesmc_poll(gesmc_server *S, uint64_t ticket, gesmc_result *out) {
    if (!S || !out) {
        set_error("null argument");
        return GESMC_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
        set_error("unknown ticket %llu", (unsigned long long)ticket);
        return GESMC_E_INVAL;
    }
    if (!it->second->finished) return GESMC_E_AGAIN;
    return serve_take_locked(S, it, out);
}

gesmc_status gesmc_wait(gesmc_server *S, uint64_t ticket, gesmc_result *out) {
    if (!S || !out) {
        set_error("null argument");
        return GESMC_E_INVAL;
    }
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
        set_error("unknown ticket %llu", (unsigned long long)ticket);
        return GESMC_E_INVAL;
    }
    ServeReq *R = it->second;
    ++S->waiters;
    S->cv_done.wait(lk, [&] { return R->finished; });  // destroy finishes every request before it frees them
    --S->waiters;
    const gesmc_status st = serve_take_locked(S, S->reqs.find(ticket), out);
    if (S->stop) S->cv_done.notify_all();  // a destroy in progress waits for the last waiter
    return st;
}

gesmc_status gesmc_cancel(gesmc_server *S, uint64_t ticket) {
    if (!S) {
        set_error("null server");
        return GESMC_E_INVAL;
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->reqs.find(ticket);
        if (it == S->reqs.end()) {
            set_error("unknown ticket %llu", (unsigned long long)ticket);
            return GESMC_E_INVAL;
        }
        it->second->cancel = true;
    }
    S->cv_work.notify_one();
    return GESMC_OK;
}

void gesmc_result_free(gesmc_result *res) {
    if (!res) return;
    free(res->edges);
    res->edges = nullptr;
}

gesmc_status gesmc_server_info_get(gesmc_server *S, gesmc_server_info *out) {
    if (!S || !out) {
        set_error("null argument");
        return GESMC_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->iterations = S->iterations;
    out->attempts = S->attempts;
    out->legal = S->legal;
    out->resident_edges = S->resident_edges;
    out->queued = (uint32_t)S->queue.size();
    out->resident = S->resident_count;
    out->busy_s = S->busy_s;
    out->copy_s = S->copy_s;
    out->wait_s = S->wait_s;
    out->now_s = seconds_since(S->t0);
    return GESMC_OK;
}

}  // extern "C"

// ParES (Alg. 2): host side of gesmc_run_es and gesmc_es_draws.  Part of the
// library's translation unit (included by gesmc.hip after its entry points).
#pragma once

namespace {

// Switches per launch of k_es_chain (an epoch): the edge set is rebuilt
// between epochs, so that its used slots (live edges plus retired ones) stay
// below m + 2 * epoch, and its slot count (a power of two at least twice
// that) keeps the load at or below one half.
uint64_t es_epoch(uint32_t m) { return std::max<uint64_t>(m / 2, 65536); }

uint64_t es_slots(uint32_t m) {
    const uint64_t want = 2 * ((uint64_t)m + 2 * es_epoch(m));
    uint64_t T = 1024;
    while (T < want) T <<= 1;
    return T;
}

gesmc_status es_ensure(gesmc_ctx *c, uint32_t m) {
    const uint64_t cap = std::max<uint64_t>(m, 1024), T = es_slots(m);
    if (!c->es_ctr) {
        GESMC_TRY(dev_alloc(c, (void **)&c->es_ctr, sizeof(EsCounters)));
        if (hipHostMalloc((void **)&c->h_es_ctr, sizeof(EsCounters), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            c->h_es_ctr = nullptr;
            set_error("hipHostMalloc failed");
            return GESMC_E_NOMEM;
        }
    }
    if (cap > c->es_cap_m) {
        for (void **q : {(void **)&c->es_E, (void **)&c->es_slot}) {
            if (*q) dev_free(c, *q);
            *q = nullptr;
        }
        c->es_cap_m = 0;
        GESMC_TRY(dev_alloc(c, (void **)&c->es_E, cap * 8));
        GESMC_TRY(dev_alloc(c, (void **)&c->es_slot, cap * 4));
        c->es_cap_m = cap;
    }
    if (T > c->es_cap_T) {
        if (c->es_H) dev_free(c, c->es_H);
        c->es_H = nullptr;
        c->es_cap_T = 0;
        GESMC_TRY(dev_alloc(c, (void **)&c->es_H, T * 8));
        c->es_cap_T = T;
    }
    return GESMC_OK;
}

gesmc_status run_es_impl(gesmc_ctx *c, void *stream, const uint64_t *d_in, uint64_t *d_out, uint64_t m64, uint32_t n,
                         uint64_t seed, uint64_t k0, uint64_t r, uint8_t *d_outcome, gesmc_es_stats *stats) {
    if (!c) {
        set_error("null context");
        return GESMC_E_INVAL;
    }
    if (m64 > 0 && (!d_in || !d_out)) {
        set_error("null edge pointer");
        return GESMC_E_INVAL;
    }
    if (m64 >= kMaxEdges) {
        set_error("m = %llu exceeds the limit 2^30 - 1", (unsigned long long)m64);
        return GESMC_E_RANGE;
    }
    if (r > ~0ull - k0) {
        set_error("switch counter k0 + r overflows 64 bits");
        return GESMC_E_INVAL;
    }
    GESMC_TRY(check_hip(hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    const uint32_t m = (uint32_t)m64;
    GESMC_TRY(es_ensure(c, m));
    const uint64_t T = es_slots(m), epoch = es_epoch(m);
    const uint32_t mask = (uint32_t)(T - 1);
    const uint32_t s0 = (uint32_t)seed, s1 = (uint32_t)(seed >> 32);
    GESMC_TRY(check_hip(hipEventRecord(c->call_a, s), "hipEventRecord"));
    GESMC_TRY(launch(c, s, KID_MISC, 0, k_zero_words, dim3(4), dim3(256), 0, c->err, (uint64_t)64));
    GESMC_TRY(launch(c, s, KID_MISC, 0, k_zero_words, dim3(1), dim3(64), 0, (uint32_t *)c->es_ctr,
                     (uint64_t)(sizeof(EsCounters) / 4)));
    if (m > 0)
        GESMC_TRY(launch(c, s, KID_LOAD, m, k_load, dim3(grid_stride_blocks(c, m)), dim3(kBlock), 0,
                         (const unsigned long long *)d_in, m, n, c->es_slot, c->es_E, c->err, 0u));
    uint64_t launches = 0;
    if (m >= 2) {
        for (uint64_t kb = k0; kb == k0 || kb - k0 < r; kb += epoch) {
            const uint64_t ke = kb + std::min<uint64_t>(epoch, r - (kb - k0));
            // (re)build the edge set from the edge list: all slots live, none retired
            GESMC_TRY(launch(c, s, KID_ES_BUILD, T, k_es_clear, dim3(grid_stride_blocks(c, T)), dim3(kBlock), 0,
                             c->es_H, T));
            GESMC_TRY(launch(c, s, KID_ES_BUILD, m, k_es_insert_all, dim3(grid_stride_blocks(c, m)), dim3(kBlock),
                             0, (const unsigned long long *)c->es_E, m, c->es_H, mask, c->es_slot, c->err,
                             c->es_ctr));
            if (ke > kb)
                GESMC_TRY(launch(c, s, KID_ES_CHAIN, ke - kb, k_es_chain, dim3(1), dim3(kEsThreads), 0, c->es_E,
                                 c->es_slot, c->es_H, mask, m, s0, s1, kb, ke, k0, d_outcome, c->es_ctr, c->err));
            ++launches;
            if (ke - k0 >= r) break;
        }
    }
    if (m > 0)
        GESMC_TRY(launch(c, s, KID_UNPERMUTE, m, k_es_out, dim3(grid_stride_blocks(c, m)), dim3(kBlock), 0,
                         (const unsigned long long *)c->es_E, m, (unsigned long long *)d_out,
                         (const uint32_t *)c->err));
    GESMC_TRY(check_hip(hipEventRecord(c->call_b, s), "hipEventRecord"));
    GESMC_TRY(check_hip(hipMemcpyAsync(c->h_err, c->err, 4, hipMemcpyDeviceToHost, s), "hipMemcpyAsync"));
    GESMC_TRY(check_hip(hipMemcpyAsync(c->h_es_ctr, c->es_ctr, sizeof(EsCounters), hipMemcpyDeviceToHost, s),
                        "hipMemcpyAsync"));
    GESMC_TRY(check_hip(hipStreamSynchronize(s), "hipStreamSynchronize"));
    if (c->profile) collect_profile(c);
    GESMC_TRY(map_err(*c->h_err));
    if (stats) {
        const EsCounters &h = *c->h_es_ctr;
        memset(stats, 0, sizeof(*stats));
        stats->attempts = m >= 2 ? r : 0;
        stats->legal = h.legal;
        stats->rej_loop = h.rej_loop;
        stats->rej_exists = h.rej_exists;
        stats->supersteps = h.supersteps;
        stats->rounds_sum = h.rounds;
        stats->rounds_max = (uint32_t)h.rounds_max;
        stats->epochs = (uint32_t)launches;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->call_a, c->call_b) == hipSuccess)
            stats->ms_device = ms;
        else
            (void)hipGetLastError();
    }
    return GESMC_OK;
}

}  // namespace

extern "C" {

gesmc_status gesmc_run_es(gesmc_ctx *ctx, void *stream, const uint64_t *d_in, uint64_t *d_out, uint64_t m, uint32_t n,
                          uint64_t seed, uint64_t k0, uint64_t r, uint32_t flags, uint8_t *d_outcome,
                          gesmc_es_stats *stats) {
    if (flags != 0) {
        set_error("flags must be 0");
        return GESMC_E_INVAL;
    }
    return run_es_impl(ctx, stream, d_in, d_out, m, n, seed, k0, r, d_outcome, stats);
}

gesmc_status gesmc_es_draws(gesmc_ctx *c, void *stream, uint64_t m, uint64_t seed, uint64_t k0, uint64_t count,
                            uint64_t *d_i, uint64_t *d_j, uint8_t *d_g) {
    if (!c || (count > 0 && (!d_i || !d_j || !d_g))) {
        set_error("null argument");
        return GESMC_E_INVAL;
    }
    if (m < 2 || m >= kMaxEdges) {
        set_error("m = %llu: draws need 2 <= m < 2^30", (unsigned long long)m);
        return GESMC_E_RANGE;
    }
    if (count > ~0ull - k0) {
        set_error("switch counter k0 + count overflows 64 bits");
        return GESMC_E_INVAL;
    }
    GESMC_TRY(check_hip(hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    if (count > 0)
        GESMC_TRY(launch(c, s, KID_MISC, count, k_es_draws, dim3(grid_stride_blocks(c, count)), dim3(kBlock), 0, k0,
                         count, (uint32_t)m, (uint32_t)seed, (uint32_t)(seed >> 32), (unsigned long long *)d_i,
                         (unsigned long long *)d_j, d_g));
    GESMC_TRY(check_hip(hipStreamSynchronize(s), "hipStreamSynchronize"));
    if (c->profile) collect_profile(c);
    return GESMC_OK;
}

}  // extern "C"

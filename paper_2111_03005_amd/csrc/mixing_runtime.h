// Mixing diagnostic (Sec. 6.1): host side of gesmc_mixing.  Part of the
// library's translation unit (included by gesmc.hip after its entry points).
#pragma once

namespace {

constexpr uint32_t kMixMaxN = 1u << 14;  // pair ids below 2^27
constexpr uint32_t kMixMaxThin = 16;

gesmc_status mixing_impl(gesmc_ctx *c, void *stream, const uint64_t *d_in, uint64_t m64, uint32_t n, uint64_t seed,
                         uint32_t chain, uint32_t pl, uint32_t K, const uint32_t *thin, uint32_t nthin,
                         gesmc_mixing_result *out, double *ms_total) {
    if (!c || !thin || !out || (m64 > 0 && !d_in)) {
        set_error("null argument");
        return GESMC_E_INVAL;
    }
    if (chain > 1 || nthin == 0 || nthin > kMixMaxThin) {
        set_error("chain must be 0 or 1 and 1 <= nthin <= %u", kMixMaxThin);
        return GESMC_E_INVAL;
    }
    for (uint32_t q = 0; q < nthin; ++q)
        if (thin[q] == 0) {
            set_error("thinning values must be at least 1");
            return GESMC_E_INVAL;
        }
    if (n < 2 || n > kMixMaxN || m64 >= kMaxEdges) {
        set_error("the mixing diagnostic needs 2 <= n <= %u (dense pair counters) and m < 2^30", kMixMaxN);
        return GESMC_E_RANGE;
    }
    if (chain == 0 && (uint64_t)K > 0x100000000ull) {
        set_error("K exceeds the 32-bit superstep counter");
        return GESMC_E_INVAL;
    }
    GESMC_TRY(check_hip(hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    const uint32_t m = (uint32_t)m64, ell = m / 2;
    const uint64_t npairs = (uint64_t)n * (n - 1) / 2, words = (npairs + 31) / 32;
    // one block: the state, the current-sample bitmap, and per thinning value
    // the previous sample's list and bitmap, the tracked bitmap and the counters
    const uint64_t mm = std::max<uint32_t>(m, 1);
    const uint64_t per_q = mm * 8 + words * 8 + npairs * sizeof(MixCount) + 256 * 3;
    const uint64_t bytes = mm * 8 + words * 4 + 64 + nthin * per_q + 256;
    unsigned char *blk = nullptr;
    GESMC_TRY(dev_alloc(c, (void **)&blk, bytes));
    struct Free {
        gesmc_ctx *c;
        unsigned char *p;
        ~Free() {
            if (p) dev_free(c, p);
        }
    } guard{c, blk};
    uint64_t off = 0;
    auto take = [&](uint64_t b) {
        off = (off + 255) & ~255ull;
        unsigned char *p = blk + off;
        off += b;
        return p;
    };
    auto *E = (unsigned long long *)take(mm * 8);
    auto *cur_bits = (uint32_t *)take(words * 4);
    auto *res = (unsigned long long *)take(64);
    std::vector<unsigned long long *> prev(nthin);
    std::vector<uint32_t *> prev_bits(nthin), ever(nthin);
    std::vector<MixCount *> cnt(nthin);
    for (uint32_t q = 0; q < nthin; ++q) {
        prev[q] = (unsigned long long *)take(mm * 8);
        prev_bits[q] = (uint32_t *)take(words * 4);
        ever[q] = (uint32_t *)take(words * 4);
        cnt[q] = (MixCount *)take(npairs * sizeof(MixCount));
    }
    GESMC_TRY(check_hip(hipMemsetAsync(blk, 0, bytes, s), "hipMemsetAsync"));
    // X_0: the input validated and canonicalised (a call with no superstep)
    GESMC_TRY(run_impl(c, stream, d_in, (uint64_t *)E, m, n, seed, 0, 0, pl, nullptr, nullptr, nullptr));
    const uint32_t gb = grid_stride_blocks(c, m);
    for (uint32_t q = 0; q < nthin && m > 0; ++q) {
        GESMC_TRY(launch(c, s, KID_MIX, m, k_mix_bits, dim3(gb), dim3(kBlock), 0, (const unsigned long long *)E, m, n,
                         prev_bits[q], true));
        GESMC_TRY(launch(c, s, KID_MIX, m, k_mix_bits, dim3(gb), dim3(kBlock), 0, (const unsigned long long *)E, m, n,
                         ever[q], true));
        GESMC_TRY(check_hip(hipMemcpyAsync(prev[q], E, m * 8ull, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync"));
    }
    auto t_start = std::chrono::steady_clock::now();
    for (uint32_t t = 0; t < K; ++t) {
        if (m >= 2) {
            if (chain == 0)
                GESMC_TRY(run_impl(c, stream, (const uint64_t *)E, (uint64_t *)E, m, n, seed, t, 1, pl, nullptr,
                                   nullptr, nullptr));
            else
                GESMC_TRY(run_es_impl(c, stream, (const uint64_t *)E, (uint64_t *)E, m, n, seed, (uint64_t)t * ell,
                                      ell, nullptr, nullptr));
        }
        const uint32_t tt = t + 1;
        bool any = false;
        for (uint32_t q = 0; q < nthin; ++q) any |= tt % thin[q] == 0;
        if (!any || m == 0) continue;
        GESMC_TRY(launch(c, s, KID_MIX, m, k_mix_bits, dim3(gb), dim3(kBlock), 0, (const unsigned long long *)E, m, n,
                         cur_bits, true));
        for (uint32_t q = 0; q < nthin; ++q) {
            if (tt % thin[q]) continue;
            GESMC_TRY(launch(c, s, KID_MIX, m, k_mix_count, dim3(gb), dim3(kBlock), 0, (const unsigned long long *)E,
                             (const unsigned long long *)prev[q], m, n, (const uint32_t *)cur_bits,
                             (const uint32_t *)prev_bits[q], cnt[q], ever[q]));
            GESMC_TRY(launch(c, s, KID_MIX, m, k_mix_bits, dim3(gb), dim3(kBlock), 0,
                             (const unsigned long long *)prev[q], m, n, prev_bits[q], false));
            GESMC_TRY(launch(c, s, KID_MIX, m, k_mix_bits, dim3(gb), dim3(kBlock), 0, (const unsigned long long *)E,
                             m, n, prev_bits[q], true));
            GESMC_TRY(check_hip(hipMemcpyAsync(prev[q], E, m * 8ull, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync"));
        }
        GESMC_TRY(launch(c, s, KID_MIX, m, k_mix_bits, dim3(gb), dim3(kBlock), 0, (const unsigned long long *)E, m, n,
                         cur_bits, false));
    }
    for (uint32_t q = 0; q < nthin; ++q) {
        const uint32_t N = K / thin[q];
        unsigned long long h[6] = {0, 0, 0, 0, 0, 0};
        GESMC_TRY(check_hip(hipMemsetAsync(res, 0, 64, s), "hipMemsetAsync"));
        GESMC_TRY(launch(c, s, KID_MIX, npairs, k_mix_decide, dim3(grid_stride_blocks(c, npairs)), dim3(kBlock), 0,
                         (const MixCount *)cnt[q], (const uint32_t *)ever[q], npairs, N, res));
        GESMC_TRY(check_hip(hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, s), "hipMemcpyAsync"));
        GESMC_TRY(check_hip(hipStreamSynchronize(s), "hipStreamSynchronize"));
        gesmc_mixing_result &o = out[q];
        memset(&o, 0, sizeof(o));
        o.k = thin[q];
        o.transitions = N;
        o.tracked = h[0];
        o.non_independent = N > 0 ? h[1] : 0;
        o.n01 = h[2];
        o.n10 = h[3];
        o.n11 = h[4];
        o.n00 = (uint64_t)N * h[0] - h[2] - h[3] - h[4];
    }
    GESMC_TRY(check_hip(hipStreamSynchronize(s), "hipStreamSynchronize"));
    if (ms_total)
        *ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (c->profile) collect_profile(c);
    return GESMC_OK;
}

}  // namespace

extern "C" {

gesmc_status gesmc_mixing(gesmc_ctx *ctx, void *stream, const uint64_t *d_in, uint64_t m, uint32_t n, uint64_t seed,
                          uint32_t chain, uint32_t pl, uint32_t K, const uint32_t *thin, uint32_t nthin,
                          gesmc_mixing_result *out, double *ms_chain) {
    return mixing_impl(ctx, stream, d_in, m, n, seed, chain, pl, K, thin, nthin, out, ms_chain);
}

}  // extern "C"

// Input realisation (the steps before the chain that build Sec. 6's synthetic
// inputs): host side of gesmc_gen_gnp, gesmc_gen_pld_degrees,
// gesmc_gen_havel_hakimi and gesmc_gen_relabel.  Part of the library's
// translation unit (included by gesmc.hip after its entry points).  Each call
// allocates its work buffers, synchronises its stream (sizes come back to
// the host) and frees them.
#pragma once

namespace {

// A block of device memory carved into aligned pieces, freed at scope exit.
struct GenBlock {
    gesmc_ctx *c;
    unsigned char *base = nullptr;
    uint64_t off = 0;
    explicit GenBlock(gesmc_ctx *ctx) : c(ctx) {}
    ~GenBlock() {
        if (base) dev_free(c, base);
    }
    template <typename T>
    T *take(uint64_t count) {
        off = (off + 255) & ~255ull;
        T *p = (T *)(base + off);
        off += std::max<uint64_t>(count, 1) * sizeof(T);
        return p;
    }
};

uint64_t gen_bytes_with_align(std::initializer_list<uint64_t> sizes) {
    uint64_t b = 0;
    for (uint64_t s : sizes) b += ((std::max<uint64_t>(s, 1) + 255) & ~255ull) + 256;
    return b;
}

constexpr uint64_t kGenScanTile = (uint64_t)kGenScanBlock * kGenScanItems;

// Exclusive scan of a[0, n) into out (u64) and the total into *total (device).
template <typename T>
gesmc_status gen_scan(gesmc_ctx *c, hipStream_t s, const T *a, uint64_t n, unsigned long long *out,
                      unsigned long long *sums, unsigned long long *total) {
    const uint32_t nb = (uint32_t)std::max<uint64_t>(1, (n + kGenScanTile - 1) / kGenScanTile);
    GESMC_TRY(launch(c, s, KID_GEN, n, k_gen_block_sums<T>, dim3(nb), dim3(kGenScanBlock), 0, a, n, sums));
    GESMC_TRY(launch(c, s, KID_GEN, 0, k_gen_scan_sums, dim3(1), dim3(kGenScanBlock), 0, sums, nb, total));
    GESMC_TRY(launch(c, s, KID_GEN, n, k_gen_scan_apply<T>, dim3(nb), dim3(kGenScanBlock), 0, a, n,
                     (const unsigned long long *)sums, out));
    return GESMC_OK;
}

uint64_t gen_scan_sums(uint64_t n) { return std::max<uint64_t>(1, (n + kGenScanTile - 1) / kGenScanTile); }

gesmc_status gen_sync(gesmc_ctx *c, hipStream_t s) {
    GESMC_TRY(check_hip(hipStreamSynchronize(s), "hipStreamSynchronize"));
    if (c->profile) collect_profile(c);
    return GESMC_OK;
}

// Chunk length of G(n,p): the smallest power of two >= 64 with L p >= 64, at
// most 2^40 (each comparison is exact: L is a power of two).
uint64_t gnp_chunk_length(double p) {
    uint64_t L = 64;
    while ((double)L * p < 64.0 && L < (1ull << 40)) L <<= 1;
    return L;
}

gesmc_status gen_gnp_impl(gesmc_ctx *c, void *stream, uint32_t n, double p, uint64_t seed, uint64_t *d_out,
                          uint64_t cap, uint64_t *m_out) {
    if (!c || !m_out || p != p) {
        set_error("null argument or p is NaN");
        return GESMC_E_INVAL;
    }
    *m_out = 0;
    if (n < 2 || !(p > 0.0)) return GESMC_OK;
    GESMC_TRY(check_hip(hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    const uint64_t N = (uint64_t)n * (n - 1) / 2;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (p >= 1.0) {
        *m_out = N;
        if (!d_out) return GESMC_OK;
        if (N > cap) {
            set_error("G(n,p) has %llu edges, more than cap = %llu", (unsigned long long)N, (unsigned long long)cap);
            return GESMC_E_RANGE;
        }
        GESMC_TRY(launch(c, s, KID_GEN, N, k_gnp_complete, dim3(grid_stride_blocks(c, N)), dim3(kBlock), 0, N,
                         (unsigned long long *)d_out));
        return gen_sync(c, s);
    }
    const uint64_t L = gnp_chunk_length(p);
    const uint64_t nchunks = (N + L - 1) / L;
    if (alloc_forbidden()) return GESMC_E_INTERNAL;
    GenBlock blk(c);
    const uint64_t nsum = gen_scan_sums(nchunks);
    GESMC_TRY(dev_alloc(c, (void **)&blk.base, gen_bytes_with_align({nchunks * 4, nchunks * 8, nsum * 8, 64})));
    uint32_t *counts = blk.take<uint32_t>(nchunks);
    unsigned long long *offs = blk.take<unsigned long long>(nchunks);
    unsigned long long *sums = blk.take<unsigned long long>(nsum);
    unsigned long long *total = blk.take<unsigned long long>(8);
    const uint32_t waves = (uint32_t)std::min<uint64_t>(nchunks, (uint64_t)c->num_cus * 64);
    const dim3 grid(std::max<uint32_t>(1, ceil_div(waves, kGnpBlock / 64)));
    // the chunk walk needs ln(1 - p); every wave computes it with the same
    // steps as the draws (no host arithmetic enters the sample)
    const double q = 1.0 - p;
    GESMC_TRY(launch(c, s, KID_GEN, nchunks, k_gnp_count, grid, dim3(kGnpBlock), 0, nchunks, L, N, q, k0, k1,
                     counts));
    GESMC_TRY(gen_scan(c, s, (const uint32_t *)counts, nchunks, offs, sums, total));
    unsigned long long h_total = 0;
    GESMC_TRY(check_hip(hipMemcpyAsync(&h_total, total, 8, hipMemcpyDeviceToHost, s), "hipMemcpyAsync"));
    GESMC_TRY(gen_sync(c, s));
    *m_out = h_total;
    if (!d_out) return GESMC_OK;
    if (h_total > cap) {
        set_error("G(n,p) drew %llu edges, more than cap = %llu", h_total, (unsigned long long)cap);
        return GESMC_E_RANGE;
    }
    GESMC_TRY(launch(c, s, KID_GEN, h_total, k_gnp_write, grid, dim3(kGnpBlock), 0, nchunks, L, N, q, k0, k1,
                     (const unsigned long long *)offs, (unsigned long long *)d_out));
    return gen_sync(c, s);
}

gesmc_status gen_pld_impl(gesmc_ctx *c, void *stream, uint32_t n, double gamma, uint32_t dmin, uint32_t dmax,
                          uint64_t seed, uint32_t *d_deg, uint64_t *sum_out) {
    if (!c || !sum_out || (n > 0 && !d_deg)) {
        set_error("null argument");
        return GESMC_E_INVAL;
    }
    if (n == 0 || dmin < 1 || dmax < dmin || dmax - dmin >= (1u << 20) || !(gamma >= 0.0) ||
        gamma * std::log((double)dmax / (double)dmin) > 690.0) {
        set_error("need n >= 1, 1 <= dmin <= dmax, dmax - dmin < 2^20, gamma >= 0 and (dmax/dmin)^gamma < e^690");
        return GESMC_E_INVAL;
    }
    GESMC_TRY(check_hip(hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t nv = dmax - dmin + 1;
    if (alloc_forbidden()) return GESMC_E_INTERNAL;
    GenBlock blk(c);
    const uint64_t nsum = gen_scan_sums(nv);
    GESMC_TRY(dev_alloc(c, (void **)&blk.base, gen_bytes_with_align({(uint64_t)nv * 8, (uint64_t)nv * 8, nsum * 8, 64})));
    unsigned long long *W = blk.take<unsigned long long>(nv);
    unsigned long long *C = blk.take<unsigned long long>(nv);
    unsigned long long *sums = blk.take<unsigned long long>(nsum);
    unsigned long long *words = blk.take<unsigned long long>(8);  // [0] scan total, [1] degree sum, [2] info
    GESMC_TRY(launch(c, s, KID_MISC, 0, k_zero_words, dim3(1), dim3(64), 0, (uint32_t *)words, (uint64_t)16));
    GESMC_TRY(launch(c, s, KID_GEN, nv, k_pld_weights, dim3(ceil_div(nv, kBlock)), dim3(kBlock), 0, nv, dmin, gamma,
                     W));
    GESMC_TRY(gen_scan(c, s, (const unsigned long long *)W, nv, C, sums, words));
    GESMC_TRY(launch(c, s, KID_GEN, nv, k_pld_cdf, dim3(ceil_div(nv, kBlock)), dim3(kBlock), 0,
                     (const unsigned long long *)W, nv, C));
    GESMC_TRY(launch(c, s, KID_GEN, n, k_pld_draw, dim3(grid_stride_blocks(c, n)), dim3(kBlock), 0, n,
                     (const unsigned long long *)C, nv, dmin, k0, k1, d_deg, words + 1));
    GESMC_TRY(launch(c, s, KID_GEN, 0, k_pld_even, dim3(1), dim3(64), 0, (const unsigned long long *)C, nv, dmin,
                     dmax, k0, k1, d_deg, words + 1, (uint32_t *)(words + 2)));
    unsigned long long h[3] = {0, 0, 0};
    GESMC_TRY(check_hip(hipMemcpyAsync(h, words, 24, hipMemcpyDeviceToHost, s), "hipMemcpyAsync"));
    GESMC_TRY(gen_sync(c, s));
    const uint32_t fail = (uint32_t)(h[2] >> 32);
    if (fail) {
        set_error("no even degree sum (a single odd degree value on an odd n, or 65535 redraws)");
        return GESMC_E_INVAL;
    }
    *sum_out = h[1];
    return GESMC_OK;
}

gesmc_status gen_hh_impl(gesmc_ctx *c, void *stream, uint32_t n, const uint32_t *d_deg, uint64_t *d_out,
                         uint64_t cap, uint64_t *m_out) {
    if (!c || !m_out || (n > 0 && !d_deg)) {
        set_error("null argument");
        return GESMC_E_INVAL;
    }
    *m_out = 0;
    if (n == 0) return GESMC_OK;
    GESMC_TRY(check_hip(hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    if (alloc_forbidden()) return GESMC_E_INTERNAL;
    // degree statistics first: the largest degree sizes the state
    GenBlock sblk(c);
    GESMC_TRY(dev_alloc(c, (void **)&sblk.base, 256));
    uint32_t *w = (uint32_t *)sblk.base;  // [0] max degree, [2..3] sum
    GESMC_TRY(launch(c, s, KID_MISC, 0, k_zero_words, dim3(1), dim3(64), 0, w, (uint64_t)8));
    GESMC_TRY(launch(c, s, KID_GEN, n, k_hh_stats, dim3(grid_stride_blocks(c, n)), dim3(kBlock), 0, d_deg, n, w,
                     (unsigned long long *)(w + 2)));
    uint32_t hw[4] = {0, 0, 0, 0};
    GESMC_TRY(check_hip(hipMemcpyAsync(hw, w, 16, hipMemcpyDeviceToHost, s), "hipMemcpyAsync"));
    GESMC_TRY(gen_sync(c, s));
    const uint32_t D = hw[0];
    const uint64_t sum = (uint64_t)hw[2] | ((uint64_t)hw[3] << 32);
    if ((sum & 1) || (sum > 0 && D >= n)) {
        set_error("the degree sequence is not graphical (%s)", (sum & 1) ? "odd sum" : "a degree >= n");
        return GESMC_E_NOT_GRAPHICAL;
    }
    const uint64_t m = sum / 2;
    *m_out = m;
    if (!d_out || m == 0) return GESMC_OK;
    if (m > cap) {
        set_error("the realisation has %llu edges, more than cap = %llu", (unsigned long long)m,
                  (unsigned long long)cap);
        return GESMC_E_RANGE;
    }
    if (D > kHhMaxDeg || m >= (1ull << 32)) {
        set_error("Havel-Hakimi on the device takes degrees up to %u and fewer than 2^32 edges", kHhMaxDeg);
        return GESMC_E_RANGE;
    }
    // ranges of T ids (a multiple of 64), at most 1024 of them
    uint32_t T = std::max<uint32_t>(4096, (uint32_t)(((uint64_t)n + 1023) / 1024));
    T = (T + 63) & ~63u;
    const uint32_t nb = ceil_div(n, T);
    const uint64_t nM = (uint64_t)(D + 1) * nb;
    const uint64_t nsum = gen_scan_sums(nM);
    GenBlock blk(c);
    GESMC_TRY(dev_alloc(c, (void **)&blk.base,
                        gen_bytes_with_align({nM * 4, nM * 8, nsum * 8, 64, (uint64_t)n * 4, (uint64_t)(D + 2) * 4,
                                              (uint64_t)n * sizeof(HhStep), 64})));
    uint32_t *M = blk.take<uint32_t>(nM);
    unsigned long long *Moff = blk.take<unsigned long long>(nM);
    unsigned long long *sums = blk.take<unsigned long long>(nsum);
    unsigned long long *total = blk.take<unsigned long long>(8);
    uint32_t *O = blk.take<uint32_t>(n);
    uint32_t *E0 = blk.take<uint32_t>(D + 2);
    HhStep *log = blk.take<HhStep>(n);
    uint32_t *status = blk.take<uint32_t>(16);
    const size_t hist_lds = (size_t)(D + 1) * 4;
    GESMC_TRY(launch(c, s, KID_GEN, n, k_hh_hist, dim3(nb), dim3(kBlock), hist_lds, d_deg, n, T, D, nb, M));
    GESMC_TRY(gen_scan(c, s, (const uint32_t *)M, nM, Moff, sums, total));
    GESMC_TRY(launch(c, s, KID_GEN, n, k_hh_place, dim3(nb), dim3(64), hist_lds, d_deg, n, T, D, nb,
                     (const unsigned long long *)Moff, O));
    GESMC_TRY(launch(c, s, KID_GEN, 0, k_hh_bounds, dim3(ceil_div(D + 2, kBlock)), dim3(kBlock), 0,
                     (const unsigned long long *)Moff, D, nb, E0));
    const size_t step_lds = (size_t)(std::max<uint32_t>(D, 64) + 2) * 4;
    GESMC_TRY(launch(c, s, KID_GEN_HH_STEPS, m, k_hh_steps, dim3(1), dim3(64), step_lds, (const uint32_t *)E0, D, n,
                     log, status));
    uint32_t hs[2] = {0, 0};
    GESMC_TRY(check_hip(hipMemcpyAsync(hs, status, 8, hipMemcpyDeviceToHost, s), "hipMemcpyAsync"));
    GESMC_TRY(gen_sync(c, s));
    if (hs[1] == 1) {
        set_error("the degree sequence is not graphical (Havel-Hakimi ran out of partners at step %u)", hs[0]);
        return GESMC_E_NOT_GRAPHICAL;
    }
    if (hs[1]) {
        set_error("Havel-Hakimi state inconsistent at step %u", hs[0]);
        return GESMC_E_INTERNAL;
    }
    const uint32_t S = hs[0];
    if (S == 0 || S > n) {
        set_error("Havel-Hakimi took %u steps on %u vertices", S, n);
        return GESMC_E_INTERNAL;
    }
    GESMC_TRY(launch(c, s, KID_GEN, m, k_hh_emit, dim3(ceil_div(S, kHhEmitSteps)), dim3(kBlock), 0,
                     (const HhStep *)log, S, (uint32_t)m, (const uint32_t *)O, n, (unsigned long long *)d_out));
    return gen_sync(c, s);
}

gesmc_status gen_relabel_impl(gesmc_ctx *c, void *stream, uint64_t *d_edges, uint64_t m, uint32_t n, uint64_t seed) {
    if (!c || (m > 0 && !d_edges)) {
        set_error("null argument");
        return GESMC_E_INVAL;
    }
    if (n == 0 || n >= kMaxEdges) {
        if (m == 0 && n == 0) return GESMC_OK;
        set_error("relabelling needs 1 <= n < 2^30");
        return GESMC_E_RANGE;
    }
    GESMC_TRY(check_hip(hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    if (alloc_forbidden()) return GESMC_E_INTERNAL;
    GenBlock blk(c);
    GESMC_TRY(dev_alloc(c, (void **)&blk.base, gen_bytes_with_align({(uint64_t)n * 4, (uint64_t)n * 4})));
    uint32_t *pi = blk.take<uint32_t>(n);
    uint32_t *sigma = blk.take<uint32_t>(n);
    GESMC_TRY(gesmc_permutation(c, stream, n, seed ^ 0x9E3779B97F4A7C15ull, 0u, pi));
    GESMC_TRY(launch(c, s, KID_MISC, 0, k_zero_words, dim3(1), dim3(64), 0, c->err, (uint64_t)64));
    GESMC_TRY(launch(c, s, KID_GEN, n, k_invert_perm, dim3(grid_stride_blocks(c, n)), dim3(kBlock), 0,
                     (const uint32_t *)pi, n, sigma));
    if (m > 0)
        GESMC_TRY(launch(c, s, KID_GEN, m, k_relabel, dim3(grid_stride_blocks(c, m)), dim3(kBlock), 0,
                         (unsigned long long *)d_edges, m, (const uint32_t *)sigma, n, c->err));
    GESMC_TRY(check_hip(hipMemcpyAsync(c->h_err, c->err, 4, hipMemcpyDeviceToHost, s), "hipMemcpyAsync"));
    GESMC_TRY(gen_sync(c, s));
    if (*c->h_err & ERR_RANGE) {
        set_error("an edge has a vertex id >= n");
        return GESMC_E_RANGE;
    }
    return map_err(*c->h_err);
}

}  // namespace

extern "C" {

gesmc_status gesmc_gen_gnp(gesmc_ctx *ctx, void *stream, uint32_t n, double p, uint64_t seed, uint64_t *d_out,
                           uint64_t cap, uint64_t *m) {
    return gen_gnp_impl(ctx, stream, n, p, seed, d_out, cap, m);
}

gesmc_status gesmc_gen_pld_degrees(gesmc_ctx *ctx, void *stream, uint32_t n, double gamma, uint32_t dmin,
                                   uint32_t dmax, uint64_t seed, uint32_t *d_deg, uint64_t *sum) {
    return gen_pld_impl(ctx, stream, n, gamma, dmin, dmax, seed, d_deg, sum);
}

gesmc_status gesmc_gen_havel_hakimi(gesmc_ctx *ctx, void *stream, uint32_t n, const uint32_t *d_deg,
                                    uint64_t *d_out, uint64_t cap, uint64_t *m) {
    return gen_hh_impl(ctx, stream, n, d_deg, d_out, cap, m);
}

gesmc_status gesmc_gen_relabel(gesmc_ctx *ctx, void *stream, uint64_t *d_edges, uint64_t m, uint32_t n,
                               uint64_t seed) {
    return gen_relabel_impl(ctx, stream, d_edges, m, n, seed);
}

}  // extern "C"

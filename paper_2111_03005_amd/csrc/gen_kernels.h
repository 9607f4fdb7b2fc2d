// Input realisation on gfx950: the steps before the chain that build the
// synthetic inputs of Sec. 6 -- G(n,p) graphs (SynGnp) and Havel-Hakimi
// realisations of i.i.d. power-law degree sequences (SynPld) -- plus the
// vertex relabelling.  The definitions (Philox draws with counter tags 3 and
// 4, the portable ln / exp, the chunk rule of G(n,p), the integer-weight
// inverse CDF, the Havel-Hakimi choice rule) are stated in include/gesmc.h;
// this file holds their kernels.
//
//   G(n,p): one wavefront per chunk of the pair index space.  The chunk's
//     draws are taken 64 at a time, one per lane; an inclusive scan of the
//     skips plus one gives every candidate pair at once, and the candidates
//     below the chunk end are the chunk's edges (the sequential walk stops
//     at the first candidate past the end, and candidates only grow).  A
//     counting pass, a scan of the chunk counts, then a writing pass whose
//     stores are coalesced runs of edges.
//   Degrees: the integer CDF by a scan of per-value weights, then one draw
//     per vertex and a binary search in the CDF.
//   Havel-Hakimi: the vertices are placed by (degree descending, id
//     ascending) with a stable counting sort.  The residual degrees then
//     stay sorted along the positions for the whole construction (taking the
//     partners of largest (residual, position) decrements a prefix and the
//     tail of the boundary run), so the state is only E[y] = the end of the
//     positions with residual >= y.  One wavefront runs the steps: E in LDS
//     while the largest residual exceeds 64, then in one register per lane.
//     Each step logs its partner ranges; a parallel pass writes the edges.
#pragma once

#include "device_common.h"

namespace gesmc {

// ---------------------------------------------------------------------------
// Portable ln / exp: correctly rounded IEEE double steps only, in a fixed
// order, never fused, so every implementation of the same steps agrees to
// the bit (see include/gesmc.h for the definition).
// ---------------------------------------------------------------------------
constexpr double kGenLn2Hi = 6.93147180369123816490e-01;  // fdlibm's split of ln 2
constexpr double kGenLn2Lo = 1.90821492927058770002e-10;

__device__ __forceinline__ double gen_ln(double x) {
#pragma clang fp contract(off)
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    int e = (int)((b >> 52) & 0x7FF) - 1023;
    double m = __longlong_as_double((long long)((b & 0xFFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
    if (m > 1.4142135623730951) {
        m = m * 0.5;
        e += 1;
    }
    const double f = m - 1.0;
    const double s = f / (2.0 + f);
    const double z = s * s;
    // 2 atanh(s) = 2s (1 + z/3 + z^2/5 + ... + z^11/23), Horner from the top
    double P = 1.0 / 23.0;
    P = P * z + 1.0 / 21.0;
    P = P * z + 1.0 / 19.0;
    P = P * z + 1.0 / 17.0;
    P = P * z + 1.0 / 15.0;
    P = P * z + 1.0 / 13.0;
    P = P * z + 1.0 / 11.0;
    P = P * z + 1.0 / 9.0;
    P = P * z + 1.0 / 7.0;
    P = P * z + 1.0 / 5.0;
    P = P * z + 1.0 / 3.0;
    const double t = 2.0 * s;
    const double lnm = t + t * (z * P);
    const double ed = (double)e;
    return ed * kGenLn2Hi + (ed * kGenLn2Lo + lnm);
}

__device__ __forceinline__ double gen_exp(double x) {  // -700 <= x <= 0
#pragma clang fp contract(off)
    const double kd = floor(x * 1.4426950408889634 + 0.5);
    const int k = (int)kd;
    const double r = (x - kd * kGenLn2Hi) - kd * kGenLn2Lo;
    // sum of r^j / j!, j = 0 .. 13, Horner from the top
    double p = 1.0 / 6227020800.0;
    p = p * r + 1.0 / 479001600.0;
    p = p * r + 1.0 / 39916800.0;
    p = p * r + 1.0 / 3628800.0;
    p = p * r + 1.0 / 362880.0;
    p = p * r + 1.0 / 40320.0;
    p = p * r + 1.0 / 5040.0;
    p = p * r + 1.0 / 720.0;
    p = p * r + 1.0 / 120.0;
    p = p * r + 1.0 / 24.0;
    p = p * r + 1.0 / 6.0;
    p = p * r + 1.0 / 2.0;
    p = p * r + 1.0;
    p = p * r + 1.0;
    return p * __longlong_as_double((long long)((uint64_t)(k + 1023) << 52));
}

// ---------------------------------------------------------------------------
// Scans (u64, exclusive, in place) for the count arrays: per-block sums,
// a one-block scan of the sums, then the blocks add their offsets.
// ---------------------------------------------------------------------------
constexpr uint32_t kGenScanBlock = 1024;
constexpr uint32_t kGenScanItems = 8;  // items per thread: 8192 per block

__device__ __forceinline__ unsigned long long block_excl_scan_u64(unsigned long long v, unsigned long long *sh,
                                                                  unsigned long long *total) {
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wid = tid >> 6;
    unsigned long long x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long y = __shfl_up(x, o, 64);
        if ((int)lane >= o) x += y;
    }
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    if (wid == 0) {
        unsigned long long w = lane < (blockDim.x >> 6) ? sh[lane] : 0ull;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned long long y = __shfl_up(w, o, 64);
            if ((int)lane >= o) w += y;
        }
        if (lane < (blockDim.x >> 6)) sh[lane] = w;
    }
    __syncthreads();
    const unsigned long long before = (wid ? sh[wid - 1] : 0ull) + x - v;
    if (total) *total = sh[(blockDim.x >> 6) - 1];
    __syncthreads();
    return before;
}

template <typename T>
__global__ __launch_bounds__(kGenScanBlock) void k_gen_block_sums(const T *__restrict__ a, uint64_t n,
                                                                   unsigned long long *__restrict__ sums) {
    __shared__ unsigned long long sh[16];
    const uint64_t base = (uint64_t)blockIdx.x * kGenScanBlock * kGenScanItems + threadIdx.x * kGenScanItems;
    unsigned long long s = 0;
#pragma unroll
    for (uint32_t j = 0; j < kGenScanItems; ++j)
        if (base + j < n) s += a[base + j];
    unsigned long long tot;
    block_excl_scan_u64(s, sh, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// One block: exclusive scan of nb block sums in place; the grand total to *total.
__global__ __launch_bounds__(kGenScanBlock) void k_gen_scan_sums(unsigned long long *__restrict__ sums, uint32_t nb,
                                                                 unsigned long long *__restrict__ total) {
    __shared__ unsigned long long sh[16];
    unsigned long long carry = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += kGenScanBlock) {
        const uint32_t i = b0 + threadIdx.x;
        const unsigned long long v = i < nb ? sums[i] : 0ull;
        unsigned long long tot;
        const unsigned long long ex = block_excl_scan_u64(v, sh, &tot);
        if (i < nb) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

// Exclusive scan of a into out (u64) with the block offsets.
template <typename T>
__global__ __launch_bounds__(kGenScanBlock) void k_gen_scan_apply(const T *__restrict__ a, uint64_t n,
                                                                  const unsigned long long *__restrict__ sums,
                                                                  unsigned long long *__restrict__ out) {
    __shared__ unsigned long long sh[16];
    const uint64_t base = (uint64_t)blockIdx.x * kGenScanBlock * kGenScanItems + threadIdx.x * kGenScanItems;
    T v[kGenScanItems];
    unsigned long long s = 0;
#pragma unroll
    for (uint32_t j = 0; j < kGenScanItems; ++j) {
        v[j] = base + j < n ? a[base + j] : (T)0;
        s += v[j];
    }
    unsigned long long run = sums[blockIdx.x] + block_excl_scan_u64(s, sh, nullptr);
#pragma unroll
    for (uint32_t j = 0; j < kGenScanItems; ++j) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
}

// ---------------------------------------------------------------------------
// G(n,p)
// ---------------------------------------------------------------------------
// Pair index q -> (w, v), q = v (v - 1) / 2 + w, w < v: a floating estimate
// corrected exactly in integers.
__device__ __forceinline__ unsigned long long gen_pair_key(uint64_t q) {
    uint64_t v = (uint64_t)((1.0 + sqrt(1.0 + 8.0 * (double)q)) * 0.5);
    while (v > 0 && v * (v - 1) / 2 > q) --v;
    while ((v + 1) * v / 2 <= q) ++v;
    const uint64_t w = q - v * (v - 1) / 2;
    return (w << 32) | v;
}

// Inclusive wave scan of 64-bit values.
__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t x, uint32_t lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(x, o, 64);
        if ((int)lane >= o) x += y;
    }
    return x;
}

constexpr uint32_t kGnpBlock = 256;                  // four wavefronts, one chunk each at a time
constexpr uint64_t kGnpSkipCap = 1ull << 41;         // skips at or above any chunk length end it

// The edges of chunk j, 64 draws at a time.  kWrite = false: returns the
// count; kWrite = true: writes them from out[first].
template <bool kWrite>
__device__ __forceinline__ uint32_t gnp_chunk_edges(uint64_t j, uint64_t L, uint64_t N, double lq, uint32_t k0,
                                                    uint32_t k1, unsigned long long *out, uint64_t first) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t end = min(j * L + L, N);
    uint64_t c = j * L;
    uint32_t cnt = 0;
    for (uint32_t t0 = 0;; t0 += 64) {
        const Philox4 x = philox4x32_10((uint32_t)j, (uint32_t)(j >> 32), t0 + lane, 3u, k0, k1);
        const uint64_t R = ((uint64_t)x.x0 << 32) | x.x1;
        const double U = (double)((R >> 11) + 1) * 0x1.0p-53;
        const double G = gen_ln(U) / lq;
        const uint64_t g = G < (double)kGnpSkipCap ? (uint64_t)G : kGnpSkipCap;
        // candidate of draw t: c + sum over earlier draws of (skip + 1) + skip
        const uint64_t inc = wave_incl_scan_u64(g + 1, lane);
        const uint64_t q = c + inc - 1;
        const bool ok = q < end;
        const uint64_t mask = __ballot(ok);
        if (kWrite && ok) out[first + cnt + lane] = gen_pair_key(q);
        const uint32_t got = (uint32_t)__popcll(mask);
        cnt += got;
        if (got < 64) break;
        c = __shfl(q, 63, 64) + 1;
        if (c >= end) break;
    }
    return cnt;
}

// q1p = 1 - p; ln(1 - p) is taken here with the draws' own steps.
__global__ __launch_bounds__(kGnpBlock) void k_gnp_count(uint64_t nchunks, uint64_t L, uint64_t N, double q1p,
                                                         uint32_t k0, uint32_t k1, uint32_t *__restrict__ counts) {
    const double lq = gen_ln(q1p);
    const uint64_t waves = (uint64_t)gridDim.x * (kGnpBlock / 64);
    for (uint64_t j = (uint64_t)blockIdx.x * (kGnpBlock / 64) + (threadIdx.x >> 6); j < nchunks; j += waves) {
        const uint32_t c = gnp_chunk_edges<false>(j, L, N, lq, k0, k1, nullptr, 0);
        if ((threadIdx.x & 63u) == 0) counts[j] = c;
    }
}

__global__ __launch_bounds__(kGnpBlock) void k_gnp_write(uint64_t nchunks, uint64_t L, uint64_t N, double q1p,
                                                         uint32_t k0, uint32_t k1,
                                                         const unsigned long long *__restrict__ offs,
                                                         unsigned long long *__restrict__ out) {
    const double lq = gen_ln(q1p);
    const uint64_t waves = (uint64_t)gridDim.x * (kGnpBlock / 64);
    for (uint64_t j = (uint64_t)blockIdx.x * (kGnpBlock / 64) + (threadIdx.x >> 6); j < nchunks; j += waves)
        gnp_chunk_edges<true>(j, L, N, lq, k0, k1, out, offs[j]);
}

// p >= 1: every pair, in pair order.
__global__ __launch_bounds__(kBlock) void k_gnp_complete(uint64_t N, unsigned long long *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t q = (uint64_t)blockIdx.x * kBlock + threadIdx.x; q < N; q += stride) out[q] = gen_pair_key(q);
}

// ---------------------------------------------------------------------------
// Power-law degrees
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_pld_weights(uint32_t nv, uint32_t dmin, double gamma,
                                                        unsigned long long *__restrict__ W) {
#pragma clang fp contract(off)
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= nv) return;
    const double l0 = gen_ln((double)dmin);
    const double a = gen_ln((double)(dmin + i)) - l0;
    const double x = -(gamma * a);
    W[i] = (unsigned long long)(gen_exp(x) * 0x1.0p43);
}

// C[i] = exclusive prefix of W plus W[i] (the inclusive CDF).
__global__ __launch_bounds__(kBlock) void k_pld_cdf(const unsigned long long *__restrict__ W, uint32_t nv,
                                                    unsigned long long *__restrict__ C) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < nv) C[i] += W[i];
}

__device__ __forceinline__ uint32_t pld_draw(uint32_t v, uint32_t r, const unsigned long long *C, uint32_t nv,
                                             uint32_t dmin, uint32_t k0, uint32_t k1) {
    const Philox4 x = philox4x32_10(v, r, 0u, 4u, k0, k1);
    const uint64_t R = ((uint64_t)x.x0 << 32) | x.x1;
    const uint64_t u = __umul64hi(R, C[nv - 1]);
    uint32_t lo = 0, hi = nv - 1;  // smallest i with C[i] > u (C[nv-1] > u always)
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (C[mid] > u)
            hi = mid;
        else
            lo = mid + 1;
    }
    return dmin + lo;
}

__global__ __launch_bounds__(kBlock) void k_pld_draw(uint32_t n, const unsigned long long *__restrict__ C,
                                                     uint32_t nv, uint32_t dmin, uint32_t k0, uint32_t k1,
                                                     uint32_t *__restrict__ deg, unsigned long long *__restrict__ sum) {
    __shared__ unsigned long long bs;
    if (threadIdx.x == 0) bs = 0;
    __syncthreads();
    unsigned long long s = 0;
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t v = blockIdx.x * kBlock + threadIdx.x; v < n; v += stride) {
        const uint32_t d = pld_draw(v, 0u, C, nv, dmin, k0, k1);
        deg[v] = d;
        s += d;
    }
    atomicAdd(&bs, s);
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(sum, bs);
}

// One thread: redraws of vertex 0 until the sum is even (info[0] = redraws,
// info[1] = 1 on failure).
__global__ void k_pld_even(const unsigned long long *__restrict__ C, uint32_t nv, uint32_t dmin, uint32_t dmax,
                           uint32_t k0, uint32_t k1, uint32_t *__restrict__ deg, unsigned long long *__restrict__ sum,
                           uint32_t *__restrict__ info) {
    if (threadIdx.x != 0) return;
    unsigned long long s = *sum;
    uint32_t r = 0, fail = 0;
    while (s & 1ull) {
        if (dmin == dmax || r == 65535u) {
            fail = 1;
            break;
        }
        ++r;
        s -= deg[0];
        deg[0] = pld_draw(0u, r, C, nv, dmin, k0, k1);
        s += deg[0];
    }
    *sum = s;
    info[0] = r;
    info[1] = fail;
}

// ---------------------------------------------------------------------------
// Havel-Hakimi
// ---------------------------------------------------------------------------
// Degree statistics: max (words[0]) and sum (words[1..2] as u64).
__global__ __launch_bounds__(kBlock) void k_hh_stats(const uint32_t *__restrict__ deg, uint32_t n,
                                                     uint32_t *__restrict__ dmax,
                                                     unsigned long long *__restrict__ sum) {
    uint32_t mx = 0;
    unsigned long long s = 0;
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t v = blockIdx.x * kBlock + threadIdx.x; v < n; v += stride) {
        const uint32_t d = deg[v];
        mx = max(mx, d);
        s += d;
    }
    for (int o = 32; o > 0; o >>= 1) {
        mx = max(mx, (uint32_t)__shfl_down(mx, o, 64));
        s += __shfl_down(s, o, 64);
    }
    if ((threadIdx.x & 63u) == 0) {
        atomicMax(dmax, mx);
        atomicAdd(sum, s);
    }
}

// Per-range degree histograms: range b = ids [b T, (b+1) T) -> M[(D - d) nb + b]
// (the layout in which one exclusive scan gives every (degree, range) its
// first position under the order (degree descending, id ascending)).
constexpr uint32_t kHhMaxDeg = 16000;  // largest degree of the LDS-resident state (64 KB)

__global__ __launch_bounds__(kBlock) void k_hh_hist(const uint32_t *__restrict__ deg, uint32_t n, uint32_t T,
                                                    uint32_t D, uint32_t nb, uint32_t *__restrict__ M) {
    extern __shared__ uint32_t hh_h[];
    for (uint32_t d = threadIdx.x; d <= D; d += kBlock) hh_h[d] = 0;
    __syncthreads();
    const uint32_t b = blockIdx.x;
    const uint64_t lo = (uint64_t)b * T, hi = min<uint64_t>(lo + T, n);
    for (uint64_t v = lo + threadIdx.x; v < hi; v += kBlock) atomicAdd(&hh_h[deg[v]], 1u);
    __syncthreads();
    for (uint32_t d = threadIdx.x; d <= D; d += kBlock) M[(size_t)(D - d) * nb + b] = hh_h[d];
}

// Places the ids of range b at their positions: one wavefront walks the
// range in id order, 64 ids a round; a lane's position is its degree's
// running offset plus the number of earlier lanes of the round with the
// same degree.
__global__ __launch_bounds__(64) void k_hh_place(const uint32_t *__restrict__ deg, uint32_t n, uint32_t T,
                                                 uint32_t D, uint32_t nb, const unsigned long long *__restrict__ Moff,
                                                 uint32_t *__restrict__ O) {
    extern __shared__ uint32_t hh_c[];
    const uint32_t b = blockIdx.x, lane = threadIdx.x;
    for (uint32_t d = lane; d <= D; d += 64) hh_c[d] = (uint32_t)Moff[(size_t)(D - d) * nb + b];
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    const uint64_t lo = (uint64_t)b * T, hi = min<uint64_t>(lo + T, n);
    for (uint64_t v0 = lo; v0 < hi; v0 += 64) {
        const uint64_t v = v0 + lane;
        const bool in = v < hi;
        const uint32_t d = in ? deg[v] : 0xFFFFFFFFu;
        uint32_t rank = 0, after = 0;
        for (uint32_t j = 0; j < 64; ++j) {
            const uint32_t dj = __shfl(d, j, 64);
            rank += (j < lane && dj == d) ? 1u : 0u;
            after += (j > lane && dj == d) ? 1u : 0u;
        }
        uint32_t base = 0;
        if (in) base = hh_c[d];
        __builtin_amdgcn_wave_barrier();
        if (in && base + rank < n) {
            O[base + rank] = (uint32_t)v;
            if (after == 0) hh_c[d] = base + rank + 1;  // the last lane of its degree in this round
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Step log of Havel-Hakimi: step s (position s) joins position s to the
// positions [s + 1, a) and [b - k, b); its edges start at off.
struct HhStep {
    uint32_t a, b, k, off;
};

// E[y] (y = 1 .. D) from the scanned histograms: the first position of
// degree y - 1, i.e. the number of positions of degree >= y; E[D+1] = 0.
__global__ __launch_bounds__(kBlock) void k_hh_bounds(const unsigned long long *__restrict__ Moff, uint32_t D,
                                                      uint32_t nb, uint32_t *__restrict__ E) {
    const uint32_t y = blockIdx.x * kBlock + threadIdx.x;
    if (y == 0 || y > D + 1) return;
    E[y] = y > D ? 0u : (uint32_t)Moff[(size_t)(D - (y - 1)) * nb];
}

// The steps, one wavefront.  E (D + 2 words, from k_hh_bounds) is copied to
// LDS; status[0] = steps taken, status[1] = 1 if not graphical (2: an
// inconsistent state, an internal error).
__global__ __launch_bounds__(64) void k_hh_steps(const uint32_t *__restrict__ E0, uint32_t D, uint32_t n,
                                                 HhStep *__restrict__ log, uint32_t *__restrict__ status) {
    extern __shared__ uint32_t E[];
    const uint32_t lane = threadIdx.x;
    const uint32_t ylast = max(D, 64u) + 1;  // lanes of the register phase read E[1 .. 64]
    for (uint32_t y = lane; y <= ylast; y += 64) E[y] = y == 0 ? 0xFFFFFFFFu : (y <= D + 1 ? E0[y] : 0u);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    uint32_t s = 0, off = 0, dcur = D, fail = 0;
    HhStep mine{0, 0, 0, 0};  // the step (s & 63) == lane of the current group
    auto flush = [&](uint32_t upto) {  // writes the log entries of steps [upto & ~63, upto)
        const uint32_t g = (upto - 1) & ~63u;
        if (g + lane < upto) log[g + lane] = mine;
    };
    // ---- steps while the largest residual exceeds 64: E in LDS ----
    // (a positive residual at position s means s < E[1] <= n; the checks on
    // s keep a corrupt state from writing past the log)
    while (dcur > 64) {
        if (s >= n) {
            fail = 2;
            break;
        }
        // d = the largest y <= dcur with E[y] > s
        uint32_t d = 0;
        for (uint32_t top = dcur; top >= 1;) {
            const uint32_t y = top >= lane ? top - lane : 0u;
            const bool ok = y >= 1 && E[y] > s;
            const uint64_t bal = __ballot(ok);
            if (bal) {
                d = top - (uint32_t)__ffsll((long long)bal) + 1;
                break;
            }
            top = top > 64 ? top - 64 : 0;
        }
        dcur = d;
        if (d <= 64) break;  // the register phase takes this step
        if (E[1] <= s + d) {  // fewer than d other positions of positive residual
            fail = 1;
            break;
        }
        // x = the largest y <= d with E[y] > s + d (E[1] > s + d holds)
        uint32_t lo = 1, hi = d;
        while (hi > lo) {
            const uint32_t st = (hi - lo + 64) / 64;
            const uint32_t y = lo + lane * st;
            const bool ok = y <= hi && E[y] > s + d;
            const uint64_t bal = __ballot(ok);
            const uint32_t top = 63u - (uint32_t)__clzll((long long)bal);
            lo = lo + top * st;
            hi = min(hi, lo + st - 1);
        }
        const uint32_t x = lo;
        const uint32_t a = max(E[x + 1], s + 1), b = E[x], k = s + d + 1 - a;
        // E[y] <- max(E[y + 1], s + 1) for x < y <= d, in rising chunks
        for (uint32_t y0 = x + 1; y0 <= d; y0 += 64) {
            const uint32_t y = y0 + lane;
            const uint32_t nv = y <= d ? max(E[y + 1], s + 1) : 0u;
            __builtin_amdgcn_wave_barrier();
            if (y <= d) E[y] = nv;
            __builtin_amdgcn_wave_barrier();
        }
        if (lane == 0) E[x] = b - k;
        __builtin_amdgcn_wave_barrier();
        if (lane == (s & 63u)) mine = HhStep{a, b, k, off};
        off += d;
        ++s;
        if ((s & 63u) == 0) flush(s);
    }
    // ---- the rest: lane l holds E[l + 1] ----
    if (!fail && dcur > 0) {
        uint32_t e = E[lane + 1];
        for (;;) {
            const uint32_t d = (uint32_t)__popcll(__ballot(e > s));
            if (d == 0) break;
            if (s >= n) {
                fail = 2;
                break;
            }
            const uint32_t x = (uint32_t)__popcll(__ballot(e > s + d));
            if (x == 0) {
                fail = 1;
                break;
            }
            // x and d are uniform: single-lane reads; E[x + 1] is lane x's
            const uint32_t ex1 = x < 64 ? (uint32_t)__builtin_amdgcn_readlane((int)e, (int)x) : 0u;
            const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)e, (int)(x - 1));  // E[x]
            const uint32_t a = max(ex1, s + 1), k = s + d + 1 - a;
            // E[y + 1] from the next lane: DPP wave_shl:1 (lane i reads lane
            // i + 1; every lane active), lane 63 takes E[65] = empty
            const uint32_t down = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)e, 0x130, 0xF, 0xF, false);
            const uint32_t nxt = lane < 63 ? down : 0u;
            const uint32_t y = lane + 1;
            if (y > x && y <= d)
                e = max(nxt, s + 1);
            else if (y == x)
                e = b - k;
            if (lane == (s & 63u)) mine = HhStep{a, b, k, off};
            off += d;
            ++s;
            if ((s & 63u) == 0) flush(s);
        }
    }
    if (s & 63u) flush(s);
    if (lane == 0) {
        status[0] = s;
        status[1] = fail;
    }
}

// The edges of the logged steps: block w takes steps [w 256, w 256 + 256),
// whose edges are contiguous; each thread finds its step in the staged
// offsets.  Edge keys (min id << 32) | max id.
constexpr uint32_t kHhEmitSteps = 256;

__global__ __launch_bounds__(kBlock) void k_hh_emit(const HhStep *__restrict__ log, uint32_t S, uint32_t m,
                                                    const uint32_t *__restrict__ O, uint32_t n,
                                                    unsigned long long *__restrict__ out) {
    __shared__ uint32_t offs[kHhEmitSteps + 1];
    __shared__ HhStep st[kHhEmitSteps];
    const uint32_t s0 = blockIdx.x * kHhEmitSteps;
    const uint32_t ns = min(kHhEmitSteps, S - s0);
    for (uint32_t i = threadIdx.x; i < ns; i += kBlock) {
        st[i] = log[s0 + i];
        offs[i] = st[i].off;
    }
    if (threadIdx.x == 0) offs[ns] = s0 + ns < S ? log[s0 + ns].off : m;
    __syncthreads();
    const uint32_t e0 = offs[0], e1 = offs[ns];
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
        uint32_t lo = 0, hi = ns - 1;  // the last step whose offset is <= e
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (offs[mid] <= e)
                lo = mid;
            else
                hi = mid - 1;
        }
        const HhStep t = st[lo];
        const uint32_t s = s0 + lo, i = e - t.off, pre = t.a - s - 1;
        const uint32_t p = i < pre ? s + 1 + i : t.b - t.k + (i - pre);
        if (p >= n || e >= m) continue;  // never for a consistent log
        const uint32_t u = O[s], v = O[p];
        out[e] = u < v ? ((unsigned long long)u << 32) | v : ((unsigned long long)v << 32) | u;
    }
}

// ---------------------------------------------------------------------------
// Relabel: sigma[pi[r]] = r, then every key rewritten and made canonical.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_invert_perm(const uint32_t *__restrict__ pi, uint32_t n,
                                                        uint32_t *__restrict__ sigma) {
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t r = blockIdx.x * kBlock + threadIdx.x; r < n; r += stride) sigma[pi[r]] = r;
}

__global__ __launch_bounds__(kBlock) void k_relabel(unsigned long long *__restrict__ E, uint64_t m,
                                                    const uint32_t *__restrict__ sigma, uint32_t n,
                                                    uint32_t *__restrict__ err) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    uint32_t f = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        const unsigned long long e = E[i];
        const uint32_t a = (uint32_t)(e >> 32), b = (uint32_t)e;
        if (a >= n || b >= n) {
            f = ERR_RANGE;
            continue;
        }
        const uint32_t x = sigma[a], y = sigma[b];
        E[i] = x < y ? ((unsigned long long)x << 32) | y : ((unsigned long long)y << 32) | x;
    }
    if (f) atomicOr(err, f);
}

}  // namespace gesmc

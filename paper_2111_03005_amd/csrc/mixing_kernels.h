// Mixing diagnostic of Sec. 6.1 on gfx950: the autocorrelation analysis of
// a chain's edge series, aggregated on the fly for a set of thinning values.
//
// Every possible edge {u, v}, u < v < n, has a pair id
//   pid(u, v) = u n - u (u + 1) / 2 + (v - u - 1)
// in [0, n (n - 1) / 2).  For each thinning value k the device keeps, per
// pair, the counts of the k-thinned series' transitions 0 -> 1, 1 -> 0 and
// 1 -> 1 (0 -> 0 follows from the number of transitions N), a bitmap of the
// pairs present in the last sample, that sample's edge list, and a bitmap of
// the pairs present in any sample (the edges tracked).  A sample costs O(m)
// integer work; the final pass runs over all pairs: G^2 of each tracked
// pair's 2x2 table in float64 and the rule of the Bayesian information
// criterion (not independent iff G^2 > ln N).
#pragma once

#include "device_common.h"

namespace gesmc {

struct MixCount {
    uint32_t n01, n10, n11;
};

__device__ __forceinline__ uint32_t mix_pid(unsigned long long e, uint32_t n) {
    const uint32_t u = (uint32_t)(e >> 32), v = (uint32_t)e;
    return u * n - (uint32_t)(((uint64_t)u * (u + 1)) >> 1) + (v - u - 1);
}

__device__ __forceinline__ bool mix_bit(const uint32_t *bits, uint32_t pid) {
    return (bits[pid >> 5] >> (pid & 31u)) & 1u;
}

// Sets (set = true) or clears the bits of the m edges of E.
__global__ __launch_bounds__(kBlock) void k_mix_bits(const unsigned long long *__restrict__ E, uint32_t m,
                                                     uint32_t n, uint32_t *__restrict__ bits, bool set) {
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        const uint32_t pid = mix_pid(E[i], n);
        if (set)
            atomicOr(&bits[pid >> 5], 1u << (pid & 31u));
        else
            atomicAnd(&bits[pid >> 5], ~(1u << (pid & 31u)));
    }
}

// One sample of a thinned series (not the first): each edge present now
// counts a 1 -> 1 or 0 -> 1 transition and joins the tracked set; each edge
// of the previous sample that is gone counts 1 -> 0.  The graph is simple,
// so every pair has one writer per counter.
__global__ __launch_bounds__(kBlock) void k_mix_count(const unsigned long long *__restrict__ E,
                                                      const unsigned long long *__restrict__ prev, uint32_t m,
                                                      uint32_t n, const uint32_t *__restrict__ cur_bits,
                                                      const uint32_t *__restrict__ prev_bits,
                                                      MixCount *__restrict__ cnt, uint32_t *__restrict__ ever) {
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        const uint32_t pid = mix_pid(E[i], n);
        if (mix_bit(prev_bits, pid))
            cnt[pid].n11 += 1;
        else
            cnt[pid].n01 += 1;
        atomicOr(&ever[pid >> 5], 1u << (pid & 31u));
        const uint32_t pq = mix_pid(prev[i], n);
        if (!mix_bit(cur_bits, pq)) cnt[pq].n10 += 1;
    }
}

// Totals of one thinning value: edges tracked, edges not independent, and
// the transition counts summed over tracked edges (out: 6 words, zeroed by
// the host).  N transitions per tracked edge.
__global__ __launch_bounds__(kBlock) void k_mix_decide(const MixCount *__restrict__ cnt,
                                                       const uint32_t *__restrict__ ever, uint64_t npairs,
                                                       uint32_t N, unsigned long long *__restrict__ out) {
    __shared__ unsigned long long acc[6];
    if (threadIdx.x < 6) acc[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long tracked = 0, flagged = 0, s01 = 0, s10 = 0, s11 = 0;
    const double lnN = log((double)N);
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x; p < npairs; p += stride) {
        if (!((ever[p >> 5] >> (p & 31u)) & 1u)) continue;
        const MixCount c = cnt[p];
        const double n01 = c.n01, n10 = c.n10, n11 = c.n11, n00 = (double)N - n01 - n10 - n11;
        const double r0 = n00 + n01, r1 = n10 + n11, c0 = n00 + n10, c1 = n01 + n11, NN = (double)N;
        double g = 0.0;
        if (n00 > 0) g += n00 * log(n00 * NN / (r0 * c0));
        if (n01 > 0) g += n01 * log(n01 * NN / (r0 * c1));
        if (n10 > 0) g += n10 * log(n10 * NN / (r1 * c0));
        if (n11 > 0) g += n11 * log(n11 * NN / (r1 * c1));
        g *= 2.0;
        ++tracked;
        flagged += g > lnN;
        s01 += c.n01;
        s10 += c.n10;
        s11 += c.n11;
    }
    if (tracked) {
        atomicAdd(&acc[0], tracked);
        atomicAdd(&acc[1], flagged);
        atomicAdd(&acc[2], s01);
        atomicAdd(&acc[3], s10);
        atomicAdd(&acc[4], s11);
    }
    __syncthreads();
    if (threadIdx.x < 5 && acc[threadIdx.x]) atomicAdd(&out[threadIdx.x], acc[threadIdx.x]);
}

}  // namespace gesmc

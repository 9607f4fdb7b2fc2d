// Kernels of the batched form: G independent graphs run as one disjoint
// union (layout and numbering in device_common.h, BatchGraph).  The per
// superstep kernels are those of the single graph; these kernels load the
// graphs into their segments, map positions to graphs, count outcomes per
// graph and write every graph's result back in its input order.
#pragma once

#include "device_common.h"

namespace gesmc {

// Largest g < ng with key(g) <= x for a non-decreasing key (binary search).
template <typename KeyOf>
__device__ __forceinline__ uint32_t upper_index(uint32_t ng, uint64_t x, KeyOf key) {
    uint32_t lo = 0, hi = ng - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (key(mid) <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Input edge i of graph g (in the caller's graph order, in_off = input
// offsets, G + 1 words) -> record (i, shifted canonical key) at position
// poff + (i - goff) of its segment; also the padding record of an odd graph
// that is switched.  Flags loops (ERR_LOOP) and ids >= n (ERR_RANGE), and
// keeps the smallest failing input position in *bad_pos (as its complement,
// with atomicMax, so that 0 means none).
__global__ __launch_bounds__(kBlock) void k_load_batch(const unsigned long long *__restrict__ in, uint32_t total,
                                                       const uint64_t *__restrict__ in_off, uint32_t G,
                                                       const uint32_t *__restrict__ rank_of,
                                                       const BatchGraph *__restrict__ gr, uint32_t *__restrict__ idx,
                                                       unsigned long long *__restrict__ key,
                                                       uint32_t *__restrict__ err, uint32_t *__restrict__ bad_pos,
                                                       uint32_t *__restrict__ gerr) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    uint32_t f = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += stride) {
        const uint32_t g = upper_index(G, i, [&](uint32_t x) { return in_off[x]; });  // skips empty graphs
        const BatchGraph b = gr[rank_of[g]];
        const unsigned long long e = in[i];
        const uint32_t u = (uint32_t)(e >> 32), v = (uint32_t)e;
        uint32_t fe = 0;
        if (u == v) fe |= ERR_LOOP;
        if (u >= b.n || v >= b.n) fe |= ERR_RANGE;
        const uint32_t p = b.poff + ((uint32_t)i - b.goff);
        idx[p] = (uint32_t)i;
        key[p] = fe ? kEmptyKey : ekey(u + b.vbase, v + b.vbase);
        if (fe) {
            f |= fe;
            atomicMax(bad_pos, ~(uint32_t)i);
            atomicOr(&gerr[rank_of[g]], fe);
        }
        if ((uint32_t)i == b.goff && b.mpad > b.m) {  // padding record of an odd switched graph
            idx[b.poff + b.m] = kPadIdx;
            key[b.poff + b.m] = kEmptyKey;
        }
    }
    if (f) atomicOr(err, f);
}

// pg[p] = rank of the graph whose segment holds position p (p < total).
__global__ __launch_bounds__(kBlock) void k_fill_pg(const BatchGraph *__restrict__ gr, uint32_t ngraphs,
                                                    uint32_t total, uint32_t *__restrict__ pg) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x; p < total; p += stride)
        pg[p] = upper_index(ngraphs, p, [&](uint32_t x) { return (uint64_t)gr[x].poff; });
}

// Outcomes of one superstep per graph: acc[4q .. 4q+3] += legal, loop,
// exists, P_L counts of graph q's switches.  Each workgroup takes a chunk of
// kStatsChunk consecutive switches (graphs own contiguous switch ranges), so
// a chunk spans a short run of graphs: counts go to LDS bins per graph of
// the chunk and leave with one device atomic per (graph, outcome) and chunk;
// graphs beyond the bins (many tiny graphs in one chunk) count directly.
constexpr uint32_t kStatsPerThread = 16;
constexpr uint32_t kStatsChunk = kStatsPerThread * kBlock;
constexpr uint32_t kStatsBins = 64;

__global__ __launch_bounds__(kBlock) void k_graph_stats(const uint8_t *__restrict__ st,
                                                        const BatchGraph *__restrict__ gr, uint32_t ngraphs,
                                                        uint32_t ell, unsigned long long *__restrict__ acc) {
    __shared__ uint32_t bins[kStatsBins * 4];
    __shared__ uint32_t s_q0;
    const uint32_t tid = threadIdx.x;
    const uint32_t kb = blockIdx.x * kStatsChunk;
    auto first_switch = [&](uint32_t q) { return (uint64_t)(gr[q].poff >> 1); };
    for (uint32_t j = tid; j < kStatsBins * 4; j += kBlock) bins[j] = 0;
    if (tid == 0) s_q0 = upper_index(ngraphs, kb, first_switch);
    __syncthreads();
    const uint32_t q0 = s_q0;
    const uint32_t k0 = kb + tid * kStatsPerThread;
    const uint32_t k1 = min(k0 + kStatsPerThread, ell);
    if (k0 < k1) {
        uint32_t q = upper_index(ngraphs, k0, first_switch);
        uint32_t qend = (gr[q].poff + gr[q].mpad) >> 1;
        for (uint32_t k = k0; k < k1; ++k) {
            while (k >= qend && q + 1 < ngraphs) {
                ++q;
                qend = (gr[q].poff + gr[q].mpad) >> 1;
            }
            const uint8_t sv = st[k];
            if (sv < ST_LEGAL || sv > ST_PL) continue;
            const uint32_t j = sv - ST_LEGAL;  // legal, loop, exists, P_L
            if (q - q0 < kStatsBins)
                atomicAdd(&bins[(q - q0) * 4 + j], 1u);
            else
                atomicAdd(&acc[4 * (size_t)q + j], 1ull);
        }
    }
    __syncthreads();
    for (uint32_t j = tid; j < kStatsBins * 4; j += kBlock) {
        const uint32_t q = q0 + j / 4;
        if (bins[j] && q < ngraphs) atomicAdd(&acc[4 * (size_t)q + (j & 3)], (unsigned long long)bins[j]);
    }
}

// Record at position p -> out[input position] = key with the graph's vertex
// shift removed.  Skipped entirely if an error flag is set (output untouched).
__global__ __launch_bounds__(kBlock) void k_unpermute_batch(const uint32_t *__restrict__ idx,
                                                            const unsigned long long *__restrict__ key,
                                                            const uint32_t *__restrict__ pg,
                                                            const BatchGraph *__restrict__ gr, uint32_t total,
                                                            unsigned long long *__restrict__ out,
                                                            const uint32_t *__restrict__ err) {
    if (*err) return;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x; p < total; p += stride) {
        const uint32_t i = idx[p];
        if (i == kPadIdx) continue;
        const uint64_t vb = gr[pg[p]].vbase;
        out[i] = key[p] - ((vb << 32) | vb);
    }
}

// Serving: moves the records of the graphs that stay resident from their old
// segments (src) into the new layout (dst), re-shifting vertex ids from the
// old base mv[q].y to the new one.  mv[q].x = old first position, or ~0 for
// a graph that is loaded into the new layout instead.
__global__ __launch_bounds__(kBlock) void k_relayout(const BatchGraph *__restrict__ gr, const uint2 *__restrict__ mv,
                                                     const uint32_t *__restrict__ pg, uint32_t total,
                                                     const uint32_t *__restrict__ src_idx,
                                                     const unsigned long long *__restrict__ src_key,
                                                     uint32_t *__restrict__ dst_idx,
                                                     unsigned long long *__restrict__ dst_key) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x; p < total; p += stride) {
        const uint32_t q = pg[p];
        const uint2 m = mv[q];
        if (m.x == 0xFFFFFFFFu) continue;
        const uint32_t sp = m.x + ((uint32_t)p - gr[q].poff);
        const uint32_t i = src_idx[sp];
        unsigned long long e = src_key[sp];
        if (i != kPadIdx) {
            const uint64_t ob = m.y, nb = gr[q].vbase;
            e = e - ((ob << 32) | ob) + ((nb << 32) | nb);
        }
        dst_idx[p] = i;
        dst_key[p] = e;
    }
}

// Serving: the records of every graph q with rb[q] != ~0 go to
// out[rb[q] + local index] with the vertex shift removed.
__global__ __launch_bounds__(kBlock) void k_extract(const uint32_t *__restrict__ idx,
                                                    const unsigned long long *__restrict__ key,
                                                    const uint32_t *__restrict__ pg,
                                                    const BatchGraph *__restrict__ gr,
                                                    const unsigned long long *__restrict__ rb, uint32_t total,
                                                    unsigned long long *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x; p < total; p += stride) {
        const uint32_t q = pg[p];
        const unsigned long long base = rb[q];
        if (base == ~0ull) continue;
        const uint32_t i = idx[p];
        if (i == kPadIdx) continue;
        const uint64_t vb = gr[q].vbase;
        out[base + (i - gr[q].goff)] = key[p] - ((vb << 32) | vb);
    }
}

}  // namespace gesmc

// Kernels of the batched form: G independent graphs run as one disjoint
// union (layout and numbering in device_common.h, BatchGraph).  The per
// superstep kernels are those of the single graph; these kernels load the
// graphs into their segments, map positions to graphs, count outcomes per
// graph and write every graph's result back in its input order.
#pragma once

#include "device_common.h"
#include "perm_kernels.h"
#include "switch_kernels.h"

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
// Position chunks {rank q, first position, end position, aux}: at most
// kChunkPos positions of one rank's segment each, listed on the host, so a
// workgroup knows its graph without a search.
constexpr uint32_t kChunkPos = 8192;

// pg[p] = rank owning position p, one workgroup per chunk (the chunks of all
// ranks cover every position).
__global__ __launch_bounds__(kBlock) void k_fill_pg(const uint4 *__restrict__ ch, uint32_t *__restrict__ pg) {
    const uint4 c = ch[blockIdx.x];
    for (uint32_t p = c.y + threadIdx.x; p < c.z; p += kBlock) pg[p] = c.x;
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
    static_assert(kStatsPerThread == 16, "one 16-byte load of statuses per thread");
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
    // counts of the run of switches of one graph, kept in registers and
    // flushed when the graph changes (a thread's 16 switches rarely span two)
    uint32_t cnt[4] = {0, 0, 0, 0};
    auto flush = [&](uint32_t q) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!cnt[j]) continue;
            if (q - q0 < kStatsBins)
                atomicAdd(&bins[(q - q0) * 4 + j], cnt[j]);
            else
                atomicAdd(&acc[4 * (size_t)q + j], (unsigned long long)cnt[j]);
            cnt[j] = 0;
        }
    };
    if (k0 < k1) {
        uint8_t sv[kStatsPerThread];
        if (k1 - k0 == kStatsPerThread) {  // k0 is a multiple of 16
            const uint4 v = *reinterpret_cast<const uint4 *>(st + k0);
            __builtin_memcpy(sv, &v, sizeof(v));
        } else {
            for (uint32_t x = 0; x < k1 - k0; ++x) sv[x] = st[k0 + x];
        }
        uint32_t q = upper_index(ngraphs, k0, first_switch);
        uint32_t qend = (gr[q].poff + gr[q].mpad) >> 1;
#pragma unroll
        for (uint32_t x = 0; x < kStatsPerThread; ++x) {
            const uint32_t k = k0 + x;
            if (k >= k1) break;
            if (k >= qend) {
                flush(q);
                while (k >= qend && q + 1 < ngraphs) {
                    ++q;
                    qend = (gr[q].poff + gr[q].mpad) >> 1;
                }
            }
            const uint8_t v = sv[x];
            if (v >= ST_LEGAL && v <= ST_PL) ++cnt[v - ST_LEGAL];  // legal, loop, exists, P_L
        }
        flush(q);
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
// old base mv[q].y to the new one; mv[q].x = old first position.  One
// workgroup per chunk of a staying graph.
__global__ __launch_bounds__(kBlock) void k_relayout(const uint4 *__restrict__ ch, const BatchGraph *__restrict__ gr,
                                                     const uint2 *__restrict__ mv,
                                                     const uint32_t *__restrict__ src_idx,
                                                     const unsigned long long *__restrict__ src_key,
                                                     uint32_t *__restrict__ dst_idx,
                                                     unsigned long long *__restrict__ dst_key) {
    const uint4 c = ch[blockIdx.x];
    const uint2 m = mv[c.x];
    const uint32_t poff = gr[c.x].poff;
    const uint64_t ob = m.y, nb = gr[c.x].vbase;
    const unsigned long long shift = ((nb << 32) | nb) - ((ob << 32) | ob);  // mod 2^64
    for (uint32_t p = c.y + threadIdx.x; p < c.z; p += kBlock) {
        const uint32_t sp = m.x + (p - poff);
        const uint32_t i = src_idx[sp];
        const unsigned long long e = src_key[sp];
        dst_idx[p] = i;
        dst_key[p] = i != kPadIdx ? e + shift : e;
    }
}

// Serving: the records of a finishing graph go to out[base + local index]
// with the vertex shift removed; one workgroup per chunk of such a graph,
// base in the chunk's aux word.
__global__ __launch_bounds__(kBlock) void k_extract(const uint4 *__restrict__ ch, const uint32_t *__restrict__ idx,
                                                    const unsigned long long *__restrict__ key,
                                                    const BatchGraph *__restrict__ gr,
                                                    unsigned long long *__restrict__ out) {
    const uint4 c = ch[blockIdx.x];
    const uint64_t vb = gr[c.x].vbase;
    const uint32_t goff = gr[c.x].goff;
    for (uint32_t p = c.y + threadIdx.x; p < c.z; p += kBlock) {
        const uint32_t i = idx[p];
        if (i == kPadIdx) continue;
        out[(uint64_t)c.w + (i - goff)] = key[p] - ((vb << 32) | vb);
    }
}

// ---------------------------------------------------------------------------
// Small graphs of a batch: one workgroup runs all r global switches of one
// graph inside LDS -- the permutation (LDS counting sort of (K_i, i) on the
// top bits of K, then ranks within cells), the switches' ERASE / INSERT
// tuples grouped by tuple hash, the rounds of decisions of Alg. 1 and the
// writes -- with the same definitions as the multi-kernel path, so the result
// is the same chain.  The records stay in LDS across supersteps.  Two sizes:
// m <= 1024 with 256 threads (39 KB of LDS, several workgroups per CU) and
// m <= 4096 with 1024 threads (158 KB, one per CU); in both each thread holds
// 4 permutation items and 2 switches (9 tuples), and there are four sort
// cells per thread.
// ---------------------------------------------------------------------------
constexpr uint32_t kSmallMax = 1024, kSmallThreads = 256;  // edges, threads
constexpr uint32_t kMidMax = 4096, kMidThreads = 1024;
constexpr uint16_t kSmTagStays = 0x7FFF;  // ERASE tag of a surviving edge; erase tags are k < 0x7FFF
constexpr uint16_t kSmTagInsert = 0x8000; // | (k << 1 | h)
constexpr uint32_t kSmNone = 0xFFFFu, kSmStays = 0xFFFEu;

template <uint32_t kMax, uint32_t kThreads>
struct SmallLds {
    unsigned long long E[kMax];       // edge keys by local index
    unsigned long long sK[2 * kMax];  // sorted permutation keys, then sorted tuple hashes
    uint32_t info[kMax];              // per target 2k+h: eraser << 16 | predecessor
    uint16_t pi[kMax];                // the permutation of this superstep
    uint16_t sT[2 * kMax];            // sorted local index, then sorted tuple tag
    uint32_t cell[4 * kThreads + 1];  // sort cells, four per thread
    uint32_t tmp[kThreads / 64 + 2];
    uint8_t st[kMax / 2];
    uint32_t undecided, flags;
    uint32_t cnt[4];
};
static_assert(kMidMax / 2 < kSmTagStays && 2 * kMidMax <= 0x10000, "small-graph tags are 16 bits");
static_assert(kSmallMax == 4 * kSmallThreads && kMidMax == 4 * kMidThreads, "4 edges per thread");

template <uint32_t kThreads>
constexpr int small_cell_bits() {  // 4 kThreads cells
    return kThreads == 256 ? 10 : kThreads == 512 ? 11 : 12;
}

// Groups up to 2 kMax items by the top cell bits of their word: they sit in
// registers (w[q], g[q] for q < kPer where present[q]); a counting sort puts
// them in cell order into sK / sT, item q at slot[q] of cell cl[q] (cell c
// spans [L.cell[c], L.cell[c + 1])).  Within a cell the order is arbitrary;
// callers read the whole cell.  Returns with a barrier passed.
template <int kPer, uint32_t kMax, uint32_t kThreads>
__device__ __forceinline__ void small_group(SmallLds<kMax, kThreads> &L, const unsigned long long *w,
                                            const uint16_t *g, const bool *present, uint32_t *cl, uint32_t *slot) {
    constexpr int kShift = 64 - small_cell_bits<kThreads>();
    constexpr uint32_t kCells = 4 * kThreads;
    const uint32_t tid = threadIdx.x;
    for (uint32_t c = tid; c < kCells; c += kThreads) L.cell[c] = 0;
    __syncthreads();
    uint32_t rank[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        if (!present[q]) continue;
        cl[q] = (uint32_t)(w[q] >> kShift);
        rank[q] = atomicAdd(&L.cell[cl[q]], 1u);
    }
    __syncthreads();
    const uint32_t total = block_exclusive_scan<kThreads>(L.cell, kCells, L.tmp);
    if (tid == 0) L.cell[kCells] = total;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        if (!present[q]) continue;
        slot[q] = L.cell[cl[q]] + rank[q];
        L.sK[slot[q]] = w[q];
        L.sT[slot[q]] = g[q];
    }
    __syncthreads();
}

// Alg. 1's rule for target 2k+h from its packed record (see judge_target_chain).
template <uint32_t kMax, uint32_t kThreads>
__device__ __forceinline__ int small_judge(const SmallLds<kMax, kThreads> &L, uint32_t rec, uint32_t k) {
    int v = V_OK;
    const uint32_t e = rec >> 16;
    if (e != kSmNone) {
        if (e == kSmStays || e >= k) return V_ILLEGAL;
        const uint8_t se = L.st[e];
        if (se == ST_UNDECIDED)
            v = V_WAIT;
        else if (se != ST_LEGAL)
            return V_ILLEGAL;
    }
    uint32_t p = rec & 0xFFFFu, below = k;
    while (p != kSmNone) {
        const uint32_t pk = p >> 1;
        if (pk >= below) return V_ILLEGAL;
        const uint8_t sp = L.st[pk];
        if (sp == ST_LEGAL) return V_ILLEGAL;
        if (sp == ST_UNDECIDED) return V_WAIT;
        below = pk;
        p = L.info[p] & 0xFFFFu;
    }
    return v;
}

// One workgroup per listed graph (ranks `small[0 .. count)`, r of rank q in
// rv[q], m of every listed graph <= kMax); records of graph q are at
// positions poff + local index of `key`; its outcome counts go to
// acc[4q .. 4q+3] (legal, loop, exists, P_L).
template <uint32_t kMax, uint32_t kThreads>
__global__ __launch_bounds__(kThreads) void k_small_chain(const uint32_t *__restrict__ small,
                                                          const BatchGraph *__restrict__ gr,
                                                          const uint32_t *__restrict__ rv,
                                                          unsigned long long *__restrict__ key,
                                                          unsigned long long *__restrict__ acc,
                                                          uint32_t *__restrict__ gerr, uint32_t *__restrict__ err) {
    __shared__ SmallLds<kMax, kThreads> L;
    const uint32_t tid = threadIdx.x;
    const uint32_t q = small[blockIdx.x];
    const BatchGraph b = gr[q];
    const uint32_t m = b.m, ell = m >> 1, r = rv[q];
    for (uint32_t li = tid; li < m; li += kThreads) L.E[li] = key[b.poff + li];
    if (tid < 4) L.cnt[tid] = 0;
    if (tid == 0) L.flags = 0;
    uint32_t c_legal = 0, c_loop = 0, c_exists = 0, c_pl = 0;
    __syncthreads();
    for (uint32_t s = 0; s < r; ++s) {
        const uint32_t t = b.t0 + s;
        // permutation: sort local indices by (K_i, i)
        {
            unsigned long long w[4];
            uint16_t g[4];
            bool pr[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                const uint32_t li = tid + x * kThreads;
                pr[x] = li < m;
                w[x] = pr[x] ? perm_key(li, t, b.k0, b.k1) : ~0ull;
                g[x] = (uint16_t)li;
            }
            uint32_t cl[4], slot[4];
            small_group<4>(L, w, g, pr, cl, slot);
            // keys (K_i, i) are distinct: an index's place is the number of smaller keys in its cell
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                if (!pr[x]) continue;
                const uint32_t a = L.cell[cl[x]], e = L.cell[cl[x] + 1];
                uint32_t rank = 0;
                for (uint32_t y = a; y < e; ++y) {
                    const unsigned long long ky = L.sK[y];
                    rank += ky < w[x] || (ky == w[x] && L.sT[y] < g[x]);
                }
                L.pi[a + rank] = g[x];
            }
            __syncthreads();
        }
        // switches: local checks and tuples (4 per switch, + the idle record of odd m)
        {
            unsigned long long w[9];
            uint16_t g[9];
            bool pr[9];
#pragma unroll
            for (int x = 0; x < 9; ++x) pr[x] = false;
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                const uint32_t k = tid + y * kThreads;
                if (k >= ell) continue;
                const uint32_t i = L.pi[2 * k], j = L.pi[2 * k + 1];
                const unsigned long long e1 = L.E[i], e2 = L.E[j];
                uint8_t status = ST_UNDECIDED;
                Targets T{0, 0, false};
                if (pl_skip(k, t, b.pl, b.k0, b.k1)) {
                    status = ST_PL;
                } else {
                    T = switch_targets(e1, e2, i < j);
                    if (T.loop)
                        status = ST_LOOP;
                    else if (T.A == e1 || T.A == e2 || T.B == e1 || T.B == e2)
                        status = ST_EXISTS;
                }
                L.st[k] = status;
                L.info[2 * k] = L.info[2 * k + 1] = 0xFFFFFFFFu;
                const uint16_t et = status == ST_UNDECIDED ? (uint16_t)k : kSmTagStays;
                w[4 * y + 0] = tuple_hash(e1);
                g[4 * y + 0] = et;
                w[4 * y + 1] = tuple_hash(e2);
                g[4 * y + 1] = et;
                pr[4 * y + 0] = pr[4 * y + 1] = true;
                if (status == ST_UNDECIDED) {
                    w[4 * y + 2] = tuple_hash(T.A);
                    g[4 * y + 2] = (uint16_t)(kSmTagInsert | (k << 1));
                    w[4 * y + 3] = tuple_hash(T.B);
                    g[4 * y + 3] = (uint16_t)(kSmTagInsert | (k << 1) | 1u);
                    pr[4 * y + 2] = pr[4 * y + 3] = true;
                }
            }
            if ((m & 1u) && tid == 0) {
                w[8] = tuple_hash(L.E[L.pi[m - 1]]);
                g[8] = kSmTagStays;
                pr[8] = true;
            }
            uint32_t cl[9], slot[9];
            small_group<9>(L, w, g, pr, cl, slot);
            // all tuples of one key share a cell; each reads its cell for the
            // group's smallest tag and the largest tag before it in (key, tag,
            // slot) order: an ERASE tuple with one before it is a second
            // eraser of its key (a duplicate edge); an INSERT tuple gets its
            // eraser from the smallest tag and its predecessor from the one before
#pragma unroll
            for (int x = 0; x < 9; ++x) {
                if (!pr[x]) continue;
                const uint32_t a = L.cell[cl[x]], e = L.cell[cl[x] + 1];
                const uint16_t tx = g[x];
                uint32_t first = tx, prev = 0;
                bool before = false;
                for (uint32_t y = a; y < e; ++y) {
                    if (y == slot[x] || L.sK[y] != w[x]) continue;
                    const uint16_t ty = L.sT[y];
                    first = min(first, (uint32_t)ty);
                    if (ty < tx || (ty == tx && y < slot[x])) {
                        prev = before ? max(prev, (uint32_t)ty) : ty;
                        before = true;
                    }
                }
                if (!(tx & kSmTagInsert)) {
                    if (before) atomicOr(&L.flags, 1u);
                    continue;
                }
                uint32_t eraser = kSmNone;
                if (!(first & kSmTagInsert)) eraser = first == kSmTagStays ? kSmStays : first;
                const uint32_t pred = (before && (prev & kSmTagInsert)) ? (prev & ~(uint32_t)kSmTagInsert) : kSmNone;
                L.info[tx & ~kSmTagInsert] = (eraser << 16) | pred;
            }
            __syncthreads();
        }
        // rounds of decisions until every switch is decided
        for (;;) {
            if (tid == 0) L.undecided = 0;
            __syncthreads();
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                const uint32_t k = tid + y * kThreads;
                if (k >= ell || L.st[k] != ST_UNDECIDED) continue;
                const int v = max(small_judge(L, L.info[2 * k], k), small_judge(L, L.info[2 * k + 1], k));
                if (v == V_WAIT)
                    atomicAdd(&L.undecided, 1u);
                else
                    L.st[k] = v == V_OK ? ST_LEGAL : ST_EXISTS;
            }
            __syncthreads();
            const uint32_t left = L.undecided;
            __syncthreads();
            if (left == 0) break;
        }
        // writes and counts
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const uint32_t k = tid + y * kThreads;
            if (k >= ell) continue;
            const uint8_t sv = L.st[k];
            if (sv == ST_LEGAL) {
                const uint32_t i = L.pi[2 * k], j = L.pi[2 * k + 1];
                const Targets T = switch_targets(L.E[i], L.E[j], i < j);
                L.E[i] = T.A;
                L.E[j] = T.B;
                ++c_legal;
            }
            c_loop += sv == ST_LOOP;
            c_exists += sv == ST_EXISTS;
            c_pl += sv == ST_PL;
        }
        __syncthreads();
    }
    for (uint32_t li = tid; li < m; li += kThreads) key[b.poff + li] = L.E[li];
    if (c_legal) atomicAdd(&L.cnt[0], c_legal);
    if (c_loop) atomicAdd(&L.cnt[1], c_loop);
    if (c_exists) atomicAdd(&L.cnt[2], c_exists);
    if (c_pl) atomicAdd(&L.cnt[3], c_pl);
    __syncthreads();
    if (tid < 4) acc[4 * (size_t)q + tid] = L.cnt[tid];  // one workgroup per graph
    if (tid == 0 && L.flags) {
        atomicOr(&gerr[q], ERR_DUP);
        atomicOr(err, ERR_DUP);
    }
}

}  // namespace gesmc

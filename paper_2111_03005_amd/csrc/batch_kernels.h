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
// Small graphs: one workgroup runs all r global switches of one graph inside
// LDS -- the permutation (LDS counting sort of (K_i, i) on the top bits of K,
// then ranks within cells), the switches' ERASE / INSERT tuples grouped by
// tuple hash, the rounds of decisions of Alg. 1 and the writes -- with the
// same definitions as the multi-kernel path, so the result is the same chain.
// The records stay in LDS across supersteps.  Size classes:
//   m <= 1024 on 256 threads (39 KB of LDS, several workgroups per CU),
//   m <= 4096 on 1024 threads (158 KB, one per CU),
//   m <= 6144 on 1024 threads with every vertex id below 2^16 ("compact":
//   edge keys (min << 16) | max and 32-bit sort words, 151 KB).
// Each thread holds kMax / kThreads permutation items and half as many
// switches; there are eight sort cells per thread.
// ---------------------------------------------------------------------------
constexpr uint32_t kSmallMax = 1024, kSmallThreads = 256;  // edges, threads
constexpr uint32_t kMidMax = 4096, kMidThreads = 1024;
constexpr uint32_t kCmpMax = 6144, kCmpThreads = 1024;     // compact keys: vertex ids < 2^16
constexpr uint32_t kCmpMaxN = 1u << 16;
constexpr uint16_t kSmTagStays = 0x7FFF;  // ERASE tag of a surviving edge; erase tags are k < 0x7FFF
constexpr uint16_t kSmTagInsert = 0x8000; // | (k << 1 | h)
constexpr uint32_t kSmNone = 0xFFFFu, kSmStays = 0xFFFEu;

// Edge keys and sort words of the LDS chain: 64-bit keys and tuple hashes, or
// (compact) 32-bit keys (min << 16) | max and a 32-bit bijective mix of them.
template <bool kCompact>
struct SmallKeys {
    using Key = unsigned long long;
    using Word = unsigned long long;
    static __device__ __forceinline__ Key pack(unsigned long long e) { return e; }
    static __device__ __forceinline__ unsigned long long unpack(Key e) { return e; }
    static __device__ __forceinline__ Word word(Key e) { return tuple_hash(e); }
};

template <>
struct SmallKeys<true> {
    using Key = uint32_t;
    using Word = uint32_t;
    static __device__ __forceinline__ Key pack(unsigned long long e) {
        return ((uint32_t)(e >> 32) << 16) | ((uint32_t)e & 0xFFFFu);
    }
    static __device__ __forceinline__ unsigned long long unpack(Key e) {
        return ((unsigned long long)(e >> 16) << 32) | (e & 0xFFFFu);
    }
    // xor-shifts and odd multipliers: a bijection on 32-bit words, so equal
    // words mean equal keys
    static __device__ __forceinline__ Word word(Key x) {
        x ^= x >> 16;
        x *= 0x7FEB352Du;
        x ^= x >> 15;
        x *= 0x846CA68Bu;
        x ^= x >> 16;
        return x;
    }
};

template <uint32_t kMax, uint32_t kThreads, bool kCompact>
struct SmallLds {
    using Key = typename SmallKeys<kCompact>::Key;
    using Word = typename SmallKeys<kCompact>::Word;
    Key E[kMax];                      // edge keys by local index
    Word sK[2 * kMax];                // sorted permutation words, then sorted tuple words
    uint32_t info[kMax];              // per target 2k+h: eraser << 16 | predecessor
    uint16_t pi[kMax];                // the permutation of this superstep
    uint16_t sT[2 * kMax];            // sorted local index, then sorted tuple tag
    // sort cells: 16-bit counts, then offsets, eight per thread (two per
    // word), and the total after them at entry 8 kThreads
    alignas(16) uint32_t cellw[4 * kThreads + 4];
    uint32_t tmp[kThreads / 64 + 2];
    uint8_t st[kMax / 2];
    uint32_t und[3], flags;  // undecided counts of rounds 0, 1, 2 mod 3
    uint32_t cnt[4];
    __device__ __forceinline__ uint32_t cell(uint32_t c) const {
        return reinterpret_cast<const uint16_t *>(cellw)[c];
    }
};
static_assert(kCmpMax / 2 < kSmTagStays && 2 * kCmpMax <= 0x10000, "small-graph tags are 16 bits");
static_assert(kSmallMax % (2 * kSmallThreads) == 0 && kMidMax % (2 * kMidThreads) == 0 &&
                  kCmpMax % (2 * kCmpThreads) == 0, "whole switches per thread");

template <uint32_t kThreads>
constexpr int small_cell_bits() {  // 8 kThreads cells
    return kThreads == 256 ? 11 : kThreads == 512 ? 12 : 13;
}

// The sort cells' 16-bit counters share 32-bit words (no count reaches 2^16,
// so a half never carries into the other).  Zeroing: four words per thread.
template <uint32_t kThreads>
__device__ __forceinline__ void small_cells_zero(uint32_t *cellw) {
    reinterpret_cast<uint4 *>(cellw)[threadIdx.x] = make_uint4(0u, 0u, 0u, 0u);
}

// Adds one to cell c; returns its count before.
__device__ __forceinline__ uint32_t small_cell_add(uint32_t *cellw, uint32_t c) {
    const uint32_t sh = (c & 1u) << 4;
    return (atomicAdd(&cellw[c >> 1], 1u << sh) >> sh) & 0xFFFFu;
}

// Counts -> exclusive offsets in place (each thread its own eight cells),
// the total at entry 8 kThreads.  Returns with a barrier passed.
template <uint32_t kThreads>
__device__ __forceinline__ void small_cells_scan(uint32_t *cellw, uint32_t *tmp) {
    const uint32_t tid = threadIdx.x;
    const uint4 q = reinterpret_cast<const uint4 *>(cellw)[tid];
    uint32_t w[4] = {q.x, q.y, q.z, q.w};
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) sum += (w[i] & 0xFFFFu) + (w[i] >> 16);
    uint32_t total;
    uint32_t acc = block_exclusive_sum<kThreads>(sum, tmp, &total);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t c0 = w[i] & 0xFFFFu, c1 = w[i] >> 16;
        w[i] = acc | ((acc + c0) << 16);
        acc += c0 + c1;
    }
    reinterpret_cast<uint4 *>(cellw)[tid] = make_uint4(w[0], w[1], w[2], w[3]);
    if (tid == 0) cellw[4 * kThreads] = total;
    __syncthreads();
}

// First slot of cell c after small_group or small_group_fn (the end of cell c - 1).
template <uint32_t kMax, uint32_t kThreads, bool kCompact>
__device__ __forceinline__ uint32_t small_cell_begin(const SmallLds<kMax, kThreads, kCompact> &L, uint32_t c) {
    return c ? L.cell(c - 1) : 0u;
}

// Groups up to 2 kMax items by the top cell bits of their word: they sit in
// registers (w[q], g[q] for q < kPer where present[q]); a counting sort puts
// them in cell order into sK / sT.  The place pass takes each slot from an
// atomic bump of its cell's offset, so no rank is kept between the passes:
// within a cell the order is arbitrary (callers walk whole cells), and
// afterwards L.cell(c) holds the END of cell c, which therefore spans
// [small_cell_begin(L, c), L.cell(c)).  Returns with a barrier passed.
template <int kPer, uint32_t kMax, uint32_t kThreads, bool kCompact>
__device__ __forceinline__ void small_group(SmallLds<kMax, kThreads, kCompact> &L,
                                            const typename SmallKeys<kCompact>::Word *w, const uint16_t *g,
                                            const bool *present) {
    constexpr int kShift = 8 * (int)sizeof(typename SmallKeys<kCompact>::Word) - small_cell_bits<kThreads>();
    small_cells_zero<kThreads>(L.cellw);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q)
        if (present[q]) small_cell_add(L.cellw, (uint32_t)(w[q] >> kShift));
    __syncthreads();
    small_cells_scan<kThreads>(L.cellw, L.tmp);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        if (!present[q]) continue;
        // an offset never passes the total (< 2^16), so a low half never carries
        const uint32_t slot = small_cell_add(L.cellw, (uint32_t)(w[q] >> kShift));
        L.sK[slot] = w[q];
        L.sT[slot] = g[q];
    }
    __syncthreads();
}

// small_group with items produced on demand: item(q, &w, &g) returns whether
// item q is present and sets its word and tag.  It is called twice per item
// (count, then place) and nothing per item is kept in between; placed(q,
// slot) is told where each present item went.  Cells as in small_group.
template <int kPer, uint32_t kMax, uint32_t kThreads, bool kCompact, typename Item, typename Placed>
__device__ __forceinline__ void small_group_fn(SmallLds<kMax, kThreads, kCompact> &L, Item item, Placed placed) {
    using Word = typename SmallKeys<kCompact>::Word;
    constexpr int kShift = 8 * (int)sizeof(Word) - small_cell_bits<kThreads>();
    small_cells_zero<kThreads>(L.cellw);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        Word w;
        uint16_t g;
        if (!item(q, &w, &g)) continue;
        small_cell_add(L.cellw, (uint32_t)(w >> kShift));
    }
    __syncthreads();
    small_cells_scan<kThreads>(L.cellw, L.tmp);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        Word w;
        uint16_t g;
        if (!item(q, &w, &g)) continue;
        const uint32_t slot = small_cell_add(L.cellw, (uint32_t)(w >> kShift));
        L.sK[slot] = w;
        L.sT[slot] = g;
        placed(q, slot);
    }
    __syncthreads();
}

// Calls fn(z) for every slot z != self of the cell [a, e) whose word equals
// wy.  The words are loaded four at a time, so a walk has several LDS loads
// in flight instead of one after another.
template <typename W, typename Fn>
__device__ __forceinline__ void cell_matches(const W *sK, uint32_t a, uint32_t e, uint32_t self, W wy, Fn fn) {
    for (uint32_t z0 = a; z0 < e; z0 += 4) {
        W wz[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) wz[u] = z0 + u < e ? sK[z0 + u] : wy;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (z0 + u < e && z0 + u != self && wz[u] == wy) fn(z0 + u);
    }
}

// Alg. 1's rule for target 2k+h from its packed record (see judge_target_chain).
template <uint32_t kMax, uint32_t kThreads, bool kCompact>
__device__ __forceinline__ int small_judge(const SmallLds<kMax, kThreads, kCompact> &L, uint32_t rec, uint32_t k) {
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

// The permutation of superstep t: L.pi[x] = the local index at position x of
// the order by (K_i, i).  Returns with a barrier passed.
template <uint32_t kMax, uint32_t kThreads, bool kCompact>
__device__ __forceinline__ void small_permute(SmallLds<kMax, kThreads, kCompact> &L, uint32_t m, uint32_t t,
                                              uint32_t k0, uint32_t k1) {
    using Word = typename SmallKeys<kCompact>::Word;
    constexpr int kPer = (int)(kMax / kThreads);
    // compact permutation words are K's high 32 bits (so their top bits are
    // K's cell bits); equal words fall back to the full keys
    constexpr int kCellShift = 8 * (int)sizeof(Word) - small_cell_bits<kThreads>();
    const uint32_t tid = threadIdx.x;
    Word w[kPer];
    uint16_t g[kPer];
    bool pr[kPer];
#pragma unroll
    for (int x = 0; x < kPer; ++x) {
        const uint32_t li = tid + x * kThreads;
        pr[x] = li < m;
        const unsigned long long kf = pr[x] ? perm_key(li, t, k0, k1) : ~0ull;
        w[x] = kCompact ? (Word)(kf >> 32) : (Word)kf;
        g[x] = (uint16_t)li;
    }
    small_group<kPer>(L, w, g, pr);
    // keys (K_i, i) are distinct: an index's place is the number of smaller
    // keys in its cell (one grouped item per thread at a time; its word's top
    // bits give its cell)
    for (uint32_t y = tid; y < m; y += kThreads) {
        const Word wy = L.sK[y];
        const uint16_t gy = L.sT[y];
        const uint32_t cc = (uint32_t)(wy >> kCellShift);
        const uint32_t a = small_cell_begin(L, cc), e = L.cell(cc);
        uint32_t rank = 0;
        for (uint32_t z0 = a; z0 < e; z0 += 4) {  // four loads in flight
            Word wz[4];
            uint16_t gz[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                wz[u] = z0 + u < e ? L.sK[z0 + u] : wy;
                gz[u] = z0 + u < e ? L.sT[z0 + u] : gy;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                bool less = wz[u] < wy;
                if (wz[u] == wy && gz[u] != gy) {
                    if (kCompact) {  // equal high words (rare): compare the full keys
                        const unsigned long long fz = perm_key(gz[u], t, k0, k1), fy = perm_key(gy, t, k0, k1);
                        less = fz < fy || (fz == fy && gz[u] < gy);
                    } else {
                        less = gz[u] < gy;
                    }
                }
                rank += less;
            }
        }
        L.pi[a + rank] = gy;
    }
    __syncthreads();
}

// Permutations of supersteps t0 .. t0 + gridDim.x - 1 of an m-edge graph,
// one workgroup each: row s of pi (kMax entries, the first m used) is the
// permutation of superstep t0 + s.  They depend on nothing but (m, t, seed),
// so k_small_plain takes them from here instead of computing them on its one
// workgroup between supersteps.  zero: null, or 16 words to clear first (the
// call's error word and counts, read by the k_small_plain launches after it).
template <uint32_t kMax, uint32_t kThreads, bool kCompact>
__global__ __launch_bounds__(kThreads) void k_small_perm(uint32_t m, uint32_t t0, uint32_t k0, uint32_t k1,
                                                         uint16_t *__restrict__ pi, uint32_t *__restrict__ zero) {
    __shared__ SmallLds<kMax, kThreads, kCompact> L;
    if (zero && blockIdx.x == 0 && threadIdx.x < 16) zero[threadIdx.x] = 0;
    small_permute(L, m, t0 + blockIdx.x, k0, k1);
    uint16_t *row = pi + (size_t)blockIdx.x * kMax;
    for (uint32_t x = threadIdx.x; x < m; x += kThreads) row[x] = L.pi[x];
}

// All r supersteps of one graph in LDS.  L.E holds its m edge keys (local
// ids) on entry and the result on exit; counts go to c[4] (legal, loop,
// exists, P_L, per thread).  A duplicate edge (two ERASE tuples of one key
// in the first superstep) sets L.flags.  kPre: the permutations of the r
// supersteps are read from pre (k_small_perm rows), else computed here.
template <bool kPre, uint32_t kMax, uint32_t kThreads, bool kCompact>
__device__ __forceinline__ void small_chain_body(SmallLds<kMax, kThreads, kCompact> &L, uint32_t m, uint32_t r,
                                                 uint32_t t0, uint32_t pl, uint32_t k0, uint32_t k1, uint32_t *c,
                                                 const uint16_t *__restrict__ pre) {
    using K = SmallKeys<kCompact>;
    using Word = typename K::Word;
    constexpr int kPer = (int)(kMax / kThreads);  // permutation items per thread
    constexpr int kSw = kPer / 2;                 // switches per thread
    static_assert(kSw <= 4, "a thread's switch statuses are the bytes of one 32-bit word");
    constexpr int kTu = 4 * kSw + 1;              // tuples per thread (+ the idle record of odd m)
    constexpr int kPiW = kPer / 2;                // 32-bit words of a permutation row per thread
    constexpr uint8_t kAbsent = 0xFF;             // a switch index at or beyond ell
    constexpr int kCellShift = 8 * (int)sizeof(Word) - small_cell_bits<kThreads>();
    const uint32_t tid = threadIdx.x;
    const uint32_t ell = m >> 1, mw = (m + 1) >> 1;
    uint32_t pw[kPiW];  // the next superstep's permutation row (kPre), loaded one superstep ahead
    if (kPre) {
        const uint32_t *row = reinterpret_cast<const uint32_t *>(pre);
#pragma unroll
        for (int q = 0; q < kPiW; ++q) {
            const uint32_t x = tid + q * kThreads;
            pw[q] = x < mw ? row[x] : 0u;
        }
    }
    for (uint32_t s = 0; s < r; ++s) {
        const uint32_t t = t0 + s;
        if (kPre) {
            uint32_t *lp = reinterpret_cast<uint32_t *>(L.pi);
#pragma unroll
            for (int q = 0; q < kPiW; ++q) {
                const uint32_t x = tid + q * kThreads;
                if (x < mw) lp[x] = pw[q];
            }
            if (s + 1 < r) {
                const uint32_t *row = reinterpret_cast<const uint32_t *>(pre + (size_t)(s + 1) * kMax);
#pragma unroll
                for (int q = 0; q < kPiW; ++q) {
                    const uint32_t x = tid + q * kThreads;
                    pw[q] = x < mw ? row[x] : 0u;
                }
            }
            __syncthreads();
        } else {
            small_permute(L, m, t, k0, k1);
        }
        // switches: local checks; this thread's switches (k = tid + y kThreads)
        // keep their indices and status (byte y of sst) in registers, and with
        // kPre (no permutation code beside them) their edge keys too
        uint32_t sij[kSw];
        uint32_t sst = 0;
        constexpr int kSe = kPre ? kSw : 1;
        typename K::Key se[kSe][2];
        // compact keys with kPre: the targets too, computed once per superstep
        // (fewer VALU instructions on the chain's one CU; the 64-bit keys of
        // the other classes would not fit the registers)
        constexpr bool kTg = kPre && kCompact;
        constexpr int kTe = kTg ? kSw : 1;
        typename K::Key tg[kTe][2];
        auto key_of = [&](int y, uint32_t h) -> typename K::Key {
            if (kPre) return se[y < kSe ? y : 0][h];
            return L.E[h ? sij[y] >> 16 : sij[y] & 0xFFFFu];
        };
        auto st_of = [&](int y) -> uint32_t { return (sst >> (8 * y)) & 0xFFu; };
        auto set_st = [&](int y, uint32_t v) { sst = (sst & ~(0xFFu << (8 * y))) | (v << (8 * y)); };
#pragma unroll
        for (int y = 0; y < kSw; ++y) {
            const uint32_t k = tid + y * kThreads;
            set_st(y, kAbsent);
            sij[y] = 0;
            if (k >= ell) continue;
            const uint32_t i = L.pi[2 * k], j = L.pi[2 * k + 1];
            sij[y] = i | (j << 16);
            const typename K::Key ki = L.E[i], kj = L.E[j];
            if (kPre) {
                se[y < kSe ? y : 0][0] = ki;
                se[y < kSe ? y : 0][1] = kj;
            }
            const unsigned long long e1 = K::unpack(ki), e2 = K::unpack(kj);
            uint8_t status = ST_UNDECIDED;
            if (pl_skip(k, t, pl, k0, k1)) {
                status = ST_PL;
            } else {
                const Targets T = switch_targets(e1, e2, i < j);
                if (kTg) {
                    tg[y < kTe ? y : 0][0] = K::pack(T.A);
                    tg[y < kTe ? y : 0][1] = K::pack(T.B);
                }
                if (T.loop)
                    status = ST_LOOP;
                else if (T.A == e1 || T.A == e2 || T.B == e1 || T.B == e2)
                    status = ST_EXISTS;
            }
            set_st(y, status);
            L.st[k] = status;
            L.info[2 * k] = L.info[2 * k + 1] = 0xFFFFFFFFu;
        }
        // tuples (4 per switch, + the idle record of odd m) grouped by word,
        // computed from the registers whenever the grouping needs them; the
        // slots of this thread's INSERT tuples are kept
        uint32_t islot[kSw];  // slots of the two INSERT tuples, 16 bits each
#pragma unroll
        for (int y = 0; y < kSw; ++y) islot[y] = 0;
        {
            auto tuple = [&](int q, Word *w, uint16_t *g) -> bool {
                if (q == kTu - 1) {  // the idle record of odd m survives the superstep
                    if (!((m & 1u) && tid == 0)) return false;
                    *w = K::word(L.E[L.pi[m - 1]]);
                    *g = kSmTagStays;
                    return true;
                }
                const int y = q >> 2;
                const uint32_t h = (uint32_t)q & 3u, k = tid + (uint32_t)y * kThreads;
                if (st_of(y) == kAbsent) return false;
                const uint32_t i = sij[y] & 0xFFFFu, j = sij[y] >> 16;
                if (h < 2) {
                    *w = K::word(key_of(y, h));
                    *g = st_of(y) == ST_UNDECIDED ? (uint16_t)k : kSmTagStays;
                    return true;
                }
                if (st_of(y) != ST_UNDECIDED) return false;
                if (kTg) {
                    *w = K::word(tg[y < kTe ? y : 0][h - 2]);
                } else {
                    const Targets T = switch_targets(K::unpack(key_of(y, 0)), K::unpack(key_of(y, 1)), i < j);
                    *w = K::word(K::pack(h == 2 ? T.A : T.B));
                }
                *g = (uint16_t)(kSmTagInsert | (k << 1) | (h - 2));
                return true;
            };
            auto placed = [&](int q, uint32_t slot) {
                if (q < kTu - 1 && (q & 3) == 2) islot[q >> 2] = slot;
                if (q < kTu - 1 && (q & 3) == 3) islot[q >> 2] |= slot << 16;
            };
            small_group_fn<kTu>(L, tuple, placed);
        }
        // all tuples of one key share a cell.  Input duplicates (first
        // superstep only: every later state is simple): an ERASE tuple with
        // another ERASE tuple of its key before it in (key, tag, slot) order.
        if (s == 0) {
            const uint32_t ntu = L.cell(8 * kThreads);
            for (uint32_t y = tid; y < ntu; y += kThreads) {
                const uint16_t ty = L.sT[y];
                if (ty & kSmTagInsert) continue;
                const Word wy = L.sK[y];
                const uint32_t cc = (uint32_t)(wy >> kCellShift);
                const uint32_t a = small_cell_begin(L, cc), e = L.cell(cc);
                bool before = false;
                cell_matches(L.sK, a, e, y, wy, [&](uint32_t z) {
                    const uint16_t tz = L.sT[z];
                    before |= tz < ty || (tz == ty && z < y);
                });
                if (before) atomicOr(&L.flags, 1u);
            }
        }
        // each INSERT tuple of an undecided switch finds in its cell its
        // key group's smallest tag (-> eraser) and the largest tag before its
        // own (-> predecessor inserter)
#pragma unroll
        for (int y = 0; y < kSw; ++y) {
            if (st_of(y) != ST_UNDECIDED) continue;
            const uint32_t k = tid + (uint32_t)y * kThreads;
            Word tw[2] = {0, 0};  // the two INSERT words, from the keys in registers (kPre)
            if (kTg) {
                tw[0] = K::word(tg[y < kTe ? y : 0][0]);
                tw[1] = K::word(tg[y < kTe ? y : 0][1]);
            } else if (kPre) {
                const Targets T = switch_targets(K::unpack(key_of(y, 0)), K::unpack(key_of(y, 1)),
                                                 (sij[y] & 0xFFFFu) < (sij[y] >> 16));
                tw[0] = K::word(K::pack(T.A));
                tw[1] = K::word(K::pack(T.B));
            }
#pragma unroll 1
            for (uint32_t h = 0; h < 2; ++h) {
                const uint32_t sl = (islot[y] >> (16 * h)) & 0xFFFFu;
                const Word wy = kPre ? (h ? tw[1] : tw[0]) : L.sK[sl];
                const uint32_t ty = kSmTagInsert | (k << 1) | h;
                const uint32_t cc = (uint32_t)(wy >> kCellShift);
                const uint32_t a = small_cell_begin(L, cc), e = L.cell(cc);
                uint32_t first = ty, prev = 0;
                bool before = false;
                cell_matches(L.sK, a, e, sl, wy, [&](uint32_t z) {
                    const uint32_t tz = L.sT[z];
                    first = min(first, tz);
                    if (tz < ty) {  // INSERT tags are distinct
                        prev = before ? max(prev, tz) : tz;
                        before = true;
                    }
                });
                uint32_t eraser = kSmNone;
                if (!(first & kSmTagInsert)) eraser = first == kSmTagStays ? kSmStays : first;
                const uint32_t pred = (before && (prev & kSmTagInsert)) ? (prev & ~(uint32_t)kSmTagInsert) : kSmNone;
                L.info[2 * k + h] = (eraser << 16) | pred;
            }
        }
        if (tid == 0) L.und[0] = 0;
        __syncthreads();
        // rounds of decisions until every switch is decided, one barrier each:
        // round x counts its waits in und[x mod 3] and clears und[x + 1 mod 3],
        // which was last read in round x - 2
        for (uint32_t x = 0;; x = x == 2 ? 0 : x + 1) {
            if (tid == 0) L.und[x == 2 ? 0 : x + 1] = 0;
#pragma unroll
            for (int y = 0; y < kSw; ++y) {
                if (st_of(y) != ST_UNDECIDED) continue;
                const uint32_t k = tid + (uint32_t)y * kThreads;
                const int v = max(small_judge(L, L.info[2 * k], k), small_judge(L, L.info[2 * k + 1], k));
                if (v == V_WAIT) {
                    atomicAdd(&L.und[x], 1u);
                } else {
                    const uint32_t d = v == V_OK ? ST_LEGAL : ST_EXISTS;
                    set_st(y, d);
                    L.st[k] = (uint8_t)d;
                }
            }
            __syncthreads();
            if (L.und[x] == 0) break;  // uniform: no count of round x changes after the barrier
        }
        // writes and counts
#pragma unroll
        for (int y = 0; y < kSw; ++y) {
            const uint32_t sv = st_of(y);
            if (sv == ST_LEGAL) {
                const uint32_t i = sij[y] & 0xFFFFu, j = sij[y] >> 16;
                if (kTg) {
                    L.E[i] = tg[y < kTe ? y : 0][0];
                    L.E[j] = tg[y < kTe ? y : 0][1];
                } else {
                    const Targets T = switch_targets(K::unpack(key_of(y, 0)), K::unpack(key_of(y, 1)), i < j);
                    L.E[i] = K::pack(T.A);
                    L.E[j] = K::pack(T.B);
                }
                ++c[0];
            }
            c[1] += sv == ST_LOOP;
            c[2] += sv == ST_EXISTS;
            c[3] += sv == ST_PL;
        }
        __syncthreads();
    }
}

template <uint32_t kMax, uint32_t kThreads, bool kCompact>
__device__ __forceinline__ void small_flush_counts(SmallLds<kMax, kThreads, kCompact> &L, const uint32_t *c) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (c[q]) atomicAdd(&L.cnt[q], c[q]);
    __syncthreads();
}

// One workgroup per listed graph of a batch (ranks `small[0 .. count)`, r of
// rank q in rv[q], m of every listed graph <= kMax, and n < 2^16 if
// kCompact); records of graph q are at positions poff + local index of
// `key` (vertex ids shifted by the graph's vbase); its outcome counts go to
// acc[4q .. 4q+3] (legal, loop, exists, P_L).
template <uint32_t kMax, uint32_t kThreads, bool kCompact>
__global__ __launch_bounds__(kThreads) void k_small_chain(const uint32_t *__restrict__ small,
                                                          const BatchGraph *__restrict__ gr,
                                                          const uint32_t *__restrict__ rv,
                                                          unsigned long long *__restrict__ key,
                                                          unsigned long long *__restrict__ acc,
                                                          uint32_t *__restrict__ gerr, uint32_t *__restrict__ err) {
    using K = SmallKeys<kCompact>;
    __shared__ SmallLds<kMax, kThreads, kCompact> L;
    const uint32_t tid = threadIdx.x;
    const uint32_t q = small[blockIdx.x];
    const BatchGraph b = gr[q];
    const unsigned long long shift = ((unsigned long long)b.vbase << 32) | b.vbase;
    for (uint32_t li = tid; li < b.m; li += kThreads) L.E[li] = K::pack(key[b.poff + li] - shift);
    if (tid < 4) L.cnt[tid] = 0;
    if (tid == 0) L.flags = 0;
    uint32_t c[4] = {0, 0, 0, 0};
    __syncthreads();
    small_chain_body<false>(L, b.m, rv[q], b.t0, b.pl, b.k0, b.k1, c, nullptr);
    for (uint32_t li = tid; li < b.m; li += kThreads) key[b.poff + li] = K::unpack(L.E[li]) + shift;
    small_flush_counts(L, c);
    if (tid < 4) acc[4 * (size_t)q + tid] = L.cnt[tid];  // one workgroup per graph
    if (tid == 0 && L.flags) {
        atomicOr(&gerr[q], ERR_DUP);
        atomicOr(err, ERR_DUP);
    }
}

// The plain form on one small graph (m <= kMax, n < 2^16 if kCompact), for
// r supersteps in one launch: loads and checks the input (canonical keys,
// ids < n, no loop), runs every superstep in LDS, and writes `out` only if no
// error was found (a duplicate shows in the first superstep).  Counts are
// added to acc[0 .. 3].  A call's supersteps may come in several launches,
// each resuming from the last one's output (in may equal out); a launch
// does nothing once an earlier one has set err[0].  pre: the r supersteps'
// permutations (k_small_perm).
template <uint32_t kMax, uint32_t kThreads, bool kCompact>
__global__ __launch_bounds__(kThreads) void k_small_plain(const unsigned long long *in, unsigned long long *out,
                                                          uint32_t m, uint32_t n, uint32_t t0, uint32_t r,
                                                          uint32_t pl, uint32_t k0, uint32_t k1,
                                                          unsigned long long *__restrict__ acc,
                                                          uint32_t *__restrict__ err,
                                                          const uint16_t *__restrict__ pre) {
    using K = SmallKeys<kCompact>;
    __shared__ SmallLds<kMax, kThreads, kCompact> L;
    const uint32_t tid = threadIdx.x;
    if (err[0] != 0) return;  // uniform: written by an earlier launch
    if (tid < 4) L.cnt[tid] = 0;
    if (tid == 0) L.flags = 0;
    __syncthreads();
    uint32_t f = 0;
    for (uint32_t li = tid; li < m; li += kThreads) {
        const unsigned long long e = in[li];
        const uint32_t a = (uint32_t)(e >> 32), b = (uint32_t)e;
        if (a == b) f |= ERR_LOOP;
        if (a >= n || b >= n || a == 0xFFFFFFFFu || b == 0xFFFFFFFFu) f |= ERR_RANGE;
        L.E[li] = K::pack(ekey(a, b));
    }
    if (f) atomicOr(&L.flags, f << 1);
    __syncthreads();
    const uint32_t bad = L.flags;
    __syncthreads();
    uint32_t c[4] = {0, 0, 0, 0};
    if (!bad) small_chain_body<true>(L, m, r, t0, pl, k0, k1, c, pre);  // uniform: every thread read the same flags
    small_flush_counts(L, c);
    const uint32_t fl = L.flags;
    if (fl) {
        if (tid == 0) atomicOr(err, (fl & 1u ? ERR_DUP : 0u) | (fl >> 1));
        return;
    }
    for (uint32_t li = tid; li < m; li += kThreads) out[li] = K::unpack(L.E[li]);
    if (tid < 4) acc[tid] += L.cnt[tid];
}

}  // namespace gesmc

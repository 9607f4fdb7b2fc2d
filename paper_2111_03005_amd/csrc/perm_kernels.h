// Permutation pi of one global switch (Def. 3.2; the random-keys shuffle the
// paper's parallel permutation builds on, Sec. 5.3): the edge records
// (index, key) are placed in ascending (K_i, i) order, where K_i is the
// Philox key of edge index i in superstep t.
//
// MSD radix layout for gfx950:
//   level 1   : coarse digit = top b1 bits of K (b1 <= 10), LDS-staged scatter;
//               run bases from per-tile digit counts and a column scan
//   level 2   : sub digit    = next b2 bits, scattered inside each coarse
//               bucket (its region is small enough to stay L2/MALL resident)
//   bucket    : each fine bucket (~400-1500 records) is counting-sorted in
//               LDS on the next kCellBits bits of K (about one record per
//               cell), then each record's place in its cell is the number of
//               smaller (K, i) keys there.
// Keys are never stored: every pass recomputes K_i from the record's index.
#pragma once

#include "device_common.h"

namespace gesmc {

// Records per scatter workgroup ("tile"): 2048, or 4096 for passes over at
// least 2^25 records, where the longer runs per digit of the second level
// pay off; on smaller passes the larger tile leaves CUs idle.
constexpr int kTileSmall = 2048, kTileLarge = 4096;
#ifndef GESMC_LARGE_TILE_RECORDS
#define GESMC_LARGE_TILE_RECORDS (1u << 25)
#endif
constexpr uint32_t kLargeTileRecords = GESMC_LARGE_TILE_RECORDS;
constexpr uint32_t kMaxCoarseBits = 10;  // digit bits of the first radix level
#ifndef GESMC_CELL_BITS
#define GESMC_CELL_BITS 10
#endif
// LDS counting-sort cells per bucket / partition = 2^bits.  Records then
// read their whole cell, so the wave's cost follows its largest cell: 1024
// cells (about one record each) beat 256 by ~15%; 2048 lose LDS occupancy.
constexpr int kCellBits = GESMC_CELL_BITS;
#ifndef GESMC_LDS_ITEMS
#define GESMC_LDS_ITEMS 6
#endif
constexpr int kSortMaxItems = GESMC_LDS_ITEMS;  // records per thread held in LDS
// Threads of a scatter workgroup per tile size: the large tile's LDS stage
// (~60 KB) allows two workgroups per CU, so it takes 512 threads to keep
// enough waves in flight; the small tile fits more workgroups at 256.
#ifndef GESMC_SCATTER_THREADS_LARGE
#define GESMC_SCATTER_THREADS_LARGE 512
#endif
#ifndef GESMC_SCATTER_THREADS_SMALL
#define GESMC_SCATTER_THREADS_SMALL 256
#endif
constexpr int scatter_threads(int tile) {
    return tile >= kTileLarge ? GESMC_SCATTER_THREADS_LARGE : GESMC_SCATTER_THREADS_SMALL;
}
constexpr uint32_t kLdsCap = kSortMaxItems * kBlock;  // records of one bucket sorted in LDS
static_assert((1 << kCellBits) >= kBlock, "every thread owns at least one cell");

// Inclusive prefix sum across one wave64 (shuffle-up ladder).
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive prefix sum of one value per thread over a workgroup of NT
// threads.  `wsum` needs NT/64 + 1 words of LDS.  Returns the thread's
// exclusive prefix; *total receives the sum over the workgroup.
template <int NT>
__device__ __forceinline__ uint32_t block_exclusive_sum(uint32_t x, uint32_t *wsum, uint32_t *total) {
    constexpr int kWaves = NT / 64;
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t incl = wave_inclusive_scan(x);
    if (lane == 63) wsum[w] = incl;
    lds_barrier();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
        const uint32_t v = wsum[q];
        before += (q < (int)w) ? v : 0u;
        all += v;
    }
    lds_barrier();
    *total = all;
    return before + incl - x;
}

// Workgroup-wide exclusive scan (in place) of n values in LDS over NT
// threads; each owns a contiguous run of ceil(n / NT).  `tmp` needs NT / 64 + 1
// words.
// Returns the total.
template <int NT = kBlock>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t *v, uint32_t n, uint32_t *tmp) {
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (n + NT - 1) / NT;
    const uint32_t b = min(tid * per, n);
    const uint32_t e = min(b + per, n);
    uint32_t s = 0;
    for (uint32_t q = b; q < e; ++q) s += v[q];
    uint32_t total;
    uint32_t acc = block_exclusive_sum<NT>(s, tmp, &total);
    for (uint32_t q = b; q < e; ++q) {
        const uint32_t x = v[q];
        v[q] = acc;
        acc += x;
    }
    lds_barrier();
    return total;
}

// ---------------------------------------------------------------------------
// Per-superstep reset: switch states, list counters and (table strategy only)
// the dependency table.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_step_clear(Slot *__restrict__ tab, uint64_t tab_slots,
                                                       uint8_t *__restrict__ st, uint32_t ell,
                                                       uint32_t *__restrict__ ucount) {
    const uint64_t nthreads = (uint64_t)gridDim.x * kBlock;
    const uint64_t gtid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    // table reset: 16-byte vector stores of {empty key, no eraser, no claim}
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    u32x4 *t4 = reinterpret_cast<u32x4 *>(tab);
    const u32x4 empty = {0xFFFFFFFFu, 0xFFFFFFFFu, kNoEraser, kClaimNone};
    for (uint64_t s = gtid; s < tab_slots; s += nthreads) __builtin_nontemporal_store(empty, &t4[s]);
    for (uint64_t k = gtid; k < ell; k += nthreads) st[k] = ST_UNDECIDED;
    if (gtid < 3) ucount[gtid] = 0;
}

// Locates the segment of tile w: the largest s with tile_first[s] <= w.
__device__ __forceinline__ uint32_t tile_segment(const uint32_t *tile_first, uint32_t nseg, uint32_t w) {
    uint32_t lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (tile_first[mid] <= w)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Radix source of a record.  kSrcPerm sorts edge records by the Philox key
// of their index (the permutation); kSrcHash sorts (tag, edge key) tuples by
// a hash of the edge key (the dependency partitions), where an empty key
// marks a tuple slot that carries nothing (the first pass turns keys into
// tuple_hash words, which the second pass, kSrcHashed, and the resolve read
// as they are); kSrcEmit is kSrcHash over the
// tuples of the switches themselves, computed from the pair records while
// they are read (slots 4k .. 4k+3 of switch k; see emit_switch), so the flat tuple
// array is never stored.  A batch of graphs sorts by the global bucket
// (graph, K range) of each record: kSrcBatch computes it from the graph of
// the record's position (level 1) and writes it out beside the record,
// kSrcBucket reads it back (level 2).  Bucket numbers are placed in the top
// B bits of the radix word, so both levels use the same shifts.
// kSrcEmitPacked is kSrcEmit writing packed 8-byte tuple words (TuplePack)
// and kSrcPacked the second level over them: no tag array is read or written.
// kSrcIdx sorts records by their own index (idx << ishift puts its top bits
// on top): the buckets of the final write-back to input order.
enum RadixSrc : int {
    kSrcPerm = 0,
    kSrcHash = 1,
    kSrcBatch = 2,
    kSrcBucket = 3,
    kSrcEmit = 4,
    kSrcHashed = 5,
    kSrcEmitPacked = 6,
    kSrcPacked = 7,
    kSrcIdx = 8,
    kSrcEmitPackedLocal = 9  // kSrcEmitPacked with tags local to each graph (TuplePack.local)
};

struct SrcArgs {
    const BatchGraph *gr;    // per graph (batches)
    const uint32_t *aux_in;  // kSrcBatch: graph of each position; kSrcBucket: bucket of each position
    uint32_t *aux_out;       // kSrcBatch: bucket of each output position
    uint32_t step;           // batch superstep
    int bbits;               // bucket bits B (1 .. 32)
    // kSrcEmit
    const uint32_t *pg;      // batch: graph of each position (nullptr: one graph)
    uint32_t m;              // records (the pair records of ell = m / 2 switches)
    uint32_t pl;             // P_L threshold (batch: nonzero if some graph has one)
    TuplePack pk;            // kSrcEmitPacked: hash width, offset and tag code bits
    uint32_t cls;            // graph class (CLS_* bits; multi-edge classes never come here)
    uint32_t ishift;         // kSrcIdx: 64 - (bits of the largest index)
    // kSrcPerm: nonzero if every vertex id is below 2^24 and a level has at
    // most 8 digit bits; the scatter then stages each record's digit in the
    // edge key's top byte (zero in such keys) instead of a digit array
    uint32_t dig_in_key;
};

template <int kSrc>
__device__ __forceinline__ constexpr bool src_reads_idx() {
    return kSrc == kSrcPerm || kSrc == kSrcBatch || kSrc == kSrcIdx;
}
template <int kSrc>
__device__ __forceinline__ constexpr bool src_reads_aux() { return kSrc == kSrcBatch || kSrc == kSrcBucket; }
// Tuple sources whose slots may be empty (kEmptyKey); the second level over
// packed words has none (every word is a tuple, and any word value occurs).
template <int kSrc>
__device__ __forceinline__ constexpr bool src_is_tuple() {
    return kSrc == kSrcHash || kSrc == kSrcEmit || kSrc == kSrcHashed || kSrc == kSrcEmitPacked ||
           kSrc == kSrcEmitPackedLocal;
}
template <int kSrc>
__device__ __host__ __forceinline__ constexpr bool src_emits_packed() {
    return kSrc == kSrcEmitPacked || kSrc == kSrcEmitPackedLocal;
}
template <int kSrc>
__device__ __forceinline__ constexpr bool src_emits() { return kSrc == kSrcEmit || src_emits_packed<kSrc>(); }
template <int kSrc>
__device__ __forceinline__ constexpr bool src_packed() { return src_emits_packed<kSrc>() || kSrc == kSrcPacked; }

// Local outcome of switch k from its pair records (ij, ee): P_L skip, the
// idle pair of a batch graph's padding record, a loop, or a target equal to
// one of its own sources or to its other target (Def. 2.1; the last occurs
// only with loops, as two loop sources); ST_UNDECIDED if it depends on others.
__device__ __forceinline__ uint8_t switch_local(uint32_t k, uint2 ij, ulonglong2 ee, uint32_t t, uint32_t k0,
                                                uint32_t k1, const SrcArgs &sa, Targets *T) {
    bool skip = false;
    if (sa.pg) {
        if (ij.x == kPadIdx || ij.y == kPadIdx) return ST_IDLE;
        if (sa.pl != 0) {  // some graph of the batch has P_L > 0
            const BatchGraph &g = sa.gr[sa.pg[2 * (size_t)k]];
            skip = pl_skip(k - (g.poff >> 1), g.t0 + sa.step, g.pl, g.k0, g.k1);
        }
    } else {
        skip = pl_skip(k, t, sa.pl, k0, k1);
    }
    if (skip) return ST_PL;
    *T = switch_targets_cls(ee.x, ee.y, ij.x < ij.y, sa.cls);
    if (T->loop) return ST_LOOP;
    if (T->A == ee.x || T->A == ee.y || T->B == ee.x || T->B == ee.y || T->A == T->B) return ST_EXISTS;
    return ST_UNDECIDED;
}

struct Tuple {
    uint32_t tag;
    unsigned long long key;
};

// The four tuple slots 4k .. 4k+3 of switch k (Alg. 1's erase and insert
// entries): j = 0, 1 the ERASE tuples of its sources, j = 2, 3 the INSERT
// tuples of its targets.  A switch decided locally keeps its sources (STAYS)
// and inserts nothing; slot 4 ell holds the idle record of odd m.
// The four tuples of switch k < ell with pair records (ij, ee), local
// outcome `status` and targets T.
__device__ __forceinline__ void switch_tuples(uint32_t k, uint2 ij, ulonglong2 ee, uint8_t status, Targets T,
                                              Tuple *tp) {
    tp[1] = tp[2] = tp[3] = Tuple{0u, kEmptyKey};
    if (status == ST_UNDECIDED) {
        tp[0] = Tuple{k, ee.x};
        tp[1] = Tuple{k, ee.y};
        tp[2] = Tuple{kTagInsert | (k << 1), T.A};
        tp[3] = Tuple{kTagInsert | (k << 1) | 1u, T.B};
    } else {
        tp[0] = Tuple{kTagStays, ij.x == kPadIdx ? kEmptyKey : ee.x};
        tp[1] = Tuple{kTagStays, ij.y == kPadIdx ? kEmptyKey : ee.y};
    }
}

__device__ __forceinline__ void emit_switch(uint32_t k, const uint32_t *si, const unsigned long long *sk, uint32_t t,
                                            uint32_t k0, uint32_t k1, const SrcArgs &sa, Tuple *tp) {
    const uint32_t ell = sa.m >> 1;
    tp[1] = tp[2] = tp[3] = Tuple{0u, kEmptyKey};
    if (k >= ell) {
        tp[0] = (k == ell && (sa.m & 1u)) ? Tuple{kTagStays, sk[sa.m - 1]} : Tuple{0u, kEmptyKey};
        return;
    }
    const uint2 ij = reinterpret_cast<const uint2 *>(si)[k];
    const ulonglong2 ee = reinterpret_cast<const ulonglong2 *>(sk)[k];
    Targets T{0, 0, false};
    const uint8_t status = switch_local(k, ij, ee, t, k0, k1, sa, &T);
    // the tuples of switch_tuples, written out here: calling it from this
    // function made the compiler keep T in scratch memory
    if (status == ST_UNDECIDED) {
        tp[0] = Tuple{k, ee.x};
        tp[1] = Tuple{k, ee.y};
        tp[2] = Tuple{kTagInsert | (k << 1), T.A};
        tp[3] = Tuple{kTagInsert | (k << 1) | 1u, T.B};
    } else {
        tp[0] = Tuple{kTagStays, ij.x == kPadIdx ? kEmptyKey : ee.x};
        tp[1] = Tuple{kTagStays, ij.y == kPadIdx ? kEmptyKey : ee.y};
    }
}

// The radix word of a tuple key emitted by kSrcEmit / kSrcEmitPacked.
template <bool kPacked>
__device__ __forceinline__ unsigned long long emitted_word(unsigned long long key, const SrcArgs &sa) {
    if (key == kEmptyKey) return kEmptyKey;
    return kPacked ? key_hash_w(key, sa.pk.db, sa.pk.w) << (64 - sa.pk.w) : tuple_hash(key);
}

// kSrcEmit tiles: each thread takes whole switches, so the four slots of a
// switch are items 4j .. 4j+3 of one thread (slot order inside a tile does
// not matter: partitions are sorted later).  kPacked: tag codes and the
// w-bit key hash aligned to the top of the word (the radix word); the
// scatter packs them.  kLocal: tags local to the switch's graph.
template <int kTileItems, int kThreads, bool kPacked, bool kLocal = false>
__device__ __forceinline__ void emit_tile(uint32_t begin, uint32_t cnt, const uint32_t *si,
                                          const unsigned long long *sk, uint32_t t, uint32_t k0, uint32_t k1,
                                          const SrcArgs &sa, uint32_t *tag, unsigned long long *key) {
    const uint32_t tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < kTileItems / 4; ++j) {
        const uint32_t sl = 4 * (tid + j * kThreads);  // first local slot of this thread's switch
        Tuple tp[4] = {{0u, kEmptyKey}, {0u, kEmptyKey}, {0u, kEmptyKey}, {0u, kEmptyKey}};
        uint32_t kbase = 0;  // first switch of the switch's graph (graph-local tags)
        if (sl < cnt) {
            const uint32_t k = (begin + sl) >> 2;
            emit_switch(k, si, sk, t, k0, k1, sa, tp);
            if (kLocal && k < (sa.m >> 1)) kbase = sa.gr[sa.pg[2 * (size_t)k]].poff >> 1;
        }
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            tag[4 * j + h] = kPacked ? tag_code(kLocal ? tag_shift(tp[h].tag, kbase, true) : tp[h].tag, sa.pk.kb)
                                     : tp[h].tag;
            key[4 * j + h] = sl + h < cnt ? emitted_word<kPacked>(tp[h].key, sa) : kEmptyKey;
        }
    }
}

// Workgroups are dispatched round-robin over the chip's XCDs (workgroup b
// runs on XCD b % kXcds), each with its own L2.  xcd_tile maps dispatch order
// v in [0, n) to a tile so that XCD x works on the contiguous tiles
// [x * n / kXcds, ...): the adjacent runs that neighbouring tiles write for
// one digit then meet in the same L2.  A bijection on [0, n); with a
// grid-stride loop the grid must be a multiple of kXcds.
#ifndef GESMC_XCD_REMAP
#define GESMC_XCD_REMAP 1
#endif
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_tile(uint32_t v, uint32_t n) {
    if (!GESMC_XCD_REMAP) return v;
    const uint32_t x = v % kXcds, i = v / kXcds, q = n / kXcds, r = n % kXcds;
    return x * q + min(x, r) + i;
}

// Radix word of one record; *bucket receives the global bucket (kSrcBatch).
template <int kSrc>
__device__ __forceinline__ uint64_t radix_word(uint32_t idx, unsigned long long key, uint32_t aux, uint32_t t,
                                               uint32_t k0, uint32_t k1, const SrcArgs &ba, uint32_t *bucket) {
    if (src_is_tuple<kSrc>() || kSrc == kSrcPacked) return key;  // tuple hashes or packed words (see the loads)
    if (kSrc == kSrcPerm) return perm_key(idx, t, k0, k1);
    if (kSrc == kSrcIdx) return (uint64_t)idx << ba.ishift;
    uint32_t b = aux;
    if (kSrc == kSrcBatch) {
        const BatchGraph &g = ba.gr[aux];
        b = batch_bucket(g, batch_perm_key(g, idx, ba.step));
        *bucket = b;
    }
    return (uint64_t)b << (64 - ba.bbits);
}

// ---------------------------------------------------------------------------
// Atomic-free radix bookkeeping.  Every scatter tile w of a segment counts
// its records per digit and writes the row counts[w][0..nd) (tile-major).
// A column scan turns the rows into run bases: the records of digit d from
// tile w go to [offs[w][d], offs[w][d] + counts[w][d]), i.e. after all
// records of smaller digits and after digit d's records of earlier tiles of
// the same segment.  No global atomics are needed (device-scope atomics are
// executed memory-side on gfx950).
// ---------------------------------------------------------------------------
// Tiles per chunk of the level-1 column scan: chosen per pass (scan_chunk on
// the host) so that there are ~192 chunks, i.e. enough workgroups for the
// column sums and applications and few rows for the one-workgroup top scan.

struct TileSpan {
    uint32_t seg, seg_begin, seg_end, begin, cnt;
};

// Segments of a radix pass: nseg segments with offsets seg_off[0..nseg] and
// first tiles tile_first[0..nseg], or (kOne) the one segment [0, n1) passed
// by value, with max(1, ceil(n1 / kTile)) tiles.
// kOne selects the one-segment form at compile time (the first level of a
// pass), so each level gets its own code.
template <int kTile, bool kOne>
__device__ __forceinline__ uint32_t pass_tiles(const uint32_t *tile_first, uint32_t nseg, uint32_t n1) {
    return !kOne ? tile_first[nseg] : max(1u, (n1 + kTile - 1) / kTile);
}

template <int kTile, bool kOne>
__device__ __forceinline__ TileSpan tile_span(const uint32_t *seg_off, const uint32_t *tile_first, uint32_t nseg,
                                              uint32_t n1, uint32_t w) {
    TileSpan ts;
    if (kOne) {
        ts.seg = 0;
        ts.seg_begin = 0;
        ts.seg_end = n1;
        ts.begin = w * kTile;
        ts.cnt = ts.begin < n1 ? min((uint32_t)kTile, n1 - ts.begin) : 0;
        return ts;
    }
    ts.seg = tile_segment(tile_first, nseg, w);
    ts.seg_begin = seg_off[ts.seg];
    ts.seg_end = seg_off[ts.seg + 1];
    ts.begin = ts.seg_begin + (w - tile_first[ts.seg]) * kTile;
    const uint32_t end = min(ts.begin + kTile, ts.seg_end);
    ts.cnt = end > ts.begin ? end - ts.begin : 0;
    return ts;
}

// One workgroup per tile (a grid smaller than the tile count walks the
// tiles grid-stride).
template <int kSrc, int kTile, bool kOne>
__global__ __launch_bounds__(kBlock) void k_tile_counts(const uint32_t *__restrict__ src_idx,
                                                        const unsigned long long *__restrict__ src_key, uint32_t t,
                                                        uint32_t k0, uint32_t k1, int shift, int dbits, uint32_t nseg,
                                                        uint32_t n1, const uint32_t *__restrict__ seg_off,
                                                        const uint32_t *__restrict__ tile_first,
                                                        uint32_t *__restrict__ counts, SrcArgs ba) {
    extern __shared__ uint32_t hs[];
    constexpr int kTileItems = kTile / kBlock;
    const uint32_t nt = pass_tiles<kTile, kOne>(tile_first, nseg, n1);
    const uint32_t nd = 1u << dbits, dmask = nd - 1, tid = threadIdx.x;
    for (uint32_t w = blockIdx.x; w < nt; w += gridDim.x) {
        const TileSpan ts = tile_span<kTile, kOne>(seg_off, tile_first, nseg, n1, w);
        uint32_t cur_i[kTileItems], cur_a[kTileItems];
        unsigned long long cur_k[kTileItems];
        if (src_emits<kSrc>()) {
            emit_tile<kTileItems, kBlock, src_emits_packed<kSrc>(), kSrc == kSrcEmitPackedLocal>(
                ts.begin, ts.cnt, src_idx, src_key, t, k0, k1, ba,
                                                                  cur_i, cur_k);
        } else {
#pragma unroll
            for (int q = 0; q < kTileItems; ++q) {
                const uint32_t p = tid + q * kBlock;
                const bool in = p < ts.cnt;
                cur_i[q] = 0u;
                cur_a[q] = 0u;
                cur_k[q] = kEmptyKey;
                if (kSrc == kSrcHash && in) cur_k[q] = tuple_hash(src_key[ts.begin + p]);
                if ((kSrc == kSrcHashed || kSrc == kSrcPacked) && in) cur_k[q] = src_key[ts.begin + p];
                if (src_reads_idx<kSrc>() && in) cur_i[q] = src_idx[ts.begin + p];
                if (src_reads_aux<kSrc>() && in) cur_a[q] = ba.aux_in[ts.begin + p];
            }
        }
        for (uint32_t d = tid; d < nd; d += kBlock) hs[d] = 0;
        lds_barrier();
#pragma unroll
        for (int q = 0; q < kTileItems; ++q) {
            const uint32_t p = tid + q * kBlock;
            if (!src_emits<kSrc>() && p >= ts.cnt) continue;  // (emit tiles mark missing slots empty)
            if (src_is_tuple<kSrc>() && cur_k[q] == kEmptyKey) continue;
            uint32_t bk = 0;
            const uint64_t word = radix_word<kSrc>(cur_i[q], cur_k[q], cur_a[q], t, k0, k1, ba, &bk);
            atomicAdd(&hs[(uint32_t)(word >> shift) & dmask], 1u);
        }
        lds_barrier();
        for (uint32_t d = tid; d < nd; d += kBlock) counts[(size_t)w * nd + d] = hs[d];
        lds_barrier();
    }
}

// Level-1 column scan, phase 1: per chunk of `chunk` tiles, the column sums.
// Workgroups of min(2^dbits, kBlock) threads.
__global__ __launch_bounds__(kBlock) void k_colsum(const uint32_t *__restrict__ counts, uint32_t ntiles, int dbits,
                                                   uint32_t chunk, uint32_t *__restrict__ partial) {
    const uint32_t nd = 1u << dbits, b = blockIdx.x;
    const uint32_t w0 = b * chunk, w1 = min(w0 + chunk, ntiles);
    for (uint32_t d = threadIdx.x; d < nd; d += blockDim.x) {
        uint32_t acc = 0;
#pragma unroll 8
        for (uint32_t w = w0; w < w1; ++w) acc += counts[(size_t)w * nd + d];
        partial[(size_t)b * nd + d] = acc;
    }
}

// Phase 2 (one workgroup): exclusive scan of the chunk sums per digit, digit
// totals -> digit bases (the coarse offsets), and the level-2 tile map.  With
// fewer digits than threads, kTopThreads / nd threads share a digit's chunk
// rows (contiguous runs, combined through LDS).
constexpr uint32_t kTopThreads = 1024;
__global__ __launch_bounds__(kTopThreads) void k_colscan_top(uint32_t *__restrict__ partial, uint32_t nchunks, int dbits,
                                                        uint32_t *__restrict__ coarse_off,
                                                        uint32_t *__restrict__ tile_first, uint32_t tile) {
    __shared__ uint32_t tot[(1u << kMaxCoarseBits) + 1], tiles[(1u << kMaxCoarseBits) + 1], tmp[kTopThreads / 64 + 1];
    __shared__ uint32_t part[kTopThreads];
    const uint32_t nd = 1u << dbits;
    const uint32_t per_digit = nd >= kTopThreads ? 1u : kTopThreads / nd;  // threads per digit
    const uint32_t rows = (nchunks + per_digit - 1) / per_digit;
    auto scan_rows = [&](uint32_t d, uint32_t r0, uint32_t r1, uint32_t run, bool write) {
        for (uint32_t b0 = r0; b0 < r1; b0 += 16) {
            uint32_t x[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) x[j] = (b0 + j < r1) ? partial[(size_t)(b0 + j) * nd + d] : 0u;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                if (write && b0 + j < r1) partial[(size_t)(b0 + j) * nd + d] = run;
                run += x[j];
            }
        }
        return run;
    };
    if (per_digit == 1) {
        for (uint32_t d = threadIdx.x; d < nd; d += kTopThreads) {
            const uint32_t run = scan_rows(d, 0, nchunks, 0u, true);
            tot[d] = run;
            tiles[d] = (run + tile - 1) / tile;
        }
    } else {
        const uint32_t d = threadIdx.x % nd, j = threadIdx.x / nd;
        const uint32_t r0 = min(j * rows, nchunks), r1 = min(r0 + rows, nchunks);
        part[threadIdx.x] = scan_rows(d, r0, r1, 0u, false);
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (uint32_t q = 0; q < per_digit; ++q) {
            const uint32_t v = part[q * nd + d];
            before += q < j ? v : 0u;
            all += v;
        }
        scan_rows(d, r0, r1, before, true);
        if (j == 0) {
            tot[d] = all;
            tiles[d] = (all + tile - 1) / tile;
        }
    }
    __syncthreads();
    uint32_t total_tiles;
    const uint32_t total = block_exclusive_scan<kTopThreads>(tot, nd, tmp);
    total_tiles = block_exclusive_scan<kTopThreads>(tiles, nd, tmp);
    for (uint32_t d = threadIdx.x; d < nd; d += kTopThreads) {
        coarse_off[d] = tot[d];
        tile_first[d] = tiles[d];
    }
    if (threadIdx.x == 0) {
        coarse_off[nd] = total;
        tile_first[nd] = total_tiles;
    }
}

// Phase 3: run bases of every (tile, digit), in place of the counts
// (workgroups as in phase 1).
__global__ __launch_bounds__(kBlock) void k_colapply(uint32_t *__restrict__ counts, uint32_t ntiles, int dbits,
                                                     uint32_t chunk, const uint32_t *__restrict__ partial,
                                                     const uint32_t *__restrict__ coarse_off) {
    const uint32_t nd = 1u << dbits, b = blockIdx.x;
    const uint32_t w0 = b * chunk, w1 = min(w0 + chunk, ntiles);
    for (uint32_t d = threadIdx.x; d < nd; d += blockDim.x) {
        uint32_t run = coarse_off[d] + partial[(size_t)b * nd + d];
        for (uint32_t wb = w0; wb < w1; wb += 16) {
            uint32_t x[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) x[j] = (wb + j < w1) ? counts[(size_t)(wb + j) * nd + d] : 0u;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                if (wb + j < w1) counts[(size_t)(wb + j) * nd + d] = run;
                run += x[j];
            }
        }
    }
}

// Level-2 scan, one workgroup per coarse segment: sub-bucket totals -> fine
// offsets, then run bases of the segment's tiles (in place of the counts).
// With fewer digits than threads, kBlock / 2^dbits threads share a digit's
// tiles (contiguous runs, combined through LDS).
__global__ __launch_bounds__(kBlock) void k_segscan(uint32_t *__restrict__ counts, int dbits, uint32_t nseg,
                                                    const uint32_t *__restrict__ coarse_off,
                                                    const uint32_t *__restrict__ tile_first,
                                                    uint32_t *__restrict__ fine_off) {
    extern __shared__ uint32_t v[];  // 2^dbits + kBlock + 1
    __shared__ uint32_t part[kBlock];
    uint32_t *tmp = v + (1u << dbits);
    const uint32_t s = blockIdx.x, nd = 1u << dbits, tid = threadIdx.x;
    const uint32_t w0 = tile_first[s], w1 = tile_first[s + 1];
    const uint32_t per_digit = nd >= kBlock ? 1u : kBlock / nd;  // threads per digit
    // thread tid takes digits d = tid % nd (+ kBlock ...) over its share of the tiles
    const uint32_t jrow = tid / nd < per_digit ? tid / nd : 0u;
    const uint32_t rows = w1 - w0, share = (rows + per_digit - 1) / per_digit;
    const uint32_t r0 = w0 + min(jrow * share, rows), r1 = w0 + min(jrow * share + share, rows);
    auto tile_sum = [&](uint32_t d, uint32_t a, uint32_t b) {
        uint32_t acc = 0;
#pragma unroll 8
        for (uint32_t w = a; w < b; ++w) acc += counts[(size_t)w * nd + d];
        return acc;
    };
    auto apply = [&](uint32_t d, uint32_t a, uint32_t b, uint32_t run) {
        for (uint32_t wb = a; wb < b; wb += 16) {
            uint32_t x[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) x[j] = (wb + j < b) ? counts[(size_t)(wb + j) * nd + d] : 0u;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                if (wb + j < b) counts[(size_t)(wb + j) * nd + d] = run;
                run += x[j];
            }
        }
    };
    const uint32_t off = coarse_off[s];
    if (per_digit == 1) {
        for (uint32_t d = tid; d < nd; d += kBlock) v[d] = tile_sum(d, w0, w1);
        __syncthreads();
        block_exclusive_scan(v, nd, tmp);
        for (uint32_t d = tid; d < nd; d += kBlock) {
            fine_off[((size_t)s << dbits) + d] = off + v[d];
            apply(d, w0, w1, off + v[d]);
        }
    } else {
        const uint32_t d = tid % nd;
        part[tid] = tile_sum(d, r0, r1);
        __syncthreads();
        uint32_t before = 0, all = 0;  // this thread's share starts after `before` records of digit d
        for (uint32_t q = 0; q < per_digit; ++q) {
            const uint32_t x = part[q * nd + d];
            before += q < jrow ? x : 0u;
            all += x;
        }
        if (jrow == 0) v[d] = all;
        __syncthreads();
        block_exclusive_scan(v, nd, tmp);
        if (jrow == 0) fine_off[((size_t)s << dbits) + d] = off + v[d];
        apply(d, r0, r1, off + v[d] + before);
    }
    if (s == nseg - 1 && tid == 0) fine_off[(size_t)nseg << dbits] = coarse_off[nseg];
}

// LDS-staged scatter of one tile of a segment by digit (word >> shift) & mask.
// Records of one digit leave the workgroup as one contiguous run starting at
// the run base offs[w][d].  With a tuple source, slots whose key is empty
// are dropped; with kSrcBatch the record's global bucket is written to
// ba.aux_out beside it.  Packed sources move key words only; kSrcEmitPacked
// packs each tuple as it is staged, dropping the dbits digit bits.  One
// workgroup per tile (grid-stride if the grid is smaller).  Dynamic LDS:
// 3 * 2^dbits + kThreads / 64 + 1 words of counters, then the staged records
// (scatter_lds_bytes on the host).

template <int kSrc, int kTile, int kThreads, bool kOne>
__global__ __launch_bounds__(kThreads) void k_scatter(const uint32_t *__restrict__ src_idx,
                                                    const unsigned long long *__restrict__ src_key,
                                                    uint32_t *__restrict__ dst_idx,
                                                    unsigned long long *__restrict__ dst_key, uint32_t t, uint32_t k0,
                                                    uint32_t k1, int shift, int dbits, uint32_t nseg, uint32_t n1,
                                                    const uint32_t *__restrict__ seg_off,
                                                    const uint32_t *__restrict__ tile_first,
                                                    const uint32_t *__restrict__ offs, uint32_t *__restrict__ err,
                                                    SrcArgs ba) {
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t s_total;
    constexpr int kTileItems = kTile / kThreads;
    constexpr uint32_t kScanWords = kThreads / 64 + 1;
    constexpr uint32_t kIdxWords = src_packed<kSrc>() ? 0u : (uint32_t)kTile;
    // second tuple level: a staged word (packed word or tuple hash, moved
    // unchanged) holds its own digit, so none is staged
    constexpr bool kDigitOfWord = kSrc == kSrcPacked || kSrc == kSrcHashed;
    // permutation records whose key has a free top byte carry the digit there
    // (no digit array: 51 KB instead of 59 KB at 4096 records, three
    // workgroups per CU instead of two)
    const bool dik = kSrc == kSrcPerm && ba.dig_in_key != 0;
    constexpr unsigned long long kKeyLow56 = 0x00FFFFFFFFFFFFFFull;
    const uint32_t nd = 1u << dbits, dmask = nd - 1;
    uint32_t *cnt = lds;                 // nd
    uint32_t *start = cnt + nd;          // nd (exclusive scan of cnt)
    uint32_t *base = start + nd;         // nd (global run base)
    uint32_t *tmp = base + nd;           // kThreads / 64 + 1
    uint32_t *s_idx = tmp + kScanWords;  // kTile (none for packed words)
    unsigned long long *s_key =
        reinterpret_cast<unsigned long long *>(s_idx + kIdxWords + ((kScanWords + 3 * nd + kIdxWords) & 1));
    uint16_t *s_dig = reinterpret_cast<uint16_t *>(s_key + kTile);
    uint32_t *s_bkt = reinterpret_cast<uint32_t *>(s_dig + kTile);  // kSrcBatch only

    const uint32_t nt = pass_tiles<kTile, kOne>(tile_first, nseg, n1);
    const uint32_t tid = threadIdx.x;
    for (uint32_t v = blockIdx.x; v < nt; v += gridDim.x) {
        const uint32_t w = xcd_tile(v, nt);
        const TileSpan ts = tile_span<kTile, kOne>(seg_off, tile_first, nseg, n1, w);
        uint32_t c_idx[kTileItems], c_aux[kTileItems];
        unsigned long long c_key[kTileItems];
        if (src_emits<kSrc>()) {
            emit_tile<kTileItems, kThreads, src_emits_packed<kSrc>(), kSrc == kSrcEmitPackedLocal>(
                ts.begin, ts.cnt, src_idx, src_key, t, k0, k1,
                                                                    ba, c_idx, c_key);
        } else {
#pragma unroll
            for (int q = 0; q < kTileItems; ++q) {
                const uint32_t p = tid + q * kThreads;
                const bool in = p < ts.cnt;
                c_idx[q] = (!src_packed<kSrc>() && in) ? src_idx[ts.begin + p] : 0u;
                c_key[q] = in ? src_key[ts.begin + p] : kEmptyKey;
                if (kSrc == kSrcHash) c_key[q] = tuple_hash(c_key[q]);  // empty stays empty
                c_aux[q] = (src_reads_aux<kSrc>() && in) ? ba.aux_in[ts.begin + p] : 0u;
            }
        }
        for (uint32_t d = tid; d < nd; d += kThreads) {
            cnt[d] = 0;
            base[d] = offs[(size_t)w * nd + d];
        }
        if (tid == 0) s_total = 0;
        lds_barrier();
        uint32_t r_dig[kTileItems], r_rank[kTileItems], r_bkt[kTileItems];
#pragma unroll
        for (int q = 0; q < kTileItems; ++q) {
            const uint32_t p = tid + q * kThreads;
            r_dig[q] = 0xFFFFFFFFu;
            r_bkt[q] = 0;
            if ((src_emits<kSrc>() || p < ts.cnt) && (!src_is_tuple<kSrc>() || c_key[q] != kEmptyKey)) {
                const uint64_t word = radix_word<kSrc>(c_idx[q], c_key[q], c_aux[q], t, k0, k1, ba, &r_bkt[q]);
                r_dig[q] = (uint32_t)(word >> shift) & dmask;
                r_rank[q] = atomicAdd(&cnt[r_dig[q]], 1u);
            }
        }
        lds_barrier();
        for (uint32_t d = tid; d < nd; d += kThreads) start[d] = cnt[d];
        lds_barrier();
        block_exclusive_scan<kThreads>(start, nd, tmp);
        uint32_t mine = 0;
#pragma unroll
        for (int q = 0; q < kTileItems; ++q) {
            if (r_dig[q] != 0xFFFFFFFFu) {
                const uint32_t lp = start[r_dig[q]] + r_rank[q];
                if (!src_packed<kSrc>()) s_idx[lp] = c_idx[q];
                // kSrcEmitPacked: the tag code goes below the hash bits left after this level's digit
                if (dik) {
                    s_key[lp] = (c_key[q] & kKeyLow56) | ((unsigned long long)r_dig[q] << 56);
                } else {
                    s_key[lp] = src_emits_packed<kSrc>() ? ((c_key[q] << dbits) | c_idx[q]) : c_key[q];
                    if (!kDigitOfWord) s_dig[lp] = (uint16_t)r_dig[q];
                }
                if (kSrc == kSrcBatch) s_bkt[lp] = r_bkt[q];
                ++mine;
            }
        }
        if (mine) atomicAdd(&s_total, mine);
        lds_barrier();
        const uint32_t staged = s_total;
        for (uint32_t lp = tid; lp < staged; lp += kThreads) {
            const unsigned long long word = s_key[lp];
            const uint32_t d = kDigitOfWord ? (uint32_t)(word >> shift) & dmask
                                            : dik ? (uint32_t)(word >> 56) : (uint32_t)s_dig[lp];
            const uint32_t g = base[d] + (lp - start[d]);
            if (g >= ts.seg_begin && g < ts.seg_end) {
                if (!src_packed<kSrc>()) dst_idx[g] = s_idx[lp];
                dst_key[g] = dik ? word & kKeyLow56 : word;
                if (kSrc == kSrcBatch) ba.aux_out[g] = s_bkt[lp];
            } else {
                atomicOr(err, ERR_INTERNAL);
            }
        }
        lds_barrier();
    }
}

// Sorts each fine bucket by (K, i): LDS counting sort on the kCellBits
// bits of K below the B bucket bits, then ranks within each cell.  One
// workgroup per bucket (grid-stride if the grid is smaller).  Buckets larger
// than `cap` (not expected: the default mean is 3/4 of cap and sizes are
// binomial) take a slow exact path that ranks every record against the whole
// bucket.  Dynamic LDS: 2^kCellBits cell counters + kBlock + 2 scan words
// + cap * 20 bytes.
__global__ __launch_bounds__(kBlock) void k_sort_buckets(const uint32_t *__restrict__ src_idx,
                                                         const unsigned long long *__restrict__ src_key,
                                                         uint32_t *__restrict__ dst_idx,
                                                         unsigned long long *__restrict__ dst_key,
                                                         unsigned long long *__restrict__ scratch_k, uint32_t t,
                                                         uint32_t k0, uint32_t k1, int bbits,
                                                         const uint32_t *__restrict__ fine_off, uint32_t nb,
                                                         uint32_t m, uint32_t cap, StepCounters *__restrict__ ctr,
                                                         const BatchGraph *__restrict__ gr, uint32_t ngraphs,
                                                         uint32_t step) {
    extern __shared__ uint32_t lds[];
    constexpr uint32_t kCells = 1u << kCellBits;
    uint32_t *cell = lds;                    // kCells
    uint32_t *tmp = cell + kCells;           // kBlock + 1 (+1 pad for 8-byte alignment)
    unsigned long long *sK = reinterpret_cast<unsigned long long *>(tmp + kBlock + 2);
    unsigned long long *sE = sK + cap;
    uint32_t *sI = reinterpret_cast<uint32_t *>(sE + cap);
    const uint32_t tid = threadIdx.x;
    const int sub_shift = 64 - kCellBits;
    const uint32_t lds_cap = min(cap, (uint32_t)(kSortMaxItems * kBlock));

    for (uint32_t f = blockIdx.x; f < nb; f += gridDim.x) {
        const uint32_t begin = min(fine_off[f], m), end = min(fine_off[f + 1], m);
        uint32_t c_idx[kSortMaxItems];
        unsigned long long c_key[kSortMaxItems];
#pragma unroll
        for (int q = 0; q < kSortMaxItems; ++q) {
            const uint32_t p = begin + tid + q * kBlock;
            c_idx[q] = p < end ? src_idx[p] : 0u;
            c_key[q] = p < end ? src_key[p] : 0ull;
        }
        const uint32_t c = end > begin ? end - begin : 0;
        // batch: the graph owning bucket f (largest g with bbase <= f); its
        // buckets split the high word of K by fast range reduction, so the
        // cell is the top of the remainder of that reduction
        BatchGraph bg{};
        if (gr && c > 0) {
            uint32_t lo = 0, hi = ngraphs - 1;
            while (lo < hi) {
                const uint32_t mid = (lo + hi + 1) >> 1;
                if (gr[mid].bbase <= f)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            bg = gr[lo];
        }
        auto key_of = [&](uint32_t idx) -> uint64_t {
            return gr ? batch_perm_key(bg, idx, step) : perm_key(idx, t, k0, k1);
        };
        auto cell_of = [&](uint64_t K) -> uint32_t {
            if (gr) return ((uint32_t)((K >> 32) * (uint64_t)bg.nb)) >> (32 - kCellBits);
            return (uint32_t)((bbits >= 64 ? 0ull : (K << bbits)) >> sub_shift);
        };
        if (c > lds_cap) {
            // exact slow path: rank_p = #{q : (K_q, i_q) < (K_p, i_p)}
            for (uint32_t p = tid; p < c; p += kBlock) scratch_k[begin + p] = key_of(src_idx[begin + p]);
            __threadfence_block();
            __syncthreads();
            for (uint32_t p = tid; p < c; p += kBlock) {
                const unsigned long long kp = scratch_k[begin + p];
                const uint32_t ip = src_idx[begin + p];
                uint32_t rank = 0;
                for (uint32_t q = 0; q < c; ++q) {
                    const unsigned long long kq = scratch_k[begin + q];
                    const uint32_t iq = src_idx[begin + q];
                    rank += (kq < kp) || (kq == kp && iq < ip);
                }
                dst_idx[begin + rank] = ip;
                dst_key[begin + rank] = src_key[begin + p];
            }
            if (tid == 0) atomicAdd(&ctr->fallback_buckets, 1ull);
            __syncthreads();
        } else if (c > 0) {
            for (uint32_t q = tid; q < kCells; q += kBlock) cell[q] = 0;
            lds_barrier();
            uint32_t r_cell[kSortMaxItems], r_rank[kSortMaxItems];
            unsigned long long r_K[kSortMaxItems];
#pragma unroll
            for (int q = 0; q < kSortMaxItems; ++q) {
                const uint32_t p = tid + q * kBlock;
                if (p < c) {
                    r_K[q] = key_of(c_idx[q]);
                    r_cell[q] = cell_of(r_K[q]);
                    r_rank[q] = atomicAdd(&cell[r_cell[q]], 1u);
                }
            }
            lds_barrier();
            block_exclusive_scan(cell, kCells, tmp);
#pragma unroll
            for (int q = 0; q < kSortMaxItems; ++q) {
                const uint32_t p = tid + q * kBlock;
                if (p < c) {
                    const uint32_t lp = cell[r_cell[q]] + r_rank[q];
                    sK[lp] = r_K[q];
                    sI[lp] = c_idx[q];
                }
            }
            lds_barrier();
            // order within a cell: the keys (K_i, i) are distinct, so an item's
            // place is the number of smaller ones in its cell (independent
            // LDS loads, no insertion sort)
            uint32_t r_pos[kSortMaxItems];
#pragma unroll
            for (int q = 0; q < kSortMaxItems; ++q) {
                const uint32_t p = tid + q * kBlock;
                if (p >= c) continue;
                const uint32_t cl = r_cell[q];
                const uint32_t a = cell[cl], b = (cl + 1 < kCells) ? cell[cl + 1] : c;
                const unsigned long long kx = r_K[q];
                const uint32_t ix = c_idx[q];
                uint32_t rank = 0;
                for (uint32_t y = a; y < b; ++y) {
                    const unsigned long long ky = sK[y];
                    rank += ky < kx || (ky == kx && sI[y] < ix);
                }
                r_pos[q] = a + rank;
            }
            lds_barrier();
#pragma unroll
            for (int q = 0; q < kSortMaxItems; ++q) {
                const uint32_t p = tid + q * kBlock;
                if (p < c) {
                    sE[r_pos[q]] = c_key[q];
                    sI[r_pos[q]] = c_idx[q];
                }
            }
            lds_barrier();
            for (uint32_t p = tid; p < c; p += kBlock) {
                dst_idx[begin + p] = sI[p];
                dst_key[begin + p] = sE[p];
            }
            lds_barrier();
        }
    }
}

// Philox permutation keys K_i for i in [0, m) (building block exposed for
// step-level checks).
__global__ __launch_bounds__(kBlock) void k_perm_keys(uint32_t m, uint32_t t, uint32_t k0, uint32_t k1,
                                                      unsigned long long *__restrict__ out) {
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < m) out[i] = perm_key((uint32_t)i, t, k0, k1);
}

}  // namespace gesmc

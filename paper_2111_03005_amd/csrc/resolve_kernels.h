// Dependency resolution of a global switch by sorting (edge key, tag) tuples
// by edge key -- an HBM-atomic-free form of Alg. 1's dependency table T.
//
// Every switch k that survives its local checks emits four tuples: an ERASE
// tuple for each source edge (Def. 3.1 / Alg. 1 "erase") and an INSERT tuple
// for each target edge ("insert"); a switch rejected locally (loop, a target
// equal to one of its own sources, P_L) and the idle position of odd m emit
// ERASE tuples marked STAYS (those edges survive the superstep).  Tuples are
// partitioned by a hash of the key with the same LDS-staged radix scatter as
// the permutation (its first pass computes them from the pair records, see
// emit_switch), so all tuples of one key meet in one workgroup, which
// sorts its partition in LDS and derives for every INSERT tuple (k, X):
//   eraser(X)  : the switch whose source X is (or STAYS / none)   -- lookup
//   pred(k, X) : the next smaller inserter of X                    -- the
//                chain behind lookup_min over non-illegal inserters.
// Only tuples with an eraser or a predecessor write their record (rare); all
// other records keep the "free" value written by the emit (k_emit or
// k_emit_counts).
//
// Decision of switch k (same rule as Alg. 1): illegal if a target is erased
// by a later switch / stays / is erased by an illegal switch, or if an
// earlier inserter of a target is legal; delayed if it depends on an
// undecided switch; else legal.  The predecessor chain of (k, X) lists every
// earlier inserter of X from the nearest down, so walking it until a legal
// (-> illegal) or undecided (-> delayed) switch, or its end (-> free),
// evaluates "no earlier legal inserter of X".
#pragma once

#include "device_common.h"
#include "perm_kernels.h"
#include "switch_kernels.h"

namespace gesmc {

// per-target record: x = eraser (kNoEraser / kStays / switch), y = predecessor (k' << 1 | h') or kNoPred
constexpr uint32_t kNoPred = 0xFFFFFFFFu;
constexpr uint32_t kWalked = 0xFFFFFFFEu;  // a resumed walk that reached the chain's end
constexpr uint32_t kListEnd = 0xFFFFu;  // end of a cell list in k_resolve (slots are < 2^16)
constexpr uint32_t kEpochNone = 0xFFFFu;  // k_resolve: no list partition yet (epochs are 0 .. 0xFFFE)
#ifndef GESMC_RESOLVE_LISTS
#define GESMC_RESOLVE_LISTS 1
#endif
static_assert(kLdsCap < kListEnd, "k_resolve slots fit 16 bits");

// ---------------------------------------------------------------------------
// Emit: one thread per switch (+ one for the idle record of odd m).  The
// local outcome of every switch (switch_local) goes to its status; a switch
// decided locally also gets its records (unchanged) and its count, an
// undecided one its two target records initialised to "free".  Workgroup 0
// clears the undecided-list counters of the rounds that follow.  This kernel
// serves the unfused schedule; by default the same work runs inside the
// first tuple count pass (k_emit_counts below), and the switches' tuples are
// never stored: the first partition pass computes them from the same pair
// records (emit_switch).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_emit(const uint32_t *__restrict__ s_idx,
                                                 const unsigned long long *__restrict__ s_key, uint32_t t, uint32_t k0,
                                                 uint32_t k1, SrcArgs sa, uint2 *__restrict__ info,
                                                 uint8_t *__restrict__ st, uint32_t *__restrict__ out_idx,
                                                 unsigned long long *__restrict__ out_key, uint4 *__restrict__ bslot,
                                                 uint32_t *__restrict__ ucount) {
    __shared__ BlockCounts bc;
    const uint32_t tid = threadIdx.x;
    if (tid == 0) bc = BlockCounts{0, 0, 0, 0};
    if (blockIdx.x == 0 && tid < 3) ucount[tid] = 0;  // the undecided-list counters of the rounds
    __syncthreads();
    const uint32_t m = sa.m, ell = m >> 1;
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t k = blockIdx.x * kBlock + tid; k <= ell; k += stride) {
        if (k == ell) {
            if (m & 1u) {
                out_idx[m - 1] = s_idx[m - 1];
                out_key[m - 1] = s_key[m - 1];
            }
            continue;
        }
        const uint2 ij = reinterpret_cast<const uint2 *>(s_idx)[k];
        const ulonglong2 ee = reinterpret_cast<const ulonglong2 *>(s_key)[k];
        Targets T{0, 0, false};
        const uint8_t status = switch_local(k, ij, ee, t, k0, k1, sa, &T);
        st[k] = status;
        if (status == ST_UNDECIDED) {
            reinterpret_cast<uint4 *>(info)[k] = make_uint4(kNoEraser, kNoPred, kNoEraser, kNoPred);
        } else {
            reinterpret_cast<uint2 *>(out_idx)[k] = ij;
            reinterpret_cast<ulonglong2 *>(out_key)[k] = ee;
            if (status == ST_PL) atomicAdd(&bc.pl, 1u);
            if (status == ST_LOOP) atomicAdd(&bc.loop, 1u);
            if (status == ST_EXISTS) atomicAdd(&bc.exists, 1u);
        }
    }
    store_counts(&bc, bslot + blockIdx.x);
}

// A superstep of a multi-edge class (Sec. 1): no target is rejected for
// being present, so each switch's outcome follows from its own pair records
// alone (P_L skip, else a loop where loops are not allowed, else legal) and
// the whole superstep is decided here, one thread per switch plus one for
// the idle record of odd m.  Writes every record of buffer 0, the status
// array and the superstep's counts.
__global__ __launch_bounds__(kBlock) void k_decide_local(const uint32_t *__restrict__ s_idx,
                                                         const unsigned long long *__restrict__ s_key, uint32_t m,
                                                         uint32_t t, uint32_t k0, uint32_t k1, uint32_t pl,
                                                         uint32_t cls, uint8_t *__restrict__ st,
                                                         uint32_t *__restrict__ out_idx,
                                                         unsigned long long *__restrict__ out_key,
                                                         StepCounters *ctr) {
    __shared__ BlockCounts bc;
    if (threadIdx.x == 0) bc = BlockCounts{0, 0, 0, 0};
    __syncthreads();
    const uint32_t ell = m >> 1;
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k <= ell; k += stride) {
        if (k == ell) {
            if (m & 1u) {
                out_idx[m - 1] = s_idx[m - 1];
                out_key[m - 1] = s_key[m - 1];
            }
            continue;
        }
        const uint2 ij = reinterpret_cast<const uint2 *>(s_idx)[k];
        const ulonglong2 ee = reinterpret_cast<const ulonglong2 *>(s_key)[k];
        uint8_t status = ST_LEGAL;
        ulonglong2 out = ee;
        if (pl_skip(k, t, pl, k0, k1)) {
            status = ST_PL;
        } else {
            const Targets T = switch_targets_cls(ee.x, ee.y, ij.x < ij.y, cls);
            if (T.loop)
                status = ST_LOOP;
            else
                out = make_ulonglong2(T.A, T.B);
        }
        st[k] = status;
        reinterpret_cast<uint2 *>(out_idx)[k] = ij;
        reinterpret_cast<ulonglong2 *>(out_key)[k] = out;
        if (status == ST_LEGAL) atomicAdd(&bc.legal, 1u);
        if (status == ST_LOOP) atomicAdd(&bc.loop, 1u);
        if (status == ST_PL) atomicAdd(&bc.pl, 1u);
    }
    flush_counts(&bc, ctr);
}

// k_emit fused into the first tuple partition pass's counts (kSrcEmit or
// kSrcEmitPacked, one segment [0, nslots) of kTile-slot tiles): the pair
// records of a switch are read once, for its status, its records and
// counts (as k_emit) and for its four tuples' digit counts (as
// k_tile_counts).  Tiles are taken grid-stride; each workgroup stores its
// outcome counts in bslot[blockIdx.x].  The per-tile digit counts equal
// k_tile_counts' (the same tiles, tuples and radix words).
template <int kSrc, int kTile>
__global__ __launch_bounds__(kBlock) void k_emit_counts(const uint32_t *__restrict__ s_idx,
                                                        const unsigned long long *__restrict__ s_key, uint32_t t,
                                                        uint32_t k0, uint32_t k1, int shift, int dbits, uint32_t nslots,
                                                        uint32_t *__restrict__ counts, SrcArgs sa,
                                                        uint2 *__restrict__ info, uint8_t *__restrict__ st,
                                                        uint32_t *__restrict__ out_idx,
                                                        unsigned long long *__restrict__ out_key,
                                                        uint4 *__restrict__ bslot, uint32_t *__restrict__ ucount) {
    static_assert(src_emits<kSrc>(), "tuples emitted from the pair records");
    extern __shared__ uint32_t hs[];
    __shared__ BlockCounts bc;
    constexpr int kSwitches = kTile / kBlock / 4;  // switches per thread and tile
    constexpr bool kPacked = src_emits_packed<kSrc>();
    const uint32_t nt = max(1u, (nslots + kTile - 1) / kTile);
    const uint32_t nd = 1u << dbits, dmask = nd - 1, tid = threadIdx.x;
    const uint32_t m = sa.m, ell = m >> 1;
    if (tid == 0) bc = BlockCounts{0, 0, 0, 0};
    if (blockIdx.x == 0 && tid < 3) ucount[tid] = 0;  // the undecided-list counters of the rounds
    for (uint32_t w = blockIdx.x; w < nt; w += gridDim.x) {
        const uint32_t begin = w * kTile;
        const uint32_t cnt = begin < nslots ? min((uint32_t)kTile, nslots - begin) : 0u;
        for (uint32_t d = tid; d < nd; d += kBlock) hs[d] = 0;
        lds_barrier();
#pragma unroll
        for (int j = 0; j < kSwitches; ++j) {
            const uint32_t sl = 4 * (tid + j * kBlock);  // first local slot of this thread's switch
            Tuple tp[4] = {{0u, kEmptyKey}, {0u, kEmptyKey}, {0u, kEmptyKey}, {0u, kEmptyKey}};
            if (sl < cnt) {
                const uint32_t k = (begin + sl) >> 2;
                if (k < ell) {
                    const uint2 ij = reinterpret_cast<const uint2 *>(s_idx)[k];
                    const ulonglong2 ee = reinterpret_cast<const ulonglong2 *>(s_key)[k];
                    Targets T{0, 0, false};
                    const uint8_t status = switch_local(k, ij, ee, t, k0, k1, sa, &T);
                    st[k] = status;
                    if (status == ST_UNDECIDED) {
                        reinterpret_cast<uint4 *>(info)[k] = make_uint4(kNoEraser, kNoPred, kNoEraser, kNoPred);
                    } else {
                        reinterpret_cast<uint2 *>(out_idx)[k] = ij;
                        reinterpret_cast<ulonglong2 *>(out_key)[k] = ee;
                        if (status == ST_PL) atomicAdd(&bc.pl, 1u);
                        if (status == ST_LOOP) atomicAdd(&bc.loop, 1u);
                        if (status == ST_EXISTS) atomicAdd(&bc.exists, 1u);
                    }
                    switch_tuples(k, ij, ee, status, T, tp);
                } else if (k == ell && (m & 1u)) {  // the idle record of odd m stays
                    out_idx[m - 1] = s_idx[m - 1];
                    out_key[m - 1] = s_key[m - 1];
                    tp[0] = Tuple{kTagStays, s_key[m - 1]};
                }
            }
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                if (sl + h >= cnt) continue;
                const unsigned long long word = emitted_word<kPacked>(tp[h].key, sa);
                if (word != kEmptyKey) atomicAdd(&hs[(uint32_t)(word >> shift) & dmask], 1u);
            }
        }
        lds_barrier();
        for (uint32_t d = tid; d < nd; d += kBlock) counts[(size_t)w * nd + d] = hs[d];
        lds_barrier();
    }
    store_counts(&bc, bslot + blockIdx.x);
}

// The tuples of every slot written out flat (tuple buffer 0), for the
// unfused schedule (GESMC_OPT_FUSE_EMIT 0): one thread per switch.
__global__ __launch_bounds__(kBlock) void k_emit_tuples(const uint32_t *__restrict__ s_idx,
                                                        const unsigned long long *__restrict__ s_key, uint32_t t,
                                                        uint32_t k0, uint32_t k1, SrcArgs sa, uint32_t nslots,
                                                        uint32_t *__restrict__ tu_tag,
                                                        unsigned long long *__restrict__ tu_key) {
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; 4 * (uint64_t)k < nslots; k += stride) {
        Tuple tp[4];
        emit_switch(k, s_idx, s_key, t, k0, k1, sa, tp);
        for (uint32_t h = 0; h < 4 && 4 * k + h < nslots; ++h) {
            tu_tag[4 * k + h] = tp[h].tag;
            tu_key[4 * k + h] = tp[h].key;
        }
    }
}

// Validation only (no superstep): one STAYS tuple per input edge, so that a
// duplicate edge shows up as two ERASE tuples of one key.
__global__ __launch_bounds__(kBlock) void k_emit_sources(const unsigned long long *__restrict__ key, uint32_t m,
                                                         uint32_t *__restrict__ tu_tag,
                                                         unsigned long long *__restrict__ tu_key) {
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < m; i += gridDim.x * kBlock) {
        tu_tag[i] = kTagStays;
        tu_key[i] = key[i];
    }
}

// Graph attribution of errors in a batch: the graph owning a key is the one
// whose vertex range holds its smaller endpoint.
struct GraphErr {
    const BatchGraph *gr;  // nullptr: no attribution
    uint32_t ngraphs;
    uint32_t *gerr;        // per graph error bits
};

// `key` is a tuple hash, or (pk.w > 0) a packed word with its tag code
// cleared; f is the tuple's partition, whose first-level digit restores the
// hash bits the packed word dropped.
// The rank of the graph holding the key of a tuple of fine partition f
// (ge.gr must be set): its smaller endpoint, by inverting the hash with the
// first level's digit restored, then the graph whose vertex range holds it.
__device__ __forceinline__ uint32_t graph_of_tuple(unsigned long long key, uint32_t f, const TuplePack &pk,
                                                   const GraphErr &ge) {
    uint32_t v;
    if (pk.w) {
        const uint64_t h = ((uint64_t)(f >> pk.b2) << (pk.w - pk.b1)) | (key >> (64 - pk.w + pk.b1));
        v = key_hash_w_vertex(h, pk.db, pk.w);
    } else {
        v = (uint32_t)(tuple_key_of(key) >> 32);
    }
    uint32_t lo = 0, hi = ge.ngraphs - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (ge.gr[mid].vbase <= v)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ void flag_duplicate(unsigned long long key, uint32_t f, const TuplePack &pk, uint32_t *err,
                                               uint32_t dup_bit, const GraphErr &ge) {
    if (dup_bit) atomicOr(err, dup_bit);
    if (ge.gr) atomicOr(&ge.gerr[graph_of_tuple(key, f, pk, ge)], ERR_DUP);
}

// Writes the records of the tuple at sorted position p, given the position
// of the first tuple of its key.  A second ERASE tuple means the edge occurs
// twice: dup_bit is raised (and the graph flagged in a batch).
__device__ __forceinline__ void resolve_one(uint32_t tag, uint32_t first_tag, uint32_t p, uint32_t first,
                                            uint32_t prev_tag, unsigned long long key, uint32_t f,
                                            const TuplePack &pk, uint2 *info, uint32_t *err, uint32_t dup_bit,
                                            const GraphErr &ge) {
    const bool ins = (tag & kTagInsert) != 0;
    if (!ins) {
        if (p != first) flag_duplicate(key, f, pk, err, dup_bit, ge);
        return;
    }
    uint32_t eraser = kNoEraser;
    if (!(first_tag & kTagInsert)) eraser = (first_tag == kTagStays) ? kStays : first_tag;
    uint32_t pred = (p > first && (prev_tag & kTagInsert)) ? (prev_tag & ~kTagInsert) : kNoPred;
    if (eraser == kNoEraser && pred == kNoPred) return;
    uint32_t slot = tag & ~kTagInsert;
    if (pk.local) {  // graph-local tags (all of one key): back to batch-wide switch ids
        const uint32_t kbase = ge.gr[graph_of_tuple(key, f, pk, ge)].poff >> 1;
        slot += 2 * kbase;
        if (eraser != kStays && eraser != kNoEraser) eraser += kbase;
        if (pred != kNoPred) pred += 2 * kbase;
    }
    info[slot] = make_uint2(eraser, pred);
}

// One workgroup per fine partition (grid-stride if the grid is smaller).
// LDS path: counting sort on kCellBits hash bits below the partition bits;
// each tuple then reads its own cell.  Partitions above `cap` (hub
// keys with many inserters) take an exact global-memory merge sort.
// Dynamic LDS: 2^kCellBits cell words + kBlock + 2 words + cap * 14 bytes
// (keys, tags and the 16-bit cell-list links), or cap * 10 bytes for packed
// words with the cell lists (the tags stay in the words).  kPacked: the tuples are
// packed words (no tag array); pbits is then the second level's bits only,
// the first level's having been dropped from the words.
template <bool kPacked>
__global__ __launch_bounds__(kBlock) void k_resolve(uint32_t *__restrict__ tu_tag, unsigned long long *__restrict__ tu_key,
                                                    uint32_t *__restrict__ sc_tag,
                                                    unsigned long long *__restrict__ sc_key, int pbits,
                                                    const uint32_t *__restrict__ part_off, uint32_t np, uint32_t cap,
                                                    uint2 *__restrict__ info, uint32_t *__restrict__ err,
                                                    uint32_t dup_bit, StepCounters *ctr, GraphErr ge, TuplePack pk) {
    extern __shared__ uint32_t lds[];
    constexpr uint32_t kCells = 1u << kCellBits;
    uint32_t *cell = lds;
    uint32_t *tmp = cell + kCells;
    unsigned long long *sK = reinterpret_cast<unsigned long long *>(tmp + kBlock + 2);
    uint32_t *sT = reinterpret_cast<uint32_t *>(sK + cap);
    const uint32_t tid = threadIdx.x;
    const int sub_shift = 64 - kCellBits;
    const uint32_t lds_cap = min(cap, (uint32_t)(kSortMaxItems * kBlock));
    const uint64_t code_mask = kPacked ? low_mask(pk.kb + 1) : 0ull;

    // cell lists: each cell word is (epoch << 16) | head slot, where the
    // epoch counts this workgroup's list-resolved partitions; a word of an
    // older epoch is an empty list, so no partition clears the cells
    uint32_t epoch = kEpochNone;
    // partition g's tuples (raw packed words, decoded at their first use)
    uint32_t c_tag[kSortMaxItems];
    unsigned long long c_key[kSortMaxItems];
    uint32_t begin = 0, end = 0;
    auto load_part = [&](uint32_t g) {
        begin = part_off[g];
        end = part_off[g + 1];
#pragma unroll
        for (int q = 0; q < kSortMaxItems; ++q) {
            const uint32_t p = begin + tid + q * kBlock;
            c_tag[q] = (!kPacked && p < end) ? tu_tag[p] : 0u;
            c_key[q] = p < end ? tu_key[p] : 0ull;
        }
    };
    if (blockIdx.x < np) load_part(blockIdx.x);
    for (uint32_t f = blockIdx.x; f < np; f += gridDim.x) {
        const uint32_t c = end > begin ? end - begin : 0;
        if (kPacked && c > lds_cap) {
            // exact slow path over packed words: their order is (key, tag)
            // order, so a merge sort of the words is the sort by (key, tag)
            unsigned long long *ak = tu_key + begin, *bk = sc_key + begin;
            for (uint32_t width = 1; width < c; width <<= 1) {
                for (uint32_t p = tid; p < c; p += kBlock) {
                    const uint32_t run = p / (2 * width);
                    const uint32_t lo = run * 2 * width, mid = min(lo + width, c), hi = min(lo + 2 * width, c);
                    const unsigned long long kp = ak[p];
                    uint32_t pos;
                    if (p < mid) {  // rank among the right run: words strictly smaller
                        uint32_t a = mid, b = hi;
                        while (a < b) {
                            const uint32_t x = (a + b) >> 1;
                            if (ak[x] < kp)
                                a = x + 1;
                            else
                                b = x;
                        }
                        pos = lo + (p - lo) + (a - mid);
                    } else {  // rank among the left run: words smaller or equal
                        uint32_t a = lo, b = mid;
                        while (a < b) {
                            const uint32_t x = (a + b) >> 1;
                            if (ak[x] <= kp)
                                a = x + 1;
                            else
                                b = x;
                        }
                        pos = lo + (p - mid) + (a - lo);
                    }
                    bk[pos] = kp;
                }
                __threadfence_block();
                __syncthreads();
                unsigned long long *xk = ak;
                ak = bk;
                bk = xk;
            }
            for (uint32_t p = tid; p < c; p += kBlock) {
                const unsigned long long kp = ak[p] & ~code_mask;
                uint32_t a = 0, b = p;
                while (a < b) {
                    const uint32_t x = (a + b) >> 1;
                    if ((ak[x] & ~code_mask) < kp)
                        a = x + 1;
                    else
                        b = x;
                }
                const auto tag_at = [&](uint32_t x) { return tag_of_code((uint32_t)(ak[x] & code_mask), pk.kb); };
                resolve_one(tag_at(p), tag_at(a), p, a, p > 0 ? tag_at(p - 1) : 0u, kp, f, pk, info, err, dup_bit,
                            ge);
            }
            if (tid == 0) atomicAdd(&ctr->fallback_buckets, 1ull);
            __syncthreads();
        } else if (c > lds_cap) {
            // exact slow path: bottom-up merge sort by (key, tag) between the
            // partition's range and the scratch range, then binary searches.
            uint32_t *at = tu_tag + begin, *bt = sc_tag + begin;
            unsigned long long *ak = tu_key + begin, *bk = sc_key + begin;
            for (uint32_t width = 1; width < c; width <<= 1) {
                for (uint32_t p = tid; p < c; p += kBlock) {
                    const uint32_t run = p / (2 * width);
                    const uint32_t lo = run * 2 * width, mid = min(lo + width, c), hi = min(lo + 2 * width, c);
                    const unsigned long long kp = ak[p];
                    const uint32_t tp = at[p];
                    uint32_t pos;
                    if (p < mid) {  // rank among the right run: elements strictly smaller
                        uint32_t a = mid, b = hi;
                        while (a < b) {
                            const uint32_t x = (a + b) >> 1;
                            if (ak[x] < kp || (ak[x] == kp && at[x] < tp))
                                a = x + 1;
                            else
                                b = x;
                        }
                        pos = lo + (p - lo) + (a - mid);
                    } else {  // rank among the left run: elements smaller or equal
                        uint32_t a = lo, b = mid;
                        while (a < b) {
                            const uint32_t x = (a + b) >> 1;
                            if (ak[x] < kp || (ak[x] == kp && at[x] <= tp))
                                a = x + 1;
                            else
                                b = x;
                        }
                        pos = lo + (p - mid) + (a - lo);
                    }
                    bt[pos] = tp;
                    bk[pos] = kp;
                }
                __threadfence_block();
                __syncthreads();
                uint32_t *xt = at;
                at = bt;
                bt = xt;
                unsigned long long *xk = ak;
                ak = bk;
                bk = xk;
            }
            for (uint32_t p = tid; p < c; p += kBlock) {
                const unsigned long long kp = ak[p];
                uint32_t a = 0, b = p;
                while (a < b) {
                    const uint32_t x = (a + b) >> 1;
                    if (ak[x] < kp)
                        a = x + 1;
                    else
                        b = x;
                }
                resolve_one(at[p], at[a], p, a, p > 0 ? at[p - 1] : 0u, kp, f, pk, info, err, dup_bit, ge);
            }
            if (tid == 0) atomicAdd(&ctr->fallback_buckets, 1ull);
            __syncthreads();
        } else if (c > 0 && GESMC_RESOLVE_LISTS) {
            // Tuples stay in their own slots p (contiguous writes); each cell
            // keeps a list of its slots, linked by one LDS exchange per tuple.
            // Packed words stay whole in sK (key bits and tag code), with no
            // tag array: 10 bytes of LDS per tuple instead of 14.
            uint16_t *nxt = reinterpret_cast<uint16_t *>(kPacked ? reinterpret_cast<uint32_t *>(sK + cap) : sT + cap);
            if (epoch >= kEpochNone - 1) {  // first list partition, or the epochs wrap: every list empty
                for (uint32_t q = tid; q < kCells; q += kBlock) cell[q] = 0xFFFFFFFFu;
                lds_barrier();
                epoch = 0;
            } else {
                ++epoch;
            }
            const uint32_t ep = epoch << 16;
            uint32_t r_cell[kSortMaxItems];
#pragma unroll
            for (int q = 0; q < kSortMaxItems; ++q) {
                const uint32_t p = tid + q * kBlock;
                if (p < c) {
                    const unsigned long long raw = c_key[q];
                    if (kPacked) {  // the key bits stay in place (cells, equality); the code is the tag
                        c_tag[q] = tag_of_code((uint32_t)(raw & code_mask), pk.kb);
                        c_key[q] = raw & ~code_mask;
                    }
                    const uint64_t hsh = c_key[q];  // tuple words are tuple hashes
                    r_cell[q] = (uint32_t)((pbits >= 64 ? 0ull : (hsh << pbits)) >> sub_shift);
                    sK[p] = raw;
                    if (!kPacked) sT[p] = c_tag[q];
                    const uint32_t old = atomicExch(&cell[r_cell[q]], ep | p);
                    nxt[p] = (old & 0xFFFF0000u) == ep ? (uint16_t)old : (uint16_t)kListEnd;
                }
            }
            lds_barrier();
            // All tuples of one key share a cell.  Each tuple walks its cell's
            // list for what the walk over the sorted group would give: the
            // group's smallest tag, whether a tuple precedes it in (key, tag,
            // slot) order and the largest preceding tag.
#pragma unroll
            for (int q = 0; q < kSortMaxItems; ++q) {
                const uint32_t p = tid + q * kBlock;
                if (p >= c) continue;
                const unsigned long long kx = c_key[q];
                const uint32_t tx = c_tag[q];
                uint32_t first_tag = tx, prev_tag = 0;
                bool before = false;
                for (uint32_t y = cell[r_cell[q]] & 0xFFFFu; y != kListEnd; y = nxt[y]) {
                    const unsigned long long wy = sK[y];
                    if (y == p || (kPacked ? (wy & ~code_mask) : wy) != kx) continue;
                    const uint32_t ty = kPacked ? tag_of_code((uint32_t)(wy & code_mask), pk.kb) : sT[y];
                    first_tag = min(first_tag, ty);
                    if (ty < tx || (ty == tx && y < p)) {
                        prev_tag = before ? max(prev_tag, ty) : ty;
                        before = true;
                    }
                }
                resolve_one(tx, first_tag, before ? 1u : 0u, 0u, prev_tag, kx, f, pk, info, err, dup_bit, ge);
            }
        } else if (c > 0) {  // counting sort into cell order
            for (uint32_t q = tid; q < kCells; q += kBlock) cell[q] = 0;
            lds_barrier();
            uint32_t r_cell[kSortMaxItems], r_rank[kSortMaxItems];
#pragma unroll
            for (int q = 0; q < kSortMaxItems; ++q) {
                const uint32_t p = tid + q * kBlock;
                if (p < c) {
                    if (kPacked) {
                        c_tag[q] = tag_of_code((uint32_t)(c_key[q] & code_mask), pk.kb);
                        c_key[q] &= ~code_mask;
                    }
                    const uint64_t hsh = c_key[q];  // tuple words are tuple hashes
                    r_cell[q] = (uint32_t)((pbits >= 64 ? 0ull : (hsh << pbits)) >> sub_shift);
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
                    sK[lp] = c_key[q];
                    sT[lp] = c_tag[q];
                }
            }
            lds_barrier();
            // All tuples of one key share a cell.  Each tuple reads its cell
            // (independent LDS loads, no sorting) for what the walk over the
            // sorted group would give: the group's smallest tag, whether a
            // tuple precedes it in (key, tag, slot) order and the largest
            // preceding tag.
#pragma unroll
            for (int q = 0; q < kSortMaxItems; ++q) {
                const uint32_t p = tid + q * kBlock;
                if (p >= c) continue;
                const uint32_t cl = r_cell[q];
                const uint32_t a = cell[cl], b = (cl + 1 < kCells) ? cell[cl + 1] : c;
                const uint32_t me = a + r_rank[q];
                const unsigned long long kx = c_key[q];
                const uint32_t tx = c_tag[q];
                uint32_t first_tag = tx, prev_tag = 0;
                bool before = false;
                for (uint32_t y = a; y < b; ++y) {
                    if (y == me || sK[y] != kx) continue;
                    const uint32_t ty = sT[y];
                    first_tag = min(first_tag, ty);
                    if (ty < tx || (ty == tx && y < me)) {
                        prev_tag = before ? max(prev_tag, ty) : ty;
                        before = true;
                    }
                }
                resolve_one(tx, first_tag, before ? 1u : 0u, 0u, prev_tag, kx, f, pk, info, err, dup_bit, ge);
            }
        }
        // the next partition's loads are issued before the barrier that ends
        // this one (every walk done before the cells are linked again), so
        // they are in flight while the slowest wave finishes
        if (f + gridDim.x < np) load_part(f + gridDim.x);
        lds_barrier();
    }
}

// ---------------------------------------------------------------------------
// Decisions
// ---------------------------------------------------------------------------
// Two shortcuts keep long chains (many switches inserting one hub edge)
// linear: inserters older than the target's eraser saw the target present,
// so they were rejected and the walk stops there; and a walk that passed
// decided-rejected inserters stores the first one it stopped at in its own
// record's predecessor link (`self`), so later walks through this switch
// skip them.  Any value so written skips only decided-rejected inserters of
// the same target, so concurrent writers are harmless.
__device__ __forceinline__ int judge_target_chain(uint2 *info, uint2 rec, uint32_t self, uint32_t k,
                                                  const uint8_t *st) {
    int v = V_OK;
    const uint32_t e = rec.x;
    if (e != kNoEraser) {
        if (e == kStays || e >= k) return V_ILLEGAL;
        const uint8_t se = load_status(st, e);
        if (se == ST_UNDECIDED)
            v = V_WAIT;
        else if (se != ST_LEGAL)
            return V_ILLEGAL;
    }
    // earlier inserters of the same target, nearest first; switch ids strictly
    // decrease along the chain (checked, so a corrupt record cannot loop)
    uint32_t p = rec.y, below = k;
    int out = v;
    while (p != kNoPred) {
        const uint32_t pk = p >> 1;
        if (pk >= below) return V_ILLEGAL;
        if (e != kNoEraser && pk < e) {  // inserted while the target was still there
            p = kNoPred;
            break;
        }
        const uint8_t sp = load_status(st, pk);
        if (sp == ST_LEGAL) {
            out = V_ILLEGAL;
            break;
        }
        if (sp == ST_UNDECIDED) {
            out = V_WAIT;
            break;
        }
        below = pk;
        p = info[p].y;
    }
    if (p != rec.y) info[self].y = p;
    return out;
}

// judge_target_chain that resumes its predecessor walk at *from (kNoPred:
// the first predecessor, rec.y) and leaves there the predecessor it waits
// for: decided predecessors never change, so a repeated judgement of the
// same switch walks each link once.
__device__ __forceinline__ int judge_target_resume(uint2 *info, uint2 rec, uint32_t self, uint32_t k,
                                                   const uint8_t *st, uint32_t *from) {
    int v = V_OK;
    const uint32_t e = rec.x;
    if (e != kNoEraser) {
        if (e == kStays || e >= k) return V_ILLEGAL;
        const uint8_t se = load_status(st, e);
        if (se == ST_UNDECIDED)
            v = V_WAIT;
        else if (se != ST_LEGAL)
            return V_ILLEGAL;
    }
    // *from: kNoPred (not started), kWalked (nothing left) or a predecessor
    uint32_t p = rec.y, below = k;
    if (*from == kWalked) {
        p = kNoPred;
    } else if (*from != kNoPred) {
        p = *from;
        below = (p >> 1) + 1;
    }
    const uint32_t p0 = p;
    int out = v;
    while (p != kNoPred) {
        const uint32_t pk = p >> 1;
        if (pk >= below) return V_ILLEGAL;
        if (e != kNoEraser && pk < e) {  // inserted while the target was still there
            p = kNoPred;
            break;
        }
        const uint8_t sp = load_status(st, pk);
        if (sp == ST_LEGAL) {
            out = V_ILLEGAL;
            break;
        }
        if (sp == ST_UNDECIDED) {
            out = V_WAIT;
            break;
        }
        below = pk;
        p = info[p].y;
    }
    if (p != p0) info[self].y = p;  // the shortcut of judge_target_chain
    *from = p == kNoPred ? kWalked : p;
    return out;
}

// Decides switch k from its two target records; the pair's records (ij, ee)
// are passed in so that callers can issue every load of the switch at once.
__device__ __forceinline__ bool decide_switch_chain(uint32_t k, uint4 recs, uint2 ij, ulonglong2 ee, uint2 *info,
                                                    uint8_t *st, uint32_t *out_idx, unsigned long long *out_key,
                                                    BlockCounts *bc, uint32_t cls) {
    const int v = max(judge_target_chain(info, make_uint2(recs.x, recs.y), 2 * k, k, st),
                      judge_target_chain(info, make_uint2(recs.z, recs.w), 2 * k + 1, k, st));
    if (v == V_WAIT) return true;
    reinterpret_cast<uint2 *>(out_idx)[k] = ij;
    if (v == V_OK) {
        const Targets T = switch_targets_cls(ee.x, ee.y, ij.x < ij.y, cls);
        reinterpret_cast<ulonglong2 *>(out_key)[k] = make_ulonglong2(T.A, T.B);
        st[k] = ST_LEGAL;
        atomicAdd(&bc->legal, 1u);
    } else {
        reinterpret_cast<ulonglong2 *>(out_key)[k] = ee;
        st[k] = ST_EXISTS;
        atomicAdd(&bc->exists, 1u);
    }
    return false;
}

// The next superstep's first radix level, counted while round 1 runs: the
// records' positions do not change in a superstep (the sorted records of
// position p keep their index), so the level-1 digit counts of superstep
// t + 1 over tiles of `tile` positions need only the indices, which round 1
// reads anyway, and the Philox work hides under its memory traffic.
// A batch (gr != nullptr) counts the global buckets of its next step's
// prefix of m positions (each position's graph from pg).
struct NextCounts {
    uint32_t *counts;  // [tile][digit], nullptr: none
    uint32_t t, k0, k1;
    int shift, dbits;
    uint32_t tile, m;
    const BatchGraph *gr;  // batch: graph records, the graph of each position,
    const uint32_t *pg;    // the next step and its bucket bits
    uint32_t step;
    int bbits;
};

// Round 1 (list == nullptr: every switch) or a later round over a list.
// With nc.counts (round 1 only), each workgroup takes whole tiles of
// nc.tile / 2 switches and also writes their counts.
__global__ __launch_bounds__(kBlock) void k_decide_chain(const uint32_t *__restrict__ s_idx,
                                                         const unsigned long long *__restrict__ s_key, uint32_t ell,
                                                         uint2 *info, uint8_t *st,
                                                         uint32_t *__restrict__ out_idx,
                                                         unsigned long long *__restrict__ out_key,
                                                         const uint32_t *__restrict__ list,
                                                         const uint32_t *__restrict__ count,
                                                         uint32_t *__restrict__ next_list,
                                                         uint32_t *__restrict__ next_count,
                                                         uint32_t *__restrict__ zero_count,
                                                         uint4 *__restrict__ bslot, StepCounters *ctr,
                                                         uint32_t cls, NextCounts nc) {
    __shared__ BlockCounts bc;
    __shared__ uint32_t hs[1u << kMaxCoarseBits];
    if (threadIdx.x == 0) bc = BlockCounts{0, 0, 0, 0};
    __syncthreads();
    // the counter cleared here is the one the round after next fills
    if (zero_count && blockIdx.x == 0 && threadIdx.x == 0) *zero_count = 0;
    auto decide_one = [&](uint32_t k, bool *wait, uint2 *ij_out) {
        const uint8_t sk = st[k];
        const uint4 recs = reinterpret_cast<const uint4 *>(info)[k];
        const uint2 ij = reinterpret_cast<const uint2 *>(s_idx)[k];
        const ulonglong2 ee = reinterpret_cast<const ulonglong2 *>(s_key)[k];
        *ij_out = ij;
        if (sk == ST_UNDECIDED) *wait = decide_switch_chain(k, recs, ij, ee, info, st, out_idx, out_key, &bc, cls);
    };
    const uint32_t n = list ? min(*count, ell) : ell;
    if (nc.counts) {
        const uint32_t nd = 1u << nc.dbits, dmask = nd - 1, half = nc.tile / 2;
        // tiles of the next step's positions (a batch's prefix may shrink: the
        // tiles then also cover this step's remaining switches, uncounted)
        const uint32_t ncount = (nc.m + nc.tile - 1) / nc.tile;
        const uint32_t ntiles = max(ncount, (ell + half - 1) / half);
        auto digit = [&](uint32_t i, uint32_t pos) -> uint32_t {
            if (!nc.gr) return (uint32_t)(perm_key(i, nc.t, nc.k0, nc.k1) >> nc.shift) & dmask;
            const BatchGraph &g = nc.gr[nc.pg[pos]];
            const uint64_t word = (uint64_t)batch_bucket(g, batch_perm_key(g, i, nc.step)) << (64 - nc.bbits);
            return (uint32_t)(word >> nc.shift) & dmask;
        };
        for (uint32_t w = blockIdx.x; w < ntiles; w += gridDim.x) {
            for (uint32_t d = threadIdx.x; d < nd; d += kBlock) hs[d] = 0;
            __syncthreads();
            for (uint32_t j = 0; j < half; j += kBlock) {
                const uint32_t k = w * half + j + threadIdx.x;
                bool wait = false;
                if (k < ell) {
                    uint2 ij;
                    decide_one(k, &wait, &ij);
                    if (2 * k + 1 < nc.m) {  // both positions of a pair lie in one graph
                        atomicAdd(&hs[digit(ij.x, 2 * k)], 1u);
                        atomicAdd(&hs[digit(ij.y, 2 * k)], 1u);
                    }
                }
                append_undecided(wait, k, next_list, next_count, &ctr->undecided_round1);
            }
            if ((nc.m & 1u) && threadIdx.x == 0 && (nc.m - 1) / nc.tile == w)  // the idle record of odd m
                atomicAdd(&hs[digit(s_idx[nc.m - 1], nc.m - 1)], 1u);
            __syncthreads();
            if (w < ncount)
                for (uint32_t d = threadIdx.x; d < nd; d += kBlock) nc.counts[(size_t)w * nd + d] = hs[d];
            __syncthreads();
        }
    } else {
        const uint32_t stride = gridDim.x * kBlock;
        const uint32_t trips = (n + stride - 1) / stride;
        for (uint32_t r = 0; r < trips; ++r) {
            const uint32_t q = r * stride + blockIdx.x * kBlock + threadIdx.x;
            bool wait = false;
            uint32_t k = 0;
            if (q < n) {
                k = list ? list[q] : q;
                uint2 ij;
                if (k < ell) decide_one(k, &wait, &ij);
            }
            append_undecided(wait, k, next_list, next_count, list ? nullptr : &ctr->undecided_round1);
        }
    }
    if (bslot)
        store_counts(&bc, bslot + blockIdx.x);
    else
        flush_counts(&bc, ctr);
    if (blockIdx.x == 0 && threadIdx.x == 0 && n > 0) atomicAdd(&ctr->rounds, 1ull);
}

// Remaining rounds in one workgroup; the next round's list counter is cleared
// by the round that fills it.  After kSweepAfter rounds with switches still
// undecided (long dependency chains: hub edges that many switches erase and
// insert), the rest is decided by a sweep in ascending switch id: a switch
// depends on smaller ids only, so chunks of kSweepChunk ids are taken in
// order, each repeated until it holds no undecided switch; earlier chunks
// are then final and only chains inside a chunk cost repeats.  Each repeat
// counts as a round.
constexpr uint32_t kSweepAfter = 8;
constexpr uint32_t kSweepChunk = 1024;
constexpr uint32_t kSweepWords = 16384;  // chunk marks: ids below 2^29 (m < 2^30)

__global__ __launch_bounds__(kFinishBlock) void k_finish_chain(const uint32_t *__restrict__ s_idx,
                                                               const unsigned long long *__restrict__ s_key,
                                                               uint32_t ell, uint2 *info,
                                                               uint8_t *st, uint32_t *__restrict__ out_idx,
                                                               unsigned long long *__restrict__ out_key,
                                                               uint32_t *list_a, uint32_t *count_a, uint32_t *list_b,
                                                               uint32_t *count_b, const uint4 *__restrict__ bslot,
                                                               uint32_t nbslot, StepCounters *ctr,
                                                               uint32_t *__restrict__ err, uint32_t round_limit,
                                                               uint32_t cls) {
    __shared__ BlockCounts bc;
    __shared__ uint32_t s_n;
    const uint32_t tid = threadIdx.x;
    if (tid == 0) {
        bc = BlockCounts{0, 0, 0, 0};
        s_n = min(*count_a, ell);
        // a caller's round budget (0: none), counted over the superstep's rounds so
        // far (the multi-workgroup rounds before this kernel included)
        const unsigned long long so_far = round_limit ? atomicAdd(&ctr->rounds, 0ull) : 0ull;
        if (round_limit && (so_far > round_limit || (so_far == round_limit && s_n > 0))) {
            atomicOr(err, ERR_ROUNDS);
            s_n = 0;
        }
    }
    __syncthreads();
    {  // fold the per-block counts of the emit and first-round kernels (eight loads in flight)
        constexpr uint32_t kFold = 8;
        uint4 acc = make_uint4(0, 0, 0, 0);
        for (uint32_t q0 = tid; q0 < nbslot; q0 += kFold * kFinishBlock) {
            uint4 v[kFold];
#pragma unroll
            for (uint32_t j = 0; j < kFold; ++j) {
                const uint32_t q = q0 + j * kFinishBlock;
                v[j] = q < nbslot ? bslot[q] : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (uint32_t j = 0; j < kFold; ++j) {
                acc.x += v[j].x;
                acc.y += v[j].y;
                acc.z += v[j].z;
                acc.w += v[j].w;
            }
        }
        if (acc.x) atomicAdd(&bc.legal, acc.x);
        if (acc.y) atomicAdd(&bc.loop, acc.y);
        if (acc.z) atomicAdd(&bc.exists, acc.z);
        if (acc.w) atomicAdd(&bc.pl, acc.w);
    }
    uint32_t *cur = list_a, *nxt = list_b, *ccur = count_a, *cnxt = count_b;
    uint32_t n = s_n;
    for (uint32_t here = 0; n > 0 && here < kSweepAfter; ++here) {
        if (tid == 0) *cnxt = 0;
        __threadfence();
        __syncthreads();
        const uint32_t trips = (n + kFinishBlock - 1) / kFinishBlock;
        for (uint32_t r = 0; r < trips; ++r) {
            const uint32_t q = r * kFinishBlock + tid;
            bool wait = false;
            uint32_t k = 0;
            if (q < n) {
                k = cur[q];
                if (k < ell && st[k] == ST_UNDECIDED)
                    wait = decide_switch_chain(k, reinterpret_cast<const uint4 *>(info)[k],
                                               reinterpret_cast<const uint2 *>(s_idx)[k],
                                               reinterpret_cast<const ulonglong2 *>(s_key)[k], info, st, out_idx,
                                               out_key, &bc, cls);
            }
            append_undecided(wait, k, nxt, cnxt);
        }
        __threadfence();
        __syncthreads();
        if (tid == 0) {
            const uint32_t nn = min(*cnxt, ell);
            if (nn >= n) atomicOr(err, ERR_INTERNAL);  // the smallest undecided switch always decides
            s_n = nn >= n ? 0 : nn;
            const unsigned long long done = atomicAdd(&ctr->rounds, 1ull) + 1;
            if (round_limit && s_n > 0 && done >= round_limit) {
                atomicOr(err, ERR_ROUNDS);
                s_n = 0;
            }
        }
        __syncthreads();
        n = s_n;
        uint32_t *tl = cur;
        cur = nxt;
        nxt = tl;
        uint32_t *tc = ccur;
        ccur = cnxt;
        cnxt = tc;
    }
    if (n > 0) {
        __shared__ uint32_t s_chunks[kSweepWords];
        __shared__ uint32_t s_wait, s_done, s_stop;
        __shared__ unsigned long long s_rounds;
        const uint32_t nwords = ((ell + kSweepChunk - 1) / kSweepChunk + 31) / 32;
        for (uint32_t w = tid; w < nwords; w += kFinishBlock) s_chunks[w] = 0;
        if (tid == 0) {
            s_rounds = atomicAdd(&ctr->rounds, 0ull);
            s_stop = 0;
        }
        __syncthreads();
        for (uint32_t q = tid; q < n; q += kFinishBlock) {
            const uint32_t k = cur[q];
            if (k < ell) atomicOr(&s_chunks[(k / kSweepChunk) >> 5], 1u << ((k / kSweepChunk) & 31));
        }
        __syncthreads();
        unsigned long long added = 0;
        for (uint32_t w = 0; w < nwords && !s_stop; ++w) {
            uint32_t bits = s_chunks[w];
            while (bits && !s_stop) {
                const uint32_t c = w * 32 + (uint32_t)(__ffs(bits) - 1);
                bits &= bits - 1;
                const uint32_t kb = c * kSweepChunk, ke = min(kb + kSweepChunk, ell);
                constexpr uint32_t kPer = kSweepChunk / kFinishBlock;
                uint2 from[kPer];  // resume points of the two predecessor walks
#pragma unroll
                for (uint32_t j = 0; j < kPer; ++j) from[j] = make_uint2(kNoPred, kNoPred);
                for (;;) {
                    if (tid == 0) {
                        s_wait = 0;
                        s_done = 0;
                    }
                    __syncthreads();
                    uint32_t waits = 0, dones = 0;
#pragma unroll
                    for (uint32_t j = 0; j < kPer; ++j) {
                        const uint32_t k = kb + tid + j * kFinishBlock;
                        if (k >= ke || load_status(st, k) != ST_UNDECIDED) continue;
                        const uint4 recs = reinterpret_cast<const uint4 *>(info)[k];
                        const int v =
                            max(judge_target_resume(info, make_uint2(recs.x, recs.y), 2 * k, k, st, &from[j].x),
                                judge_target_resume(info, make_uint2(recs.z, recs.w), 2 * k + 1, k, st, &from[j].y));
                        if (v == V_WAIT) {
                            ++waits;
                            continue;
                        }
                        ++dones;
                        const uint2 ij = reinterpret_cast<const uint2 *>(s_idx)[k];
                        const ulonglong2 ee = reinterpret_cast<const ulonglong2 *>(s_key)[k];
                        reinterpret_cast<uint2 *>(out_idx)[k] = ij;
                        if (v == V_OK) {
                            const Targets T = switch_targets_cls(ee.x, ee.y, ij.x < ij.y, cls);
                            reinterpret_cast<ulonglong2 *>(out_key)[k] = make_ulonglong2(T.A, T.B);
                            st[k] = ST_LEGAL;
                            atomicAdd(&bc.legal, 1u);
                        } else {
                            reinterpret_cast<ulonglong2 *>(out_key)[k] = ee;
                            st[k] = ST_EXISTS;
                            atomicAdd(&bc.exists, 1u);
                        }
                    }
                    if (waits) atomicAdd(&s_wait, waits);
                    if (dones) atomicAdd(&s_done, dones);
                    __syncthreads();
                    const uint32_t W = s_wait, D = s_done;
                    if (tid == 0) {
                        ++added;
                        // the smallest undecided switch of the chunk always decides
                        if (W > 0 && D == 0) {
                            atomicOr(err, ERR_INTERNAL);
                            s_stop = 1;
                        } else if (W > 0 && round_limit && s_rounds + added >= round_limit) {
                            atomicOr(err, ERR_ROUNDS);
                            s_stop = 1;
                        }
                    }
                    __syncthreads();
                    if (W == 0 || s_stop) break;
                }
            }
        }
        if (tid == 0 && added) atomicAdd(&ctr->rounds, added);
    }
    flush_counts(&bc, ctr);
}

}  // namespace gesmc

// Permutation pi of one global switch (Def. 3.2; the random-keys shuffle the
// paper's parallel permutation builds on, Sec. 5.3): the edge records
// (index, key) are placed in ascending (K_i, i) order, where K_i is the
// Philox key of edge index i in superstep t.
//
// MSD radix layout for gfx950:
//   level 1   : coarse digit = top b1 bits of K (b1 <= 8), LDS-staged scatter
//   level 2   : sub digit    = next b2 bits, scattered inside each coarse
//               bucket (its region is small enough to stay L2/MALL resident)
//   bucket    : each fine bucket (~0.5-1k records) is counting-sorted in LDS
//               on the next 11 bits of K, then ties inside a 12-bit cell are
//               settled by insertion sort on (K, i).
// Keys are never stored: every pass recomputes K_i from the record's index.
#pragma once

#include "device_common.h"

namespace gesmc {

#ifndef GESMC_SCATTER_TILE
#define GESMC_SCATTER_TILE 2048
#endif
#ifndef GESMC_SORT_SUB_BITS
#define GESMC_SORT_SUB_BITS 10
#endif
constexpr int kScatterTile = GESMC_SCATTER_TILE;     // records per scatter workgroup
constexpr int kSortSubBits = GESMC_SORT_SUB_BITS;    // counting-sort cells per bucket = 2^bits
constexpr int kSortMaxItems = (1 << kSortSubBits) / kBlock;  // per-thread records (cap <= 2^bits)

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
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
        const uint32_t v = wsum[q];
        before += (q < (int)w) ? v : 0u;
        all += v;
    }
    __syncthreads();
    *total = all;
    return before + incl - x;
}

// Workgroup-wide exclusive scan (in place) of n values in LDS; each thread
// owns a contiguous run of ceil(n / kBlock).  `tmp` needs kBlock + 1 words.
// Returns the total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t *v, uint32_t n, uint32_t *tmp) {
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (n + kBlock - 1) / kBlock;
    const uint32_t b = min(tid * per, n);
    const uint32_t e = min(b + per, n);
    uint32_t s = 0;
    for (uint32_t q = b; q < e; ++q) s += v[q];
    uint32_t total;
    uint32_t acc = block_exclusive_sum<kBlock>(s, tmp, &total);
    for (uint32_t q = b; q < e; ++q) {
        const uint32_t x = v[q];
        v[q] = acc;
        acc += x;
    }
    __syncthreads();
    return total;
}

// ---------------------------------------------------------------------------
// Histogram of the coarse digit over all edge indices i in [0, m) -- the set
// of indices is the same every superstep, so nothing is read -- fused with
// the per-superstep reset of the dependency table and switch states.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_hist_clear(uint32_t m, uint32_t t, uint32_t k0, uint32_t k1, int b1,
                                                       uint32_t *__restrict__ coarse_hist, Slot *__restrict__ tab,
                                                       uint64_t tab_slots, uint8_t *__restrict__ st, uint32_t ell,
                                                       uint32_t *__restrict__ ucount) {
    __shared__ uint32_t h[256];
    const uint32_t tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const uint64_t nthreads = (uint64_t)gridDim.x * kBlock;
    const uint64_t gtid = (uint64_t)blockIdx.x * kBlock + tid;
    if (b1 > 0) {
        const int shift = 64 - b1;
        for (uint64_t i = gtid; i < m; i += nthreads) {
            const uint64_t K = perm_key((uint32_t)i, t, k0, k1);
            atomicAdd(&h[(uint32_t)(K >> shift)], 1u);
        }
    } else if (gtid == 0) {
        atomicAdd(&h[0], m);
    }
    // table reset: 16-byte vector stores of {empty key, no eraser, no claim}
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    u32x4 *t4 = reinterpret_cast<u32x4 *>(tab);
    const u32x4 empty = {0xFFFFFFFFu, 0xFFFFFFFFu, kNoEraser, kClaimNone};
    for (uint64_t s = gtid; s < tab_slots; s += nthreads) __builtin_nontemporal_store(empty, &t4[s]);
    for (uint64_t k = gtid; k < ell; k += nthreads) st[k] = ST_UNDECIDED;
    if (gtid == 0) {
        ucount[0] = 0;
        ucount[1] = 0;
        ucount[2] = 0;
    }
    __syncthreads();
    if (b1 > 0) {
        for (uint32_t d = tid; d < (1u << b1); d += kBlock)
            if (h[d]) atomicAdd(&coarse_hist[d], h[d]);
    } else if (tid == 0) {
        atomicAdd(&coarse_hist[0], h[0]);
    }
}

// Coarse scan (one workgroup): coarse offsets, level-1 cursors, and the
// level-2 tile map (tiles of kScatterTile records inside each coarse bucket).
// Clears the histogram for the next superstep.
__global__ __launch_bounds__(kBlock) void k_scan_coarse(uint32_t ncoarse, uint32_t *__restrict__ coarse_hist,
                                                        uint32_t *__restrict__ coarse_off,
                                                        uint32_t *__restrict__ coarse_cursor,
                                                        uint32_t *__restrict__ tile_first) {
    __shared__ uint32_t v[257], w[257], tmp[kBlock + 1];
    const uint32_t tid = threadIdx.x;
    for (uint32_t d = tid; d < ncoarse; d += kBlock) {
        v[d] = coarse_hist[d];
        w[d] = (v[d] + kScatterTile - 1) / kScatterTile;
        coarse_hist[d] = 0;
    }
    __syncthreads();
    const uint32_t total = block_exclusive_scan(v, ncoarse, tmp);
    const uint32_t tiles = block_exclusive_scan(w, ncoarse, tmp);
    for (uint32_t d = tid; d < ncoarse; d += kBlock) {
        coarse_off[d] = v[d];
        coarse_cursor[d] = v[d];
        tile_first[d] = w[d];
    }
    if (tid == 0) {
        coarse_off[ncoarse] = total;
        tile_first[ncoarse] = tiles;
    }
}

// Fine scan, one workgroup per coarse segment s: the 2^dbits sub-counts of s
// (in LDS) scanned and offset by the segment's start give the fine offsets
// and cursors; the histogram is cleared for the next use.
__global__ __launch_bounds__(kBlock) void k_scan_fine(int dbits, const uint32_t *__restrict__ coarse_off,
                                                      uint32_t ncoarse, uint32_t *__restrict__ fine_hist,
                                                      uint32_t *__restrict__ fine_off,
                                                      uint32_t *__restrict__ fine_cursor) {
    extern __shared__ uint32_t v[];  // 2^dbits + kBlock + 1
    uint32_t *tmp = v + (1u << dbits);
    const uint32_t s = blockIdx.x, nd = 1u << dbits, base = s << dbits;
    for (uint32_t d = threadIdx.x; d < nd; d += kBlock) {
        v[d] = fine_hist[base + d];
        fine_hist[base + d] = 0;
    }
    __syncthreads();
    block_exclusive_scan(v, nd, tmp);
    const uint32_t off = coarse_off[s];
    for (uint32_t d = threadIdx.x; d < nd; d += kBlock) {
        fine_off[base + d] = off + v[d];
        fine_cursor[base + d] = off + v[d];
    }
    if (s == ncoarse - 1 && threadIdx.x == 0) fine_off[ncoarse << dbits] = coarse_off[ncoarse];
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

// Radix source of a record: kByKeyHash = false sorts edge records by the
// Philox key of their index (the permutation); true sorts (tag, edge key)
// tuples by a hash of the edge key (the dependency partitions), where an
// empty key marks a tuple slot that carries nothing.
template <bool kByKeyHash>
__device__ __forceinline__ uint64_t radix_word(uint32_t idx, unsigned long long key, uint32_t t, uint32_t k0,
                                               uint32_t k1) {
    if (kByKeyHash) return slot_hash(key);
    return perm_key(idx, t, k0, k1);
}

// Level-2 histogram: sub digit counts of each coarse segment, per tile in LDS,
// added into the global fine histogram.
template <bool kByKeyHash>
__global__ __launch_bounds__(kBlock) void k_hist_sub(const uint32_t *__restrict__ src_idx,
                                                     const unsigned long long *__restrict__ src_key, uint32_t t,
                                                     uint32_t k0, uint32_t k1, int shift, int dbits, uint32_t nseg,
                                                     const uint32_t *__restrict__ seg_off,
                                                     const uint32_t *__restrict__ tile_first,
                                                     uint32_t *__restrict__ fine_hist) {
    extern __shared__ uint32_t hs[];
    const uint32_t w = blockIdx.x;
    if (w >= tile_first[nseg]) return;
    const uint32_t s = tile_segment(tile_first, nseg, w);
    const uint32_t begin = seg_off[s] + (w - tile_first[s]) * kScatterTile;
    const uint32_t end = min(begin + kScatterTile, seg_off[s + 1]);
    const uint32_t nd = 1u << dbits, dmask = nd - 1;
    for (uint32_t d = threadIdx.x; d < nd; d += kBlock) hs[d] = 0;
    __syncthreads();
    for (uint32_t p = begin + threadIdx.x; p < end; p += kBlock) {
        const uint64_t K = kByKeyHash ? radix_word<true>(0, src_key[p], t, k0, k1)
                                      : radix_word<false>(src_idx[p], 0, t, k0, k1);
        atomicAdd(&hs[(uint32_t)(K >> shift) & dmask], 1u);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < nd; d += kBlock)
        if (hs[d]) atomicAdd(&fine_hist[(s << dbits) | d], hs[d]);
}

// LDS-staged scatter of one tile of a segment by digit (K >> shift) & mask.
// Records of one digit leave the workgroup as one contiguous run.  With
// kByKeyHash, tuple slots whose key is empty are dropped.
// Dynamic LDS: 3 * 2^dbits + 1 + kBlock + 1 words of counters, then the
// staged records.
template <bool kByKeyHash>
__global__ __launch_bounds__(kBlock) void k_scatter(const uint32_t *__restrict__ src_idx,
                                                    const unsigned long long *__restrict__ src_key,
                                                    uint32_t *__restrict__ dst_idx,
                                                    unsigned long long *__restrict__ dst_key, uint32_t t, uint32_t k0,
                                                    uint32_t k1, int shift, int dbits, uint32_t nseg,
                                                    const uint32_t *__restrict__ seg_off,
                                                    const uint32_t *__restrict__ tile_first,
                                                    uint32_t *__restrict__ cursor, uint32_t *__restrict__ err) {
    extern __shared__ uint32_t lds[];
    const uint32_t nd = 1u << dbits, dmask = nd - 1;
    uint32_t *cnt = lds;                 // nd
    uint32_t *start = cnt + nd;          // nd (exclusive scan of cnt)
    uint32_t *base = start + nd;         // nd (global run base)
    uint32_t *tmp = base + nd;           // kBlock + 1
    uint32_t *s_idx = tmp + kBlock + 1;  // kScatterTile
    unsigned long long *s_key =
        reinterpret_cast<unsigned long long *>(s_idx + kScatterTile + ((kBlock + 1 + 3 * nd + kScatterTile) & 1));
    uint16_t *s_dig = reinterpret_cast<uint16_t *>(s_key + kScatterTile);

    const uint32_t w = blockIdx.x;
    if (w >= tile_first[nseg]) return;
    const uint32_t s = tile_segment(tile_first, nseg, w);
    const uint32_t seg_begin = seg_off[s], seg_end = seg_off[s + 1];
    const uint32_t begin = seg_begin + (w - tile_first[s]) * kScatterTile;
    const uint32_t end = min(begin + kScatterTile, seg_end);
    const uint32_t cnt_here = end > begin ? end - begin : 0;
    const uint32_t tid = threadIdx.x;

    for (uint32_t d = tid; d < nd; d += kBlock) cnt[d] = 0;
    __syncthreads();

    constexpr int kItems = kScatterTile / kBlock;
    uint32_t r_idx[kItems], r_dig[kItems], r_rank[kItems];
    unsigned long long r_key[kItems];
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
        const uint32_t p = tid + q * kBlock;
        r_dig[q] = 0xFFFFFFFFu;
        if (p < cnt_here) {
            r_idx[q] = src_idx[begin + p];
            r_key[q] = src_key[begin + p];
            if (!kByKeyHash || r_key[q] != kEmptyKey) {
                const uint64_t K = radix_word<kByKeyHash>(r_idx[q], r_key[q], t, k0, k1);
                r_dig[q] = (uint32_t)(K >> shift) & dmask;
                r_rank[q] = atomicAdd(&cnt[r_dig[q]], 1u);
            }
        }
    }
    __syncthreads();
    for (uint32_t d = tid; d < nd; d += kBlock) start[d] = cnt[d];
    __syncthreads();
    block_exclusive_scan(start, nd, tmp);
    for (uint32_t d = tid; d < nd; d += kBlock)
        if (cnt[d]) base[d] = atomicAdd(&cursor[(s << dbits) | d], cnt[d]);
    __shared__ uint32_t s_total;
    if (tid == 0) s_total = 0;
    __syncthreads();
    uint32_t mine = 0;
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
        const uint32_t p = tid + q * kBlock;
        if (p < cnt_here && r_dig[q] != 0xFFFFFFFFu) {
            const uint32_t lp = start[r_dig[q]] + r_rank[q];
            s_idx[lp] = r_idx[q];
            s_key[lp] = r_key[q];
            s_dig[lp] = (uint16_t)r_dig[q];
            ++mine;
        }
    }
    if (mine) atomicAdd(&s_total, mine);
    __syncthreads();
    const uint32_t staged = s_total;
    for (uint32_t lp = tid; lp < staged; lp += kBlock) {
        const uint32_t d = s_dig[lp];
        const uint32_t g = base[d] + (lp - start[d]);
        if (g >= seg_begin && g < seg_end) {
            dst_idx[g] = s_idx[lp];
            dst_key[g] = s_key[lp];
        } else {
            atomicOr(err, ERR_INTERNAL);
        }
    }
}

// Sorts each fine bucket by (K, i): LDS counting sort on the 11 bits of K
// below the B bucket bits, then insertion sort inside each cell.  Buckets
// larger than `cap` (never expected: the mean is <= 1024 and the cap 2048)
// take a slow exact path that ranks every record against the whole bucket.
// Dynamic LDS: 2048 cell counters + kBlock + 2 scan words + cap * 20 bytes.
__global__ __launch_bounds__(kBlock) void k_sort_buckets(const uint32_t *__restrict__ src_idx,
                                                         const unsigned long long *__restrict__ src_key,
                                                         uint32_t *__restrict__ dst_idx,
                                                         unsigned long long *__restrict__ dst_key,
                                                         unsigned long long *__restrict__ scratch_k, uint32_t t,
                                                         uint32_t k0, uint32_t k1, int bbits,
                                                         const uint32_t *__restrict__ fine_off, uint32_t m, uint32_t cap,
                                                         StepCounters *__restrict__ ctr) {
    extern __shared__ uint32_t lds[];
    constexpr uint32_t kCells = 1u << kSortSubBits;
    uint32_t *cell = lds;                    // kCells
    uint32_t *tmp = cell + kCells;           // kBlock + 1 (+1 pad for 8-byte alignment)
    unsigned long long *sK = reinterpret_cast<unsigned long long *>(tmp + kBlock + 2);
    unsigned long long *sE = sK + cap;
    uint32_t *sI = reinterpret_cast<uint32_t *>(sE + cap);

    const uint32_t f = blockIdx.x;
    const uint32_t begin = min(fine_off[f], m), end = min(fine_off[f + 1], m);
    const uint32_t c = end > begin ? end - begin : 0;
    const uint32_t tid = threadIdx.x;
    if (c == 0) return;

    if (c > cap || c > (uint32_t)(kSortMaxItems * kBlock)) {
        // exact slow path: rank_p = #{q : (K_q, i_q) < (K_p, i_p)}
        for (uint32_t p = tid; p < c; p += kBlock) scratch_k[begin + p] = perm_key(src_idx[begin + p], t, k0, k1);
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
        return;
    }

    for (uint32_t q = tid; q < kCells; q += kBlock) cell[q] = 0;
    __syncthreads();
    const int sub_shift = 64 - kSortSubBits;
    uint32_t r_idx[kSortMaxItems], r_cell[kSortMaxItems], r_rank[kSortMaxItems];
    unsigned long long r_key[kSortMaxItems], r_K[kSortMaxItems];
#pragma unroll
    for (int q = 0; q < kSortMaxItems; ++q) {
        const uint32_t p = tid + q * kBlock;
        if (p < c) {
            r_idx[q] = src_idx[begin + p];
            r_key[q] = src_key[begin + p];
            r_K[q] = perm_key(r_idx[q], t, k0, k1);
            r_cell[q] = (uint32_t)((bbits >= 64 ? 0ull : (r_K[q] << bbits)) >> sub_shift);
            r_rank[q] = atomicAdd(&cell[r_cell[q]], 1u);
        }
    }
    __syncthreads();
    block_exclusive_scan(cell, kCells, tmp);
#pragma unroll
    for (int q = 0; q < kSortMaxItems; ++q) {
        const uint32_t p = tid + q * kBlock;
        if (p < c) {
            const uint32_t lp = cell[r_cell[q]] + r_rank[q];
            sK[lp] = r_K[q];
            sE[lp] = r_key[q];
            sI[lp] = r_idx[q];
        }
    }
    __syncthreads();
    // settle ties of the counting sort: each thread owns 16 consecutive cells
    for (uint32_t q = tid * (kCells / kBlock); q < (tid + 1) * (kCells / kBlock); ++q) {
        const uint32_t a = cell[q];
        const uint32_t b = (q + 1 < kCells) ? cell[q + 1] : c;
        for (uint32_t x = a + 1; x < b; ++x) {
            const unsigned long long kx = sK[x], ex = sE[x];
            const uint32_t ix = sI[x];
            uint32_t y = x;
            while (y > a && (sK[y - 1] > kx || (sK[y - 1] == kx && sI[y - 1] > ix))) {
                sK[y] = sK[y - 1];
                sE[y] = sE[y - 1];
                sI[y] = sI[y - 1];
                --y;
            }
            sK[y] = kx;
            sE[y] = ex;
            sI[y] = ix;
        }
    }
    __syncthreads();
    for (uint32_t p = tid; p < c; p += kBlock) {
        dst_idx[begin + p] = sI[p];
        dst_key[begin + p] = sE[p];
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

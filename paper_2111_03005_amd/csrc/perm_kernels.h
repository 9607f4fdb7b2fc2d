// Permutation pi of one global switch (Def. 3.2; the random-keys shuffle the
// paper's parallel permutation builds on, Sec. 5.3): the edge records
// (index, key) are placed in ascending (K_i, i) order, where K_i is the
// Philox key of edge index i in superstep t.
//
// MSD radix layout for gfx950:
//   level 1   : coarse digit = top b1 bits of K (b1 <= 8), LDS-staged scatter
//   level 2   : sub digit    = next b2 bits, scattered inside each coarse
//               bucket (its region is small enough to stay L2/MALL resident)
//   bucket    : each fine bucket (~1-2.5k records) is counting-sorted in LDS
//               on the next 12 bits of K, then ties inside a 12-bit cell are
//               settled by insertion sort on (K, i).
// Keys are never stored: every pass recomputes K_i from the record's index.
#pragma once

#include "device_common.h"

namespace gesmc {

constexpr int kScatterTile = 4096;  // records per scatter workgroup
constexpr int kSortSubBits = 12;    // counting-sort cells per fine bucket = 4096
constexpr int kSortMaxItems = 12;   // per-thread records in the LDS sort (cap <= 3072)

// Workgroup-wide exclusive scan of n <= kBlock * per values held in LDS
// (in place).  `tmp` needs kBlock + 1 entries.  Returns the total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t *v, uint32_t n, uint32_t *tmp) {
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (n + kBlock - 1) / kBlock;
    const uint32_t b = tid * per;
    const uint32_t e = min(b + per, n);
    uint32_t s = 0;
    for (uint32_t q = b; q < e; ++q) s += v[q];
    tmp[tid] = s;
    __syncthreads();
    if (tid == 0) {
        uint32_t acc = 0;
        for (int q = 0; q < kBlock; ++q) {
            uint32_t x = tmp[q];
            tmp[q] = acc;
            acc += x;
        }
        tmp[kBlock] = acc;
    }
    __syncthreads();
    uint32_t acc = tmp[tid];
    for (uint32_t q = b; q < e; ++q) {
        uint32_t x = v[q];
        v[q] = acc;
        acc += x;
    }
    __syncthreads();
    return tmp[kBlock];
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

// Fine scan (one workgroup of 1024 threads): offsets and cursors of all 2^B
// fine buckets; clears the fine histogram.
__global__ __launch_bounds__(1024) void k_scan_fine(uint32_t nfine, uint32_t *__restrict__ fine_hist,
                                                    uint32_t *__restrict__ fine_off,
                                                    uint32_t *__restrict__ fine_cursor) {
    __shared__ uint32_t part[1025];
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (nfine + 1023) / 1024;
    const uint32_t b = tid * per, e = min(b + per, nfine);
    uint32_t s = 0;
    for (uint32_t q = b; q < e; ++q) s += fine_hist[q];
    part[tid] = s;
    __syncthreads();
    if (tid == 0) {
        uint32_t acc = 0;
        for (int q = 0; q < 1024; ++q) {
            uint32_t x = part[q];
            part[q] = acc;
            acc += x;
        }
        part[1024] = acc;
    }
    __syncthreads();
    uint32_t acc = part[tid];
    for (uint32_t q = b; q < e; ++q) {
        const uint32_t x = fine_hist[q];
        fine_off[q] = acc;
        fine_cursor[q] = acc;
        fine_hist[q] = 0;
        acc += x;
    }
    if (tid == 0) fine_off[nfine] = part[1024];
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

// Level-2 histogram: sub digit counts of each coarse segment, per tile in LDS,
// added into the global fine histogram.
__global__ __launch_bounds__(kBlock) void k_hist_sub(const uint32_t *__restrict__ src_idx, uint32_t t, uint32_t k0,
                                                     uint32_t k1, int shift, int dbits, uint32_t nseg,
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
        const uint64_t K = perm_key(src_idx[p], t, k0, k1);
        atomicAdd(&hs[(uint32_t)(K >> shift) & dmask], 1u);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < nd; d += kBlock)
        if (hs[d]) atomicAdd(&fine_hist[(s << dbits) | d], hs[d]);
}

// LDS-staged scatter of one tile of a segment by digit (K >> shift) & mask.
// Records of one digit leave the workgroup as one contiguous run.
// Dynamic LDS: 3 * 2^dbits + 1 + kBlock + 1 words of counters, then the
// staged records.
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
        if (p < cnt_here) {
            r_idx[q] = src_idx[begin + p];
            r_key[q] = src_key[begin + p];
            const uint64_t K = perm_key(r_idx[q], t, k0, k1);
            r_dig[q] = (uint32_t)(K >> shift) & dmask;
            r_rank[q] = atomicAdd(&cnt[r_dig[q]], 1u);
        }
    }
    __syncthreads();
    for (uint32_t d = tid; d < nd; d += kBlock) start[d] = cnt[d];
    __syncthreads();
    block_exclusive_scan(start, nd, tmp);
    for (uint32_t d = tid; d < nd; d += kBlock)
        if (cnt[d]) base[d] = atomicAdd(&cursor[(s << dbits) | d], cnt[d]);
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
        const uint32_t p = tid + q * kBlock;
        if (p < cnt_here) {
            const uint32_t lp = start[r_dig[q]] + r_rank[q];
            s_idx[lp] = r_idx[q];
            s_key[lp] = r_key[q];
            s_dig[lp] = (uint16_t)r_dig[q];
        }
    }
    __syncthreads();
    for (uint32_t lp = tid; lp < cnt_here; lp += kBlock) {
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

// Sorts each fine bucket by (K, i): LDS counting sort on the 12 bits of K
// below the B bucket bits, then insertion sort inside each cell.  Buckets
// larger than `cap` (never expected: the mean is <= 2560 and the cap 3072)
// take a slow exact path that ranks every record against the whole bucket.
// Dynamic LDS: 4096 cell counters + kBlock + 1 scan words + cap * 20 bytes.
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

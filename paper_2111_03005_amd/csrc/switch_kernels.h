// The switches of one global switch and their dependency resolution
// (Def. 2.1, Def. 3.2, Alg. 1 of arXiv 2111.03005), for gfx950.
//
// After the permutation kernels, record r of the sorted array holds the edge
// at position pi[r]; switch k owns records 2k and 2k+1: i = pi[2k],
// j = pi[2k+1], e1 = E[i], e2 = E[j], g = [i < j].
//
// Sequential meaning that every schedule below reproduces (Sec. 4): switch k
// is rejected iff a target is a loop, or a target X is present when k runs:
//   X in E0 and X's eraser (the switch owning X's position) is not an
//   earlier legal switch,  or  an earlier legal switch inserted X.
// Round structure (the rounds of Alg. 1, bulk-synchronous over kernels):
//   build    : E0 keys get their eraser id, targets claim with atomicMin
//              (earliest inserter wins); switches that are rejected without
//              looking at anyone else (loop, target = own source, P_L) are
//              decided here and their sources marked as staying.
//   round 1  : every switch decides from the table; the undecided go to a list.
//   round r  : claims of the listed switches' targets are recomputed over
//              the still-undecided inserters (a legal inserter's claim is
//              frozen), then they decide again.  The smallest undecided switch
//              always decides, so the loop ends.
#pragma once

#include "device_common.h"

namespace gesmc {

// ---------------------------------------------------------------------------
// Input load: records (i, E[i]), undirected keys made canonical; loops
// (unless the class allows them) and out-of-range ids flagged.  Class 0 is
// the simple undirected graph; directed keys are kept as (tail, head).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_load(const unsigned long long *__restrict__ in, uint32_t m, uint32_t n,
                                                 uint32_t *__restrict__ idx, unsigned long long *__restrict__ key,
                                                 uint32_t *__restrict__ err, uint32_t cls) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    uint32_t f = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        const unsigned long long e = in[i];
        const uint32_t a = (uint32_t)(e >> 32), b = (uint32_t)e;
        if (a == b && !(cls & CLS_LOOPS)) f |= ERR_LOOP;
        if (a >= n || b >= n || a == 0xFFFFFFFFu || b == 0xFFFFFFFFu) f |= ERR_RANGE;
        idx[i] = (uint32_t)i;
        key[i] = (cls & CLS_DIRECTED) ? e : ekey(a, b);
    }
    if (f) atomicOr(err, f);
}

// Duplicate check of the input edges (used when no superstep runs).
__global__ __launch_bounds__(kBlock) void k_validate(const unsigned long long *__restrict__ key, uint32_t m, Slot *tab,
                                                     uint32_t nslots, uint32_t *__restrict__ err) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        const uint32_t s = table_find_or_insert(tab, nslots, key[i]);
        if (s == kNoSlot)
            atomicOr(err, ERR_INTERNAL);
        else if (atomicCAS(&tab[s].eraser, kNoEraser, kStays) != kNoEraser)
            atomicOr(err, ERR_DUP);
    }
}

// Per-workgroup counter accumulation into the superstep's counters.
struct BlockCounts {
    uint32_t legal, loop, exists, pl;
};

__device__ __forceinline__ void flush_counts(BlockCounts *bc, StepCounters *ctr) {
    __syncthreads();
    if (threadIdx.x == 0) {
        if (bc->legal) atomicAdd(&ctr->legal, (unsigned long long)bc->legal);
        if (bc->loop) atomicAdd(&ctr->rej_loop, (unsigned long long)bc->loop);
        if (bc->exists) atomicAdd(&ctr->rej_exists, (unsigned long long)bc->exists);
        if (bc->pl) atomicAdd(&ctr->rej_pl, (unsigned long long)bc->pl);
    }
}

// Stores the block's counts into a slot of its own (plain stores, no
// device-scope atomics, which would serialise memory-side on one address);
// a single-workgroup kernel folds the slots later.
__device__ __forceinline__ void store_counts(BlockCounts *bc, uint4 *slot) {
    __syncthreads();
    if (threadIdx.x == 0) *slot = make_uint4(bc->legal, bc->loop, bc->exists, bc->pl);
}

// ---------------------------------------------------------------------------
// Build: one thread per switch (plus one for the idle record of odd m).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_build(const uint32_t *__restrict__ s_idx,
                                                  const unsigned long long *__restrict__ s_key, uint32_t m, uint32_t t,
                                                  uint32_t k0, uint32_t k1, uint32_t pl, Slot *tab, uint32_t nslots,
                                                  uint32_t *__restrict__ sw_slot, uint8_t *__restrict__ st,
                                                  uint32_t *__restrict__ out_idx,
                                                  unsigned long long *__restrict__ out_key, StepCounters *ctr,
                                                  uint32_t *__restrict__ err, uint32_t dup_bit) {
    __shared__ BlockCounts bc;
    if (threadIdx.x == 0) bc = BlockCounts{0, 0, 0, 0};
    __syncthreads();
    const uint32_t ell = m >> 1;
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k == ell && (m & 1u)) {
        // idle position pi[m-1]: its edge stays
        const unsigned long long e = s_key[m - 1];
        const uint32_t s = table_find_or_insert(tab, nslots, e);
        if (s == kNoSlot)
            atomicOr(err, ERR_INTERNAL);
        else if (atomicCAS(&tab[s].eraser, kNoEraser, kStays) != kNoEraser)
            atomicOr(err, dup_bit);
        out_idx[m - 1] = s_idx[m - 1];
        out_key[m - 1] = e;
    } else if (k < ell) {
        const uint32_t i = s_idx[2 * k], j = s_idx[2 * k + 1];
        const unsigned long long e1 = s_key[2 * k], e2 = s_key[2 * k + 1];
        uint8_t status = ST_UNDECIDED;
        Targets T{0, 0, false};
        if (pl_skip(k, t, pl, k0, k1)) {
            status = ST_PL;
        } else {
            T = switch_targets(e1, e2, i < j);
            if (T.loop)
                status = ST_LOOP;
            else if (T.A == e1 || T.A == e2 || T.B == e1 || T.B == e2)
                status = ST_EXISTS;  // a target is one of the switch's own (present) sources
        }
        const uint32_t eraser = status == ST_UNDECIDED ? k : kStays;
        const uint32_t s1 = table_find_or_insert(tab, nslots, e1);
        const uint32_t s2 = table_find_or_insert(tab, nslots, e2);
        if (s1 == kNoSlot || s2 == kNoSlot)
            atomicOr(err, ERR_INTERNAL);
        else {
            if (atomicCAS(&tab[s1].eraser, kNoEraser, eraser) != kNoEraser) atomicOr(err, dup_bit);
            if (atomicCAS(&tab[s2].eraser, kNoEraser, eraser) != kNoEraser) atomicOr(err, dup_bit);
        }
        if (status == ST_UNDECIDED) {
            const uint32_t sa = table_find_or_insert(tab, nslots, T.A);
            const uint32_t sb = table_find_or_insert(tab, nslots, T.B);
            if (sa == kNoSlot || sb == kNoSlot) {
                atomicOr(err, ERR_INTERNAL);
            } else {
                if (atomicMin(&tab[sa].claim, k << 2) != kClaimNone) atomicOr(&tab[sa].claim, kClaimContended);
                if (atomicMin(&tab[sb].claim, k << 2) != kClaimNone) atomicOr(&tab[sb].claim, kClaimContended);
            }
            sw_slot[2 * k] = sa;
            sw_slot[2 * k + 1] = sb;
        } else {
            st[k] = status;
            out_idx[2 * k] = i;
            out_key[2 * k] = e1;
            out_idx[2 * k + 1] = j;
            out_key[2 * k + 1] = e2;
            if (status == ST_PL) atomicAdd(&bc.pl, 1u);
            if (status == ST_LOOP) atomicAdd(&bc.loop, 1u);
            if (status == ST_EXISTS) atomicAdd(&bc.exists, 1u);
        }
    }
    flush_counts(&bc, ctr);
}

// ---------------------------------------------------------------------------
// Decision of one switch from the table (Alg. 1's lookup / lookup_min and
// its legal / illegal / delayed rule).
// ---------------------------------------------------------------------------
enum Verdict : int { V_OK = 0, V_WAIT = 1, V_ILLEGAL = 2 };

__device__ __forceinline__ uint8_t load_status(const uint8_t *st, uint32_t k) {
    return __hip_atomic_load(st + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int judge_target(const Slot *tab, uint32_t s, uint32_t k, const uint8_t *st,
                                            uint32_t *claim_out, uint32_t *err) {
    const uint32_t e = tab[s].eraser;
    const uint32_t cw = __hip_atomic_load(&tab[s].claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *claim_out = cw;
    int v = V_OK;
    // erase side: X in E0 survives unless its eraser is an earlier legal switch
    if (e != kNoEraser) {
        if (e == kStays || e >= k) return V_ILLEGAL;
        const uint8_t se = load_status(st, e);
        if (se == ST_UNDECIDED)
            v = V_WAIT;
        else if (se != ST_LEGAL)
            return V_ILLEGAL;
    }
    // insert side: the earliest not-excluded inserter of X
    const uint32_t q = cw >> 2;
    if (q < k) {
        if (cw & kClaimLegal) return V_ILLEGAL;
        if (load_status(st, q) == ST_LEGAL) return V_ILLEGAL;
        v = V_WAIT;  // q undecided, or rejected (a later inserter may still precede k)
    } else if (q > k) {
        atomicOr(err, ERR_INTERNAL);  // k is an inserter, so the minimum cannot exceed it
        v = V_WAIT;
    }
    return v;
}

// Wave-aggregated append of k to the undecided list.
__device__ __forceinline__ void append_undecided(bool want, uint32_t k, uint32_t *list, uint32_t *count,
                                                 unsigned long long *tally = nullptr) {
    const unsigned long long mask = __ballot(want);
    if (mask == 0) return;
    const uint32_t lane = __lane_id();
    const uint32_t leader = __ffsll((long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader) {
        base = atomicAdd(count, (uint32_t)__popcll(mask));
        if (tally) atomicAdd(tally, (unsigned long long)__popcll(mask));
    }
    base = __shfl(base, leader);
    if (want) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = k;
}

// Decides switch k (all inputs re-read; writes the outcome, the output
// records and the LEGAL marks).  Returns true if k stays undecided.
__device__ __forceinline__ bool decide_switch(uint32_t k, const uint32_t *s_idx, const unsigned long long *s_key,
                                              Slot *tab, const uint32_t *sw_slot, uint8_t *st, uint32_t *out_idx,
                                              unsigned long long *out_key, bool always_mark, BlockCounts *bc,
                                              uint32_t *err) {
    const uint32_t i = s_idx[2 * k], j = s_idx[2 * k + 1];
    const unsigned long long e1 = s_key[2 * k], e2 = s_key[2 * k + 1];
    const uint32_t sa = sw_slot[2 * k], sb = sw_slot[2 * k + 1];
    uint32_t ca = 0, cb = 0;
    if (sa == kNoSlot || sb == kNoSlot) {  // build already flagged the error; decide it away
        __hip_atomic_store(st + k, (uint8_t)ST_EXISTS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
    }
    const int va = judge_target(tab, sa, k, st, &ca, err);
    const int vb = judge_target(tab, sb, k, st, &cb, err);
    const int v = max(va, vb);
    if (v == V_WAIT) return true;
    if (v == V_OK) {
        const Targets T = switch_targets(e1, e2, i < j);
        out_idx[2 * k] = i;
        out_key[2 * k] = T.A;
        out_idx[2 * k + 1] = j;
        out_key[2 * k + 1] = T.B;
        if (always_mark || (ca & kClaimContended)) atomicOr(&tab[sa].claim, kClaimLegal);
        if (always_mark || (cb & kClaimContended)) atomicOr(&tab[sb].claim, kClaimLegal);
        __hip_atomic_store(st + k, (uint8_t)ST_LEGAL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        atomicAdd(&bc->legal, 1u);
    } else {
        out_idx[2 * k] = i;
        out_key[2 * k] = e1;
        out_idx[2 * k + 1] = j;
        out_key[2 * k + 1] = e2;
        __hip_atomic_store(st + k, (uint8_t)ST_EXISTS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        atomicAdd(&bc->exists, 1u);
    }
    return false;
}

// Round 1: every switch not decided by the build kernel.
__global__ __launch_bounds__(kBlock) void k_decide_first(const uint32_t *__restrict__ s_idx,
                                                         const unsigned long long *__restrict__ s_key, uint32_t ell,
                                                         Slot *tab, const uint32_t *__restrict__ sw_slot, uint8_t *st,
                                                         uint32_t *__restrict__ out_idx,
                                                         unsigned long long *__restrict__ out_key,
                                                         uint32_t *__restrict__ list, uint32_t *__restrict__ count,
                                                         StepCounters *ctr, uint32_t *__restrict__ err) {
    __shared__ BlockCounts bc;
    if (threadIdx.x == 0) bc = BlockCounts{0, 0, 0, 0};
    __syncthreads();
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    bool wait = false;
    if (k < ell && st[k] == ST_UNDECIDED)
        wait = decide_switch(k, s_idx, s_key, tab, sw_slot, st, out_idx, out_key, false, &bc, err);
    append_undecided(wait, k, list, count, &ctr->undecided_round1);
    flush_counts(&bc, ctr);
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&ctr->rounds, 1ull);
}

// Rounds >= 2, phase 1: clear the (not frozen) claims of listed targets and
// the next round's list counter.
__global__ __launch_bounds__(kBlock) void k_round_reset(const uint32_t *__restrict__ list,
                                                        const uint32_t *__restrict__ count, uint32_t ell, Slot *tab,
                                                        const uint32_t *__restrict__ sw_slot,
                                                        uint32_t *__restrict__ next_count) {
    const uint32_t n = min(*count, ell);
    const uint32_t stride = gridDim.x * kBlock;
    if (blockIdx.x == 0 && threadIdx.x == 0) *next_count = 0;
    for (uint32_t q = blockIdx.x * kBlock + threadIdx.x; q < n; q += stride) {
        const uint32_t k = list[q];
        if (k >= ell) continue;
        for (int h = 0; h < 2; ++h) {
            const uint32_t sl = sw_slot[2 * k + h];
            if (sl == kNoSlot) continue;
            uint32_t *c = &tab[sl].claim;
            if (!(*c & kClaimLegal)) *c = kClaimNone;
        }
    }
}

// Phase 2: listed switches claim their targets again (earliest wins).
__global__ __launch_bounds__(kBlock) void k_round_claim(const uint32_t *__restrict__ list,
                                                        const uint32_t *__restrict__ count, uint32_t ell, Slot *tab,
                                                        const uint32_t *__restrict__ sw_slot) {
    const uint32_t n = min(*count, ell);
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t q = blockIdx.x * kBlock + threadIdx.x; q < n; q += stride) {
        const uint32_t k = list[q];
        if (k >= ell) continue;
        for (int h = 0; h < 2; ++h) {
            const uint32_t sl = sw_slot[2 * k + h];
            if (sl == kNoSlot) continue;
            uint32_t *c = &tab[sl].claim;
            if (!(__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kClaimLegal)) atomicMin(c, k << 2);
        }
    }
}

// Phase 3: listed switches decide; the still undecided form the next list.
__global__ __launch_bounds__(kBlock) void k_round_decide(const uint32_t *__restrict__ s_idx,
                                                         const unsigned long long *__restrict__ s_key, uint32_t ell,
                                                         Slot *tab, const uint32_t *__restrict__ sw_slot, uint8_t *st,
                                                         uint32_t *__restrict__ out_idx,
                                                         unsigned long long *__restrict__ out_key,
                                                         const uint32_t *__restrict__ list,
                                                         const uint32_t *__restrict__ count,
                                                         uint32_t *__restrict__ next_list,
                                                         uint32_t *__restrict__ next_count, StepCounters *ctr,
                                                         uint32_t *__restrict__ err) {
    __shared__ BlockCounts bc;
    if (threadIdx.x == 0) bc = BlockCounts{0, 0, 0, 0};
    __syncthreads();
    const uint32_t n = min(*count, ell);
    const uint32_t stride = gridDim.x * kBlock;
    const uint32_t rounds_up = (n + stride - 1) / stride;  // uniform trip count for the wave ballots
    for (uint32_t r = 0; r < rounds_up; ++r) {
        const uint32_t q = r * stride + blockIdx.x * kBlock + threadIdx.x;
        bool wait = false;
        uint32_t k = 0;
        if (q < n) {
            k = list[q];
            if (k < ell && st[k] == ST_UNDECIDED)
                wait = decide_switch(k, s_idx, s_key, tab, sw_slot, st, out_idx, out_key, true, &bc, err);
        }
        append_undecided(wait, k, next_list, next_count);
    }
    flush_counts(&bc, ctr);
    if (blockIdx.x == 0 && threadIdx.x == 0 && n > 0) atomicAdd(&ctr->rounds, 1ull);
}

// Remaining rounds inside one workgroup (barriers instead of kernel
// boundaries), until no switch is undecided.
constexpr int kFinishBlock = 1024;

__global__ __launch_bounds__(kFinishBlock) void k_finish(const uint32_t *__restrict__ s_idx,
                                                         const unsigned long long *__restrict__ s_key, uint32_t ell,
                                                         Slot *tab, const uint32_t *__restrict__ sw_slot, uint8_t *st,
                                                         uint32_t *__restrict__ out_idx,
                                                         unsigned long long *__restrict__ out_key, uint32_t *list_a,
                                                         uint32_t *count_a, uint32_t *list_b, uint32_t *count_b,
                                                         StepCounters *ctr, uint32_t *__restrict__ err) {
    __shared__ BlockCounts bc;
    __shared__ uint32_t s_n;
    const uint32_t tid = threadIdx.x;
    if (tid == 0) {
        bc = BlockCounts{0, 0, 0, 0};
        s_n = min(*count_a, ell);
    }
    __syncthreads();
    uint32_t *cur = list_a, *nxt = list_b, *ncnt_cur = count_a, *ncnt_nxt = count_b;
    uint32_t n = s_n;
    uint64_t guard = 0;
    while (n > 0) {
        if (++guard > (uint64_t)ell + 2) {
            if (tid == 0) atomicOr(err, ERR_INTERNAL);
            break;
        }
        if (tid == 0) *ncnt_nxt = 0;
        for (uint32_t q = tid; q < n; q += kFinishBlock) {
            const uint32_t k = cur[q];
            if (k >= ell) continue;
            for (int h = 0; h < 2; ++h) {
                const uint32_t sl = sw_slot[2 * k + h];
                if (sl == kNoSlot) continue;
                uint32_t *c = &tab[sl].claim;
                if (!(*c & kClaimLegal)) *c = kClaimNone;
            }
        }
        __threadfence();
        __syncthreads();
        for (uint32_t q = tid; q < n; q += kFinishBlock) {
            const uint32_t k = cur[q];
            if (k >= ell) continue;
            for (int h = 0; h < 2; ++h) {
                const uint32_t sl = sw_slot[2 * k + h];
                if (sl == kNoSlot) continue;
                uint32_t *c = &tab[sl].claim;
                if (!(__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kClaimLegal))
                    atomicMin(c, k << 2);
            }
        }
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
                    wait = decide_switch(k, s_idx, s_key, tab, sw_slot, st, out_idx, out_key, true, &bc, err);
            }
            append_undecided(wait, k, nxt, ncnt_nxt);
        }
        __threadfence();
        __syncthreads();
        if (tid == 0) {
            const uint32_t nn = min(*ncnt_nxt, ell);
            // the smallest undecided switch always decides; no progress = a bug
            if (nn >= n) atomicOr(err, ERR_INTERNAL);
            s_n = nn >= n ? 0 : nn;
            atomicAdd(&ctr->rounds, 1ull);
        }
        __syncthreads();
        n = s_n;
        uint32_t *tl = cur;
        cur = nxt;
        nxt = tl;
        uint32_t *tc = ncnt_cur;
        ncnt_cur = ncnt_nxt;
        ncnt_nxt = tc;
    }
    flush_counts(&bc, ctr);
}

// ---------------------------------------------------------------------------
// Final placement: out[i] = edge of record with index i (skipped on error,
// leaving the caller's output untouched).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_unpermute(const uint32_t *__restrict__ idx,
                                                      const unsigned long long *__restrict__ key, uint32_t m,
                                                      unsigned long long *__restrict__ out,
                                                      const uint32_t *__restrict__ err) {
    if (*err) return;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t r = (uint64_t)blockIdx.x * kBlock + threadIdx.x; r < m; r += stride) {
        const uint32_t i = idx[r];
        if (i < m) out[i] = key[r];
    }
}

// The write-back of large states after their records were distributed into
// buckets of consecutive input indices (bucket b = records [boff[b],
// boff[b+1]), indices below 2^20 apart): workgroup w runs on XCD w % 8 and
// the workgroups of one XCD take its buckets b = x, x + 8, ... together, so
// at any time each XCD writes into one window of `out` (at most 8 MB, 1 MB at
// 2^26 edges) instead of all of it.  The stores still leave L2 as 32-byte
// partial writes (the request-size counters show no merging), so the gain is
// locality, not fewer bytes.  The grid is a multiple of 8.  Skipped entirely
// if an error flag is set (output untouched).
__global__ __launch_bounds__(kBlock) void k_unpermute_buckets(const uint32_t *__restrict__ idx,
                                                              const unsigned long long *__restrict__ key,
                                                              const uint32_t *__restrict__ boff, uint32_t nb,
                                                              uint32_t m, unsigned long long *__restrict__ out,
                                                              const uint32_t *__restrict__ err) {
    if (*err) return;
    constexpr uint32_t kXcd = 8;
    const uint32_t x = blockIdx.x % kXcd, j = blockIdx.x / kXcd, per = gridDim.x / kXcd;
    for (uint32_t b = x; b < nb; b += kXcd) {
        const uint32_t lo = boff[b], hi = boff[b + 1];
        for (uint32_t r = lo + j * kBlock + threadIdx.x; r < hi; r += per * kBlock) {
            const uint32_t i = idx[r];
            if (i < m) out[i] = key[r];
        }
    }
}

// pi[r] = index of sorted record r (building block exposed for checks).
__global__ __launch_bounds__(kBlock) void k_extract_pi(const uint32_t *__restrict__ idx, uint32_t m,
                                                       uint32_t *__restrict__ pi) {
    const uint64_t r = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r < m) pi[r] = idx[r];
}

}  // namespace gesmc

// ParES (Alg. 2 of arXiv 2111.03005): the exact parallel execution of the
// Edge Switching Markov Chain (ES-MC, Def. 2.1) on gfx950.
//
// ES-MC applies r edge switches in sequence; switch k draws
//   (x0, x1, x2, x3) = Philox(ctr = (k_lo, k_hi, 0, 2), key = seed)
//   i = floor(((x0 << 32) | x1) * m / 2^64)
//   j' = floor(((x2 << 32) | x3) * (m - 1) / 2^64),  j = j' + [j' >= i]
//   g = x1 & 1
// (distinct indices, as Alg. 2 samples them).  Alg. 2 cuts the sequence into
// supersteps without source dependencies -- runs of switches whose edge
// indices are pairwise distinct -- and runs each one with the superstep
// algorithm of Sec. 4 (Alg. 1).  Any such cut gives the sequential result, so
// a superstep here is also capped at one switch per thread.
//
// One workgroup owns one graph for a whole launch and walks its switches:
//   A. draws of the next kEsThreads switches; superstep boundary by
//      insert_if_min over their edge indices in an LDS table (the smallest
//      later switch that reuses an index is the first one left out);
//   B. sources E[i], E[j] and their table slots; targets tau(e1, e2, g); a
//      probe of the HBM edge set for each target that is not a loop;
//   C. ERASE (sources) and INSERT (targets) tuples in LDS, linked per cell of
//      key-hash bits;
//   D. per target: the switch erasing that key in this superstep (if any) and
//      the previous inserter of the same key;
//   E. rounds of Alg. 1's rule until every switch is decided;
//   F. accepted switches write E[i], E[j], retire their sources' slots and
//      insert their targets into the edge set.
// The edge set is open addressing with linear probing and tombstones over a
// power-of-two slot count; the host rebuilds it between launches (epochs), so
// that at most m + 2 * (switches of the epoch) slots are ever used and the load
// stays at or below one half.
#pragma once

#include "device_common.h"

namespace gesmc {

constexpr int kEsThreads = 1024;                 // switches per superstep at most (one per thread)
constexpr uint32_t kEsIdxSlots = 4096;           // LDS table of the boundary search (2 indices per switch)
constexpr uint32_t kEsCells = 2048;              // LDS cells of the tuples
constexpr uint32_t kEsNone = 0xFFFFFFFFu;
constexpr unsigned long long kEsEmpty = ~0ull;   // never a valid (min, max) key
constexpr unsigned long long kEsTomb = ~0ull - 1;

// Counters of one launch (device, cleared by the host's zero kernel).
struct EsCounters {
    unsigned long long legal, rej_loop, rej_exists, supersteps, rounds, rounds_max, used_slots, pad;
};

__device__ __forceinline__ uint64_t es_mulhi(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

struct EsDraw {
    uint32_t i, j;
    bool g;
};

// Switch k's draw on m >= 2 edges (the definition above).
__device__ __forceinline__ EsDraw es_draw(uint64_t k, uint32_t m, uint32_t k0, uint32_t k1) {
    const Philox4 x = philox4x32_10((uint32_t)k, (uint32_t)(k >> 32), 0u, 2u, k0, k1);
    const uint64_t w0 = ((uint64_t)x.x0 << 32) | x.x1, w1 = ((uint64_t)x.x2 << 32) | x.x3;
    EsDraw d;
    d.i = (uint32_t)es_mulhi(w0, m);
    const uint32_t jp = (uint32_t)es_mulhi(w1, (uint64_t)m - 1);
    d.j = jp + (jp >= d.i ? 1u : 0u);
    d.g = (x.x1 & 1u) != 0;
    return d;
}

__device__ __forceinline__ uint32_t es_home(unsigned long long key, uint32_t mask) {
    return (uint32_t)slot_hash(key) & mask;
}

// Accesses of the chain kernel to the edge list, slots and edge set.  One
// workgroup owns a graph for a whole launch, so workgroup scope suffices:
// loads and compare-and-swaps are served by the CU's own caches and its
// XCD's L2 instead of going memory-side, and the workgroup barrier between
// supersteps orders them.  (Kernel boundaries order them with the build
// kernels, which use device-scope atomics across workgroups.)
__device__ __forceinline__ unsigned long long es_load64(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t es_load32(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ unsigned long long es_cas(unsigned long long *p, unsigned long long expected,
                                                     unsigned long long desired) {
    __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
    return expected;  // the value found (equal to the expected one on success)
}

// Probes the edge set for two keys at once (their linear-probing chains
// interleaved, so the loads of both are in flight together).  For each key:
// whether it is present, and the first free slot of its chain (a retired
// slot before the end, else the empty slot that ends the chain) with the
// value seen there -- where an insert of the key may go.  The chains end at
// an empty slot (load <= 1/2); their length is bounded by the slot count.
struct EsProbe {
    bool found;
    uint32_t free_slot;
    unsigned long long free_seen;
};

__device__ __forceinline__ void es_probe2(const unsigned long long *H, uint32_t mask, unsigned long long ka,
                                          unsigned long long kb, EsProbe *pa, EsProbe *pb, uint32_t *err) {
    uint32_t sa = es_home(ka, mask), sb = es_home(kb, mask);
    bool da = false, db = false;
    pa->found = pb->found = false;
    pa->free_slot = pb->free_slot = kEsNone;
    pa->free_seen = pb->free_seen = kEsEmpty;
    // one slot of each chain per step: a single workgroup is bound by the
    // random lines it keeps in flight, so wider steps (measured: four slots)
    // only add loads
    for (uint32_t p = 0; p <= mask && !(da && db); ++p) {
        const unsigned long long ca = da ? 0 : es_load64(H + sa);
        const unsigned long long cb = db ? 0 : es_load64(H + sb);
        if (!da) {
            if (ca == ka) {
                pa->found = true;
                da = true;
            } else if (ca == kEsEmpty || ca == kEsTomb) {
                if (pa->free_slot == kEsNone) {
                    pa->free_slot = sa;
                    pa->free_seen = ca;
                }
                da = ca == kEsEmpty;
            }
            sa = (sa + 1) & mask;
        }
        if (!db) {
            if (cb == kb) {
                pb->found = true;
                db = true;
            } else if (cb == kEsEmpty || cb == kEsTomb) {
                if (pb->free_slot == kEsNone) {
                    pb->free_slot = sb;
                    pb->free_seen = cb;
                }
                db = cb == kEsEmpty;
            }
            sb = (sb + 1) & mask;
        }
    }
    if (!(da && db)) atomicOr(err, ERR_INTERNAL);
}

// Inserts `key` (absent once its superstep's erases are done) at the first
// empty or retired slot of its chain from slot s on; returns the slot.
// *fresh is set if it took an empty one.
__device__ __forceinline__ uint32_t es_insert_from(unsigned long long *H, uint32_t mask, uint32_t s,
                                                   unsigned long long key, bool *fresh, uint32_t *err) {
    // a slot changes at most twice in a superstep (retired once, taken once),
    // so the lost races are bounded too
    for (uint32_t p = 0, tries = 0; p <= mask && tries < 2 * mask + 64; ++tries) {
        const unsigned long long cur = es_load64(H + s);
        if (cur == kEsEmpty || cur == kEsTomb) {
            const unsigned long long prev = es_cas(H + s, cur, key);
            if (prev == cur) {
                *fresh = cur == kEsEmpty;
                return s;
            }
            continue;  // taken meanwhile: look at the same slot again
        }
        s = (s + 1) & mask;
        ++p;
    }
    atomicOr(err, ERR_INTERNAL);
    return 0;
}

// ---- the edge set between launches ---------------------------------------
__global__ __launch_bounds__(kBlock) void k_es_clear(unsigned long long *__restrict__ H, uint64_t nslots) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t q = (uint64_t)blockIdx.x * kBlock + threadIdx.x; q < nslots; q += stride) H[q] = kEsEmpty;
}

// Inserts every edge (slot_of[i] = its slot); a key met twice is a duplicate
// edge of the input (ERR_DUP).
__global__ __launch_bounds__(kBlock) void k_es_insert_all(const unsigned long long *__restrict__ E, uint32_t m,
                                                          unsigned long long *__restrict__ H, uint32_t mask,
                                                          uint32_t *__restrict__ slot_of, uint32_t *__restrict__ err,
                                                          EsCounters *ctr) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        const unsigned long long key = E[i];
        uint32_t s = es_home(key, mask);
        bool done = false;
        for (uint32_t p = 0; p <= mask && !done; ++p) {
            const unsigned long long prev = atomicCAS(H + s, kEsEmpty, key);
            if (prev == kEsEmpty) {
                slot_of[i] = s;
                done = true;
            } else if (prev == key) {
                atomicOr(err, ERR_DUP);
                done = true;
            } else {
                s = (s + 1) & mask;
            }
        }
        if (!done) atomicOr(err, ERR_INTERNAL);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&ctr->used_slots, (unsigned long long)m);
}

// Copies the result to the caller's buffer unless an error was raised.
__global__ __launch_bounds__(kBlock) void k_es_out(const unsigned long long *__restrict__ E, uint32_t m,
                                                   unsigned long long *__restrict__ out,
                                                   const uint32_t *__restrict__ err) {
    if (*err) return;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) out[i] = E[i];
}

// The draws of switches k0 .. k0 + count - 1 (parity hook).
__global__ __launch_bounds__(kBlock) void k_es_draws(uint64_t k0, uint64_t count, uint32_t m, uint32_t s0,
                                                     uint32_t s1, unsigned long long *__restrict__ di,
                                                     unsigned long long *__restrict__ dj, uint8_t *__restrict__ dg) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t q = (uint64_t)blockIdx.x * kBlock + threadIdx.x; q < count; q += stride) {
        const EsDraw d = es_draw(k0 + q, m, s0, s1);
        di[q] = d.i;
        dj[q] = d.j;
        dg[q] = d.g ? 1 : 0;
    }
}

// ---- the ParES chain -------------------------------------------------------
// Outcome of one target when its switch runs.
enum : int { ES_ABSENT = 0, ES_WAIT = 1, ES_PRESENT = 2 };

struct EsShared {
    uint32_t ikey[kEsIdxSlots];   // A: edge index (kEsNone: empty)
    uint32_t ival[kEsIdxSlots];   // A: smallest local switch that drew it
};

struct EsTuples {
    unsigned long long key[4 * kEsThreads];  // tuple 4q + h: ERASE source h (h < 2), INSERT target h - 2
    uint32_t next[4 * kEsThreads];           // cell list link
    uint32_t head[kEsCells];
};

// Switches k = kbeg .. kend - 1 of one graph (one workgroup, kEsThreads
// threads).  E, slot_of and H are the graph's edge list, slots and edge set
// (mask = slot count - 1).  outcome (nullable) receives the outcome code of
// switch k at outcome[k - kbase].
__global__ __launch_bounds__(kEsThreads) void k_es_chain(unsigned long long *__restrict__ E,
                                                         uint32_t *__restrict__ slot_of,
                                                         unsigned long long *__restrict__ H, uint32_t mask,
                                                         uint32_t m, uint32_t s0, uint32_t s1, uint64_t kbeg,
                                                         uint64_t kend, uint64_t kbase, uint8_t *__restrict__ outcome,
                                                         EsCounters *__restrict__ ctr, uint32_t *__restrict__ err) {
    __shared__ union {
        EsShared a;
        EsTuples t;
    } sh;
    __shared__ uint32_t pred[2 * kEsThreads];  // INSERT tuple -> previous inserter's tuple of the same key
    __shared__ uint8_t st[kEsThreads];
    __shared__ uint32_t s_len, s_more;
    __shared__ unsigned long long s_start;
    __shared__ uint32_t c_legal, c_loop, c_exists, c_rounds, c_steps, c_fresh, c_rmax;
    const uint32_t tid = threadIdx.x;
    if (tid == 0) {
        s_start = kbeg;
        c_legal = c_loop = c_exists = c_rounds = c_steps = c_fresh = c_rmax = 0;
    }
    __syncthreads();
    // nothing to do, or the input failed its checks (the edge set may then be incomplete)
    if (m < 2 || *err != 0) return;
    for (;;) {
        const uint64_t s = s_start;  // uniform: written by thread 0 before the barrier that ends a superstep
        if (s >= kend) break;
        const uint64_t rem64 = kend - s;
        const uint32_t cand = rem64 < (uint64_t)kEsThreads ? (uint32_t)rem64 : (uint32_t)kEsThreads;
        // ---- A: draws and the superstep boundary --------------------------
        for (uint32_t q = tid; q < kEsIdxSlots; q += kEsThreads) {
            sh.a.ikey[q] = kEsNone;
            sh.a.ival[q] = kEsNone;
        }
        if (tid == 0) s_len = cand;
        __syncthreads();
        EsDraw d{0, 0, false};
        if (tid < cand) {
            d = es_draw(s + tid, m, s0, s1);
            uint32_t coll = kEsNone;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const uint32_t x = h ? d.j : d.i;
                uint32_t q = (uint32_t)(slot_hash(x) & (kEsIdxSlots - 1));
                for (uint32_t p = 0; p < kEsIdxSlots; ++p) {
                    const uint32_t prev = atomicCAS(&sh.a.ikey[q], kEsNone, x);
                    if (prev == kEsNone || prev == x) {
                        // insert_if_min: the earlier of two switches sharing an
                        // index keeps it; the later one bounds the superstep
                        const uint32_t old = atomicMin(&sh.a.ival[q], tid);
                        if (old != kEsNone) coll = min(coll, max(old, tid));
                        break;
                    }
                    q = (q + 1) & (kEsIdxSlots - 1);
                }
            }
            if (coll != kEsNone) atomicMin(&s_len, coll);
        }
        __syncthreads();
        const uint32_t L = s_len;  // switches s .. s + L - 1 share no edge index
        const bool act = tid < L;
        // ---- B: sources, targets, presence in the edge set ---------------
        unsigned long long e1 = 0, e2 = 0;
        uint32_t so1 = 0, so2 = 0;
        Targets T{0, 0, true};
        EsProbe pr[2];
        pr[0].found = pr[1].found = false;
        if (act) {
            e1 = es_load64(E + d.i);
            e2 = es_load64(E + d.j);
            so1 = es_load32(slot_of + d.i);
            so2 = es_load32(slot_of + d.j);
            T = switch_targets(e1, e2, d.g);
            if (!T.loop) es_probe2(H, mask, T.A, T.B, &pr[0], &pr[1], err);
        }
        const bool ex[2] = {pr[0].found, pr[1].found};
        // ---- C: tuples in LDS cells (the boundary table is no longer needed)
        __syncthreads();
        for (uint32_t q = tid; q < kEsCells; q += kEsThreads) sh.t.head[q] = kEsNone;
        if (act) st[tid] = T.loop ? ST_LOOP : ST_UNDECIDED;
        __syncthreads();
        if (act) {
            const unsigned long long kk[4] = {e1, e2, T.A, T.B};
            const int nt = T.loop ? 2 : 4;  // a loop inserts nothing
            for (int h = 0; h < nt; ++h) {
                const uint32_t t = 4 * tid + h;
                sh.t.key[t] = kk[h];
                sh.t.next[t] = atomicExch(&sh.t.head[(uint32_t)slot_hash(kk[h]) & (kEsCells - 1)], t);
            }
        }
        __syncthreads();
        // ---- D: eraser and previous inserter of each target ---------------
        uint32_t er[2] = {kEsNone, kEsNone};
        if (act && !T.loop) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const unsigned long long key = h ? T.B : T.A;
                uint32_t best = kEsNone;
                for (uint32_t t = sh.t.head[(uint32_t)slot_hash(key) & (kEsCells - 1)]; t != kEsNone;
                     t = sh.t.next[t]) {
                    if (sh.t.key[t] != key) continue;
                    const uint32_t q = t >> 2;
                    if ((t & 3u) < 2u) {
                        er[h] = q;  // a key is a source of at most one switch: indices are distinct
                    } else if (q < tid && (best == kEsNone || q > (best >> 2))) {
                        best = t;
                    }
                }
                pred[2 * tid + h] = best;
            }
        }
        __syncthreads();
        // ---- E: rounds of Alg. 1's rule -----------------------------------
        uint32_t rounds = 0;
        for (;;) {
            bool undecided = act && st[tid] == ST_UNDECIDED;
            if (undecided) {
                int v = ES_ABSENT;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    int w = ES_ABSENT;
                    bool chain = true;
                    if (ex[h]) {  // in the edge set when the superstep starts
                        const uint32_t p = er[h];
                        if (p == kEsNone || p >= tid) {
                            w = ES_PRESENT;  // never erased before this switch (its own source included)
                            chain = false;
                        } else {
                            const uint8_t sp = st[p];
                            if (sp == ST_UNDECIDED) {
                                w = ES_WAIT;
                                chain = false;
                            } else if (sp != ST_LEGAL) {
                                w = ES_PRESENT;
                                chain = false;
                            }
                        }
                    }
                    for (uint32_t t = chain ? pred[2 * tid + h] : kEsNone; t != kEsNone;) {
                        const uint8_t sq = st[t >> 2];
                        if (sq == ST_UNDECIDED) {
                            w = ES_WAIT;
                            break;
                        }
                        if (sq == ST_LEGAL) {
                            w = ES_PRESENT;
                            break;
                        }
                        t = pred[2 * (t >> 2) + (t & 1u)];  // an earlier inserter of the same key
                    }
                    v = max(v, w);
                }
                if (v != ES_WAIT) {
                    st[tid] = v == ES_PRESENT ? ST_EXISTS : ST_LEGAL;
                    undecided = false;
                }
            }
            ++rounds;
            if (!__syncthreads_or(undecided)) break;
            if (rounds > L) {  // the smallest undecided switch always decides
                if (tid == 0) atomicOr(err, ERR_INTERNAL);
                break;
            }
        }
        // ---- F: apply -----------------------------------------------------
        if (act) {
            const uint8_t sk = st[tid];
            if (sk == ST_LEGAL) {
                E[d.i] = T.A;
                E[d.j] = T.B;
                H[so1] = kEsTomb;
                H[so2] = kEsTomb;
                // A target its probe did not find goes to the free slot the probe
                // saw, if that is still free (both compare-and-swaps in flight
                // together), else further along its chain.  A target that was
                // present (its eraser runs earlier in this superstep) is
                // inserted from its home slot.
                const bool qa = !pr[0].found && pr[0].free_slot != kEsNone;
                const bool qb = !pr[1].found && pr[1].free_slot != kEsNone;
                const unsigned long long ga = qa ? es_cas(H + pr[0].free_slot, pr[0].free_seen, T.A) : 0;
                const unsigned long long gb = qb ? es_cas(H + pr[1].free_slot, pr[1].free_seen, T.B) : 0;
                bool f1 = pr[0].free_seen == kEsEmpty, f2 = pr[1].free_seen == kEsEmpty;
                uint32_t sa = pr[0].free_slot, sb = pr[1].free_slot;
                if (!qa || ga != pr[0].free_seen)
                    sa = es_insert_from(H, mask, qa ? sa : es_home(T.A, mask), T.A, &f1, err);
                if (!qb || gb != pr[1].free_seen)
                    sb = es_insert_from(H, mask, qb ? sb : es_home(T.B, mask), T.B, &f2, err);
                slot_of[d.i] = sa;
                slot_of[d.j] = sb;
                atomicAdd(&c_legal, 1u);
                if (f1 || f2) atomicAdd(&c_fresh, (uint32_t)f1 + (uint32_t)f2);
            } else if (sk == ST_LOOP) {
                atomicAdd(&c_loop, 1u);
            } else {
                atomicAdd(&c_exists, 1u);
            }
            if (outcome) outcome[s + tid - kbase] = sk == ST_UNDECIDED ? ST_EXISTS : sk;
        }
        // every access to the graph's arrays in this launch comes from this
        // workgroup (one CU, one L2), so the barrier orders the writes above
        // before the next superstep's loads; no device-wide fence is needed
        if (tid == 0) {
            s_start = s + L;
            ++c_steps;
            c_rounds += rounds;
            c_rmax = max(c_rmax, rounds);
        }
        __syncthreads();
    }
    if (tid == 0) {
        atomicAdd(&ctr->legal, (unsigned long long)c_legal);
        atomicAdd(&ctr->rej_loop, (unsigned long long)c_loop);
        atomicAdd(&ctr->rej_exists, (unsigned long long)c_exists);
        atomicAdd(&ctr->supersteps, (unsigned long long)c_steps);
        atomicAdd(&ctr->rounds, (unsigned long long)c_rounds);
        atomicMax(&ctr->rounds_max, (unsigned long long)c_rmax);
        atomicAdd(&ctr->used_slots, (unsigned long long)c_fresh);
    }
}

}  // namespace gesmc

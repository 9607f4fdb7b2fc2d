// Device-side building blocks shared by the gfx950 kernels of libgesmc.
//
// Counter-based randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11).  Every random choice
// of a global switch (Def. 3.2 of arXiv 2111.03005) is a pure function of
// (seed, superstep t, index), so any kernel can recompute it instead of
// storing it:
//   permutation key of edge index i : K_i = (x0 << 32) | x1 at counter (i, 0, t, 0)
//   P_L skip test of switch k       : x0 at counter (k, 0, t, 1), skip iff x0 < pl
// The permutation pi of superstep t lists the edge indices in ascending
// (K_i, i) order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tuple_pack.h"

namespace gesmc {

constexpr int kBlock = 256;  // threads per workgroup (4 wave64s)

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also
// fences global memory, which makes every wave wait for its outstanding
// global loads -- including loads issued early to prefetch the next tile.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// Philox4x32-10
// ---------------------------------------------------------------------------
struct Philox4 {
    uint32_t x0, x1, x2, x3;
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                 uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // each 32x32 -> 64 product in one instruction (v_mad_u64_u32) rather
        // than separate high and low multiplies
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t h0 = (uint32_t)(p0 >> 32), l0 = (uint32_t)p0;
        const uint32_t h1 = (uint32_t)(p1 >> 32), l1 = (uint32_t)p1;
        const uint32_t y0 = h1 ^ c1 ^ k0;
        const uint32_t y2 = h0 ^ c3 ^ k1;
        c0 = y0;
        c1 = l1;
        c2 = y2;
        c3 = l0;
        k0 += 0x9E3779B9u;  // Weyl key schedule
        k1 += 0xBB67AE85u;
    }
    return Philox4{c0, c1, c2, c3};
}

// Permutation key of edge index i in superstep t (m < 2^32, so the high
// counter word of i is 0).
__device__ __forceinline__ uint64_t perm_key(uint32_t i, uint32_t t, uint32_t k0, uint32_t k1) {
    const Philox4 r = philox4x32_10(i, 0u, t, 0u, k0, k1);
    return ((uint64_t)r.x0 << 32) | r.x1;
}

__device__ __forceinline__ bool pl_skip(uint32_t k, uint32_t t, uint32_t pl, uint32_t k0, uint32_t k1) {
    if (pl == 0) return false;
    return philox4x32_10(k, 0u, t, 1u, k0, k1).x0 < pl;
}

// ---------------------------------------------------------------------------
// Edge keys (Sec. 5.1): smaller endpoint in the high word, larger in the low.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t ekey_lo_vertex(uint64_t e) { return (uint32_t)(e >> 32); }
__device__ __forceinline__ uint32_t ekey_hi_vertex(uint64_t e) { return (uint32_t)e; }
__device__ __forceinline__ uint64_t ekey(uint32_t a, uint32_t b) {
    const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
    return ((uint64_t)lo << 32) | hi;
}

// Per-switch outcome codes (also the status array of a superstep).  ST_IDLE
// marks a pair holding a graph's padding record in a batch (no attempt).
enum : uint8_t { ST_UNDECIDED = 0, ST_LEGAL = 1, ST_LOOP = 2, ST_EXISTS = 3, ST_PL = 4, ST_IDLE = 5 };

// ---------------------------------------------------------------------------
// Batches of independent graphs.  Graph vertex ids are shifted by a per-graph
// base so that the batch is one simple graph (a disjoint union) whose
// switches never mix graphs: every graph owns an even-length segment of the
// switch positions (a graph of odd m gets one padding record that the
// permutation places last, so its pair is idle -- the idle position of odd m).
// The permutation of graph g sorts by (K_i, i) with g's own seed, local
// index i and superstep t0_g + s; its buckets are numbered globally so that
// bucket order is (graph, K range).
// ---------------------------------------------------------------------------
constexpr uint32_t kPadIdx = 0xFFFFFFFFu;  // index of a padding record (its key sorts last)

struct BatchGraph {
    uint32_t poff;   // first switch position of the graph's segment (even)
    uint32_t mpad;   // records in the segment: m, +1 if m is odd
    uint32_t goff;   // first input position (local index = input position - goff)
    uint32_t vbase;  // vertex id shift
    uint32_t k0, k1; // Philox key (seed)
    uint32_t t0;     // superstep of the batch's first superstep
    uint32_t nb;     // permutation buckets of the graph
    uint32_t bbase;  // its first global bucket
    uint32_t m, n;   // edges, vertices
    uint32_t pl;     // P_L = pl / 2^32 of the graph
};

// Switch k's targets from its sources (tau of Def. 2.1 on canonical edges).
struct Targets {
    uint64_t A, B;
    bool loop;
};

__device__ __forceinline__ Targets switch_targets(uint64_t e1, uint64_t e2, bool g) {
    const uint32_t u = ekey_lo_vertex(e1), v = ekey_hi_vertex(e1);
    const uint32_t x = ekey_lo_vertex(e2), y = ekey_hi_vertex(e2);
    // g = 0: (u,x),(v,y)     g = 1: (u,y),(v,x)
    const uint32_t a1 = g ? y : x, b1 = g ? x : y;
    Targets T;
    T.loop = (u == a1) || (v == b1);
    T.A = ekey(u, a1);
    T.B = ekey(v, b1);
    return T;
}

// Graph classes (Sec. 1): bit 1 loops allowed, bit 2 multi-edges allowed,
// bit 4 directed.  Class 0 is the simple undirected graph of Def. 2.1.
enum : uint32_t { CLS_LOOPS = 1u, CLS_MULTI = 2u, CLS_DIRECTED = 4u, CLS_ALL = 7u };

// Targets of a switch in class cls.  Directed edges are stored (tail, head)
// in the key's (high, low) word and the switch exchanges the heads whatever
// g is, which keeps every out- and in-degree.  Undirected edges are stored
// canonically and tau of Def. 2.1 applies.  `loop` asks for rejection as a
// loop: a loop target where loops are not allowed, and, for undirected
// graphs with loops and no multi-edges, a switch with g = 1 that has a loop
// among its sources -- such a switch gives the same targets for both g while
// its reverse move has only one, so only g = 0 runs and the chain stays
// symmetric (Thm. 3.3).
__device__ __forceinline__ Targets switch_targets_cls(uint64_t e1, uint64_t e2, bool g, uint32_t cls) {
    if (cls == 0) return switch_targets(e1, e2, g);
    const uint32_t u = ekey_lo_vertex(e1), v = ekey_hi_vertex(e1);
    const uint32_t x = ekey_lo_vertex(e2), y = ekey_hi_vertex(e2);
    Targets T;
    if (cls & CLS_DIRECTED) {
        T.A = ((uint64_t)u << 32) | y;
        T.B = ((uint64_t)x << 32) | v;
        T.loop = !(cls & CLS_LOOPS) && (u == y || x == v);
    } else {
        const uint32_t a1 = g ? y : x, b1 = g ? x : y;
        T.A = ekey(u, a1);
        T.B = ekey(v, b1);
        T.loop = (cls & CLS_LOOPS) ? (cls == CLS_LOOPS && g && (u == v || x == y)) : (u == a1 || v == b1);
    }
    return T;
}

// Permutation key of record (input position idx) of graph g in batch superstep s.
__device__ __forceinline__ uint64_t batch_perm_key(const BatchGraph &g, uint32_t idx, uint32_t s) {
    if (idx == kPadIdx) return ~0ull;
    return perm_key(idx - g.goff, g.t0 + s, g.k0, g.k1);
}

// Global bucket of permutation key K in graph g: monotone in K (fast range
// reduction of its high word).
__device__ __forceinline__ uint32_t batch_bucket(const BatchGraph &g, uint64_t K) {
    return g.bbase + (uint32_t)(((K >> 32) * (uint64_t)g.nb) >> 32);
}

// ---------------------------------------------------------------------------
// Dependency table (rebuilt every superstep): open addressing, linear probing,
// power-of-two slot count, load <= 1/2.  One 16-byte slot per edge key that is
// a source or a target of the superstep.
//   key     : the edge key, or kEmptyKey
//   eraser  : switch id whose source this edge is (Def. 3.1 / Alg. 1 erase
//             tuple), kNoEraser if the key is not a source, kStays if it is a
//             source that survives the superstep for certain (idle position,
//             or its switch is rejected before any lookup)
//   claim   : (earliest not-yet-excluded inserter << 2) | LEGAL | CONTENDED
//             -- the "smallest non-illegal inserter" lookup of Alg. 1
// ---------------------------------------------------------------------------
struct __align__(16) Slot {
    unsigned long long key;
    uint32_t eraser;
    uint32_t claim;
};

constexpr unsigned long long kEmptyKey = ~0ull;  // a loop at 0xFFFFFFFF: never a valid key
constexpr uint32_t kNoEraser = 0xFFFFFFFFu;
constexpr uint32_t kStays = 0xFFFFFFFEu;
constexpr uint32_t kClaimNone = 0xFFFFFFFCu;  // larger than any (k << 2), flags clear
constexpr uint32_t kClaimContended = 1u;
constexpr uint32_t kClaimLegal = 2u;

__device__ __forceinline__ uint64_t slot_hash(uint64_t x) {
    x ^= x >> 32;
    x *= 0xD6E8FEB86659FD93ull;
    x ^= x >> 32;
    x *= 0xD6E8FEB86659FD93ull;
    x ^= x >> 32;
    return x;
}

// Tuples carry tuple_hash(key) instead of the key: slot_hash is a bijection
// on 64-bit words (xor-shift by 32 is its own inverse, the multiplier is
// odd), so equal hashes mean equal keys, and the partition passes and the
// resolve read digits and cells straight from the word.  The constant makes
// the empty key its own image, so no edge key hashes to it.
constexpr unsigned long long kEmptyHashXor = 0x448E29CED4103459ull ^ ~0ull;  // slot_hash(~0) ^ ~0

__device__ __forceinline__ uint64_t tuple_hash(uint64_t key) { return slot_hash(key) ^ kEmptyHashXor; }

// The key of a tuple hash (error reporting only).
__device__ __forceinline__ uint64_t tuple_key_of(uint64_t h) {
    constexpr unsigned long long kInv = 0xCFEE444D8B59A89Bull;  // inverse of the multiplier mod 2^64
    uint64_t x = h ^ kEmptyHashXor;
    x ^= x >> 32;
    x *= kInv;
    x ^= x >> 32;
    x *= kInv;
    x ^= x >> 32;
    return x;
}

// Finds or inserts `key`; returns its slot.  `nslots` need not be a power of
// two: the home slot is the high word of hash * nslots (multiply-shift range
// reduction).  The table is never more than half full, so the probe ends at
// an empty slot; the probe count is bounded anyway (kNoSlot: table full, an
// internal error).
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t table_home(unsigned long long key, uint32_t nslots) {
    return (uint32_t)__umul64hi(slot_hash(key), (unsigned long long)nslots);
}

__device__ __forceinline__ uint32_t table_find_or_insert(Slot *tab, uint32_t nslots, unsigned long long key) {
    uint32_t s = table_home(key, nslots);
    for (uint32_t probes = 0; probes < nslots; ++probes) {
        const unsigned long long cur = tab[s].key;
        if (cur == key) return s;
        if (cur == kEmptyKey) {
            const unsigned long long prev = atomicCAS(&tab[s].key, kEmptyKey, key);
            if (prev == kEmptyKey || prev == key) return s;
        }
        s = (s + 1 == nslots) ? 0 : s + 1;
    }
    return kNoSlot;
}

// Error bits raised by kernels (read back by the host at the end of a call).
enum : uint32_t {
    ERR_LOOP = 1u,       // input contains a loop
    ERR_RANGE = 2u,      // vertex id >= n (or 0xFFFFFFFF)
    ERR_DUP = 4u,        // input contains a duplicate edge
    ERR_INTERNAL = 8u,   // an internal consistency check failed
    ERR_ROUNDS = 16u,    // a superstep needed more decision rounds than the caller's limit
};

// Per-superstep statistics kept on the device.
struct StepCounters {
    unsigned long long legal, rej_loop, rej_exists, rej_pl;
    unsigned long long rounds, undecided_round1, fallback_buckets, pad;
};

}  // namespace gesmc

// Tuple tags and the packed 8-byte tuple word of the dependency partitions
// (host and device: the host test of the packing includes this file).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gesmc {

// Dependency tuples (tag, edge key): an ERASE tuple carries the switch that
// erases its key (or kTagStays for an edge that survives the superstep), an
// INSERT tuple kTagInsert | (k << 1 | h) for target h of switch k.
constexpr uint32_t kTagInsert = 0x80000000u;
constexpr uint32_t kTagStays = 0x7FFFFFFEu;

// Packed tuples: one 8-byte word per tuple when the bits allow it.  An edge
// key (u, v), u < v, with u below 2^vb and v - u below 2^db is coded on
// w = vb + db bits as (u << db) | (v - u): one graph has db = vb, and in a
// batch, whose graphs' vertex ranges are disjoint, db covers the largest
// graph while vb covers them all.  mix_w is a bijection on w-bit words
// (xor-shift by at least w/2 is its own inverse, odd multipliers are
// invertible mod 2^w), so equal hashes still mean equal keys; one multiply
// between two xor-shifts spreads the keys over partitions and cells as
// evenly as two (measured on the benchmark graphs and structured sets).  A tag is coded
// on tb = kb + 1 bits in the order of the 32-bit tags: ERASE k -> k,
// STAYS -> 2^kb - 1, INSERT (k, h) -> 2^kb | 2k+h (2 ell < 2^kb).  The first
// partition pass writes (H << (64 - w + b1)) | code: the b1 hash bits it
// partitioned by are implied by the partition and dropped, the rest stays on
// top for the second level's digits and the resolve's cells.  In a batch too
// large for batch-wide switch ids in the code, tags are local to the
// tuple's graph (switch k - poff / 2 of its graph): all tuples of one key
// belong to one graph, so their order is the same, and kb then covers only
// the largest graph.
struct TuplePack {
    int w;      // hash bits vb + db (0: 12-byte tuples)
    int db;     // bits of the larger endpoint's offset v - u
    int kb;     // tag code bits below the INSERT flag
    int b1;     // hash bits dropped by the first partition pass
    int b2;     // hash bits of the second partition pass
    int local;  // tags local to the tuple's graph (batches)
};

__host__ __device__ __forceinline__ uint64_t low_mask(int w) { return w >= 64 ? ~0ull : ((1ull << w) - 1); }

constexpr unsigned long long kMixMul1 = 0xD6E8FEB86659FD93ull, kMixMul2 = 0x9E3779B97F4A7C15ull;
constexpr unsigned long long inverse_mod_2_64(unsigned long long a) {  // Newton: x <- x (2 - a x)
    unsigned long long x = a;
    for (int i = 0; i < 6; ++i) x *= 2ull - a * x;
    return x;
}

#ifndef GESMC_MIX_ROUNDS
#define GESMC_MIX_ROUNDS 1  // multiply rounds of mix_w (1 or 2)
#endif

__host__ __device__ __forceinline__ uint64_t mix_w(uint64_t x, int w) {
    const uint64_t mask = low_mask(w);
    const int s = (w + 1) >> 1;
    x ^= x >> s;
    x = (x * kMixMul1) & mask;
    x ^= x >> s;
    if (GESMC_MIX_ROUNDS > 1) {
        x = (x * kMixMul2) & mask;
        x ^= x >> s;
    }
    return x;
}

__host__ __device__ __forceinline__ uint64_t unmix_w(uint64_t x, int w) {
    constexpr unsigned long long kInv1 = inverse_mod_2_64(kMixMul1), kInv2 = inverse_mod_2_64(kMixMul2);
    const uint64_t mask = low_mask(w);
    const int s = (w + 1) >> 1;
    x ^= x >> s;
    if (GESMC_MIX_ROUNDS > 1) {
        x = (x * kInv2) & mask;
        x ^= x >> s;
    }
    x = (x * kInv1) & mask;
    x ^= x >> s;
    return x;
}

// The w-bit hash of a canonical edge key (u << 32) | v.
__host__ __device__ __forceinline__ uint64_t key_hash_w(uint64_t key, int db, int w) {
    const uint32_t u = (uint32_t)(key >> 32), v = (uint32_t)key;  // u < v
    return mix_w(((uint64_t)u << db) | (uint32_t)(v - u), w);
}

// The smaller endpoint of the key with w-bit hash h (error reporting only).
__host__ __device__ __forceinline__ uint32_t key_hash_w_vertex(uint64_t h, int db, int w) {
    return (uint32_t)(unmix_w(h, w) >> db);
}

__host__ __device__ __forceinline__ uint32_t tag_code(uint32_t tag, int kb) {
    if (tag & kTagInsert) return (1u << kb) | (tag & ~kTagInsert);
    return tag == kTagStays ? (1u << kb) - 1u : tag;
}

__host__ __device__ __forceinline__ uint32_t tag_of_code(uint32_t code, int kb) {
    if (code >> kb) return kTagInsert | (code & ((1u << kb) - 1u));
    return code == (1u << kb) - 1u ? kTagStays : code;
}

// A tag moved by kbase switches (kbase = the first switch of the tuple's
// graph): to_local subtracts it, to_global adds it back.  STAYS is unchanged.
__host__ __device__ __forceinline__ uint32_t tag_shift(uint32_t tag, uint32_t kbase, bool to_local) {
    if (tag == kTagStays) return tag;
    const uint32_t d = (tag & kTagInsert) ? 2u * kbase : kbase;
    return to_local ? tag - d : tag + d;
}

}  // namespace gesmc

// libgesmc: host runtime and C ABI for the G-ES-MC global switch on gfx950.
// The declarations and their meaning are in include/gesmc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "gesmc.h"
#include "perm_kernels.h"
#include "switch_kernels.h"
#include "resolve_kernels.h"
#include "batch_kernels.h"
#include "es_kernels.h"
#include "mixing_kernels.h"
#include "gen_kernels.h"

using namespace gesmc;

// Device memory of gesmc_run_noalloc: one fixed array per device, held for
// the whole process.  In host code its name is a host-side stand-in: host
// code uses only the device address that hipGetSymbolAddress returns for it
// (noalloc_scratch_ptr), never the name itself.
static __device__ __align__(256) unsigned char scratch[(size_t)GESMC_NOALLOC_SCRATCH_MIB << 20];

namespace {

thread_local char g_last_error[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
}

// Set on the calling thread for the duration of gesmc_run_noalloc: every
// path that would allocate or free device or pinned memory fails instead.
thread_local bool t_no_alloc = false;

bool alloc_forbidden() {
    if (!t_no_alloc) return false;
    set_error("internal: gesmc_run_noalloc reached an allocation");
    return true;
}

// Supersteps per piece of the small-graph path, and the bytes of its
// permutation rows (one row of kCmpMax 16-bit entries per superstep).
constexpr uint32_t kSmallPiSteps = 32;
constexpr size_t kSmallPiBytes = (size_t)kSmallPiSteps * kCmpMax * sizeof(uint16_t);

enum KernelId {
    KID_LOAD,
    KID_STEP_CLEAR,
    KID_COUNTS1,
    KID_SCATTER1,
    KID_COUNTS2,
    KID_SCAN,
    KID_SCATTER2,
    KID_SORT,
    KID_BUILD,
    KID_DECIDE1,
    KID_ROUND_RESET,
    KID_ROUND_CLAIM,
    KID_ROUND_DECIDE,
    KID_FINISH,
    KID_UNPERMUTE,
    KID_VALIDATE,
    KID_MISC,
    KID_EMIT,
    KID_TCOUNTS1,
    KID_TSCATTER1,
    KID_TCOUNTS2,
    KID_TSCATTER2,
    KID_RESOLVE,
    KID_DECIDE_CHAIN1,
    KID_DECIDE_CHAIN,
    KID_FINISH_CHAIN,
    KID_SMALL,
    KID_SMALL_MID,
    KID_SMALL_CMP,
    KID_ES_BUILD,
    KID_ES_CHAIN,
    KID_MIX,
    KID_DECIDE_LOCAL,
    KID_GEN,
    KID_GEN_HH_STEPS,
    KID_SMALL_PERM,
    KID_COUNT
};

const char *kKernelNames[KID_COUNT] = {
    "k_load",         "k_step_clear",   "k_counts1",    "k_scatter1",      "k_counts2",     "k_scan",
    "k_scatter2",     "k_sort_buckets", "k_build",      "k_decide_first",  "k_round_reset", "k_round_claim",
    "k_round_decide", "k_finish",       "k_unpermute",  "k_validate",      "k_misc",
    "k_emit",         "k_tcounts1",     "k_tscatter1",  "k_tcounts2",      "k_tscatter2",   "k_resolve",
    "k_decide_chain1", "k_decide_chain", "k_finish_chain", "k_small_chain", "k_small_chain_4096",
    "k_small_chain_compact",
    "k_es_build",     "k_es_chain",     "k_mixing",     "k_decide_local", "k_gen",
    "k_hh_steps",     "k_small_perm"};

__global__ void k_setup_level1(uint32_t *seg_off, uint32_t *tile_first, uint32_t m, uint32_t ntiles) {
    if (threadIdx.x == 0) {
        seg_off[0] = 0;
        seg_off[1] = m;
        tile_first[0] = 0;
        tile_first[1] = ntiles;
    }
}

__global__ void k_zero_words(uint32_t *p, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) p[q] = 0;
}

__global__ void k_identity_records(uint32_t *idx, unsigned long long *key, uint32_t m) {
    const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < m) {
        idx[r] = (uint32_t)r;
        key[r] = r;
    }
}

__global__ void k_copy_bytes(const uint8_t *src, uint8_t *dst, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) dst[q] = src[q];
}

inline uint32_t ceil_div(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

}  // namespace

// A buffer from the caller's allocator and the free function that returns it.
struct HookedBuffer {
    gesmc_free_fn free_fn;
    void *user;
};

struct gesmc_ctx {
    int device = 0;
    int num_cus = 256;
    // options
    uint32_t bucket_avg = 3 * kLdsCap / 4;  // partition means fall in (avg / 2, avg]
    uint32_t sort_cap = kLdsCap;
    int fast_rounds = 2;
    // GESMC_OPT_FAST_ROUNDS never set: a plain call runs adapt_rounds
    // multi-workgroup rounds, taken from the previous plain call's rounds
    bool fast_rounds_auto = true;
    int adapt_rounds = 2;
    uint32_t round_limit = 0;  // decision rounds per superstep before GESMC_E_ROUNDS (0: none)
    int persist_mult = 0;  // persistent grids: resident workgroups x this (0: one workgroup per unit)
    uint32_t level1_cap = 0;  // first-level digit bits (0: even split)
    bool fuse_emit = true;    // tuples computed in the first partition pass (else stored flat)
    // hipGraph capture of batched calls (GESMC_OPT_GRAPH)
    bool use_graph = false, capturing = false;
    uint64_t graph_key = 0, graph_last_key = 0, graph_replays = 0;
    hipGraphExec_t graph_exec = nullptr;
    int strategy = 0;  // 0: tuples partitioned by key and resolved in LDS; 1: HBM table
    bool profile = false;
    int profile_only = -1;  // kernel id timed while profiling (-1: every kernel)
    // device buffers (capacity in edges)
    uint64_t cap_m = 0;
    uint32_t *idx[3] = {nullptr, nullptr, nullptr};
    unsigned long long *key[3] = {nullptr, nullptr, nullptr};
    Slot *tab = nullptr;
    uint64_t tab_slots = 0;
    uint32_t *sw_slot = nullptr;
    uint8_t *st = nullptr;
    uint32_t *ulist[2] = {nullptr, nullptr};
    // dependency tuples: flat (per switch), and two partitioned buffers
    uint64_t cap_tu = 0;
    uint32_t *tu_tag[3] = {nullptr, nullptr, nullptr};
    unsigned long long *tu_key[3] = {nullptr, nullptr, nullptr};
    uint2 *info = nullptr;
    // radix bookkeeping: per-tile digit counts / run bases of both levels, chunk sums
    uint64_t cap_counts1 = 0, cap_counts2 = 0, cap_partial = 0;
    uint32_t *counts1 = nullptr, *counts2 = nullptr, *partial = nullptr;
    uint32_t *small = nullptr;  // counters, histograms, offsets (fixed size)
    uint16_t *small_pi = nullptr;  // permutations of the small-graph path (kSmallPiSteps rows of kCmpMax)
    std::string device_key;        // architecture and PCI address (the tuning cache's device)
    bool tune_cache = true;        // the autotuner reuses and keeps choices per device and shape class
    uint4 *bslot = nullptr;     // per-block counts of the grid-stride kernels (2 grids)
    // batches: per graph (rank order) and per position
    uint64_t cap_g = 0, cap_pos = 0;
    BatchGraph *gr = nullptr;
    uint64_t *in_off = nullptr;
    uint32_t *rank_of = nullptr;
    unsigned long long *gacc = nullptr;
    unsigned long long *h_gacc = nullptr;
    uint32_t *gerr = nullptr, *h_gerr = nullptr;
    uint32_t *pg = nullptr, *bk = nullptr;
    std::vector<BatchGraph> h_gr;
    std::vector<uint32_t> h_rank_of, h_order, h_small, h_mid, h_cmp, h_rrank;
    std::vector<uint4> h_chunks;   // position chunks of the ranks' segments (k_fill_pg, serving kernels)
    uint64_t *hr_dev = nullptr, *h_hr = nullptr;  // gesmc_run_host: device in/out (2 x cap), pinned staging
    uint64_t hr_cap = 0, h_hr_cap = 0;              // words
    unsigned char *h_up = nullptr;  // pinned staging of a call's small uploads (up_begin / up_copy)
    uint64_t up_cap = 0, up_used = 0;
    hipEvent_t up_ev = nullptr;     // recorded after a call's last upload
    bool up_pending = false;
    uint4 *chunks = nullptr;
    uint64_t chunk_cap = 0;
    uint32_t *small_list = nullptr, *rrank = nullptr;  // small graphs' ranks; r per rank
    bool small_graphs = true;                         // graphs with m <= kSmallMax run in LDS
    bool unpermute_buckets = true;                    // large write-backs by index buckets
    gesmc_alloc_fn alloc_fn = nullptr;                // the caller's allocator (gesmc_set_allocator)
    gesmc_free_fn free_fn = nullptr;
    void *alloc_user = nullptr;
    std::unordered_map<void *, HookedBuffer> hooked;  // live buffers of caller allocators
    bool serving = false;                             // a gesmc_server owns the context
    int pack_tuples = 1;  // 8-byte tuple words where the bits allow (2: batches always with graph-local tags)
    uint32_t tuple_bytes = 0;                         // tuple size of the call's last superstep
    StepCounters *ctr = nullptr;
    StepCounters *ctr_step = nullptr;  // counters of the superstep being enqueued
    uint64_t ctr_cap = 0;
    // views into `small`
    uint32_t *err = nullptr, *ucount = nullptr, *coarse_off = nullptr, *tile_first = nullptr,
             *lvl1_seg = nullptr, *lvl1_tiles = nullptr, *fine_off = nullptr;
    // host staging (pinned)
    uint32_t *h_err = nullptr;
    StepCounters *h_ctr = nullptr;
    uint64_t h_ctr_cap = 0;
    // profiling
    struct Rec {
        int kid;
        uint64_t items;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<Rec> recs;
    double prof_ms[KID_COUNT] = {0};
    uint64_t prof_launch[KID_COUNT] = {0};
    uint64_t prof_items[KID_COUNT] = {0};
    hipEvent_t call_a = nullptr, call_b = nullptr;
    // ParES (gesmc_run_es): edge list, slot of each edge, edge set, counters
    unsigned long long *es_E = nullptr, *es_H = nullptr;
    uint32_t *es_slot = nullptr;
    uint64_t es_cap_m = 0, es_cap_T = 0;
    EsCounters *es_ctr = nullptr, *h_es_ctr = nullptr;
    // side streams of the batch's LDS small-graph kernels (default priority),
    // forked from and joined back into the call's stream with these events
    hipStream_t side[2] = {nullptr, nullptr};
    hipEvent_t fork_ev = nullptr, join_ev[2] = {nullptr, nullptr};
};

namespace {

// Bucket bits of a radix pass: 21 keeps the mean tuple partition within the
// LDS capacity up to the largest input (2^31 tuple slots at m < 2^30).
constexpr uint32_t kMaxFineBits = 21;
constexpr uint32_t kMaxLevelBits = 12;  // digit bits of one radix level (first <= kMaxCoarseBits)
constexpr uint64_t kMaxEdges = 1ull << 30;

void dev_free(gesmc_ctx *c, void *p);

void free_buffers(gesmc_ctx *c) {
    for (int q = 0; q < 3; ++q) {
        if (c->idx[q]) dev_free(c, c->idx[q]);
        if (c->key[q]) dev_free(c, c->key[q]);
        c->idx[q] = nullptr;
        c->key[q] = nullptr;
    }
    if (c->tab) dev_free(c, c->tab);
    if (c->sw_slot) dev_free(c, c->sw_slot);
    if (c->st) dev_free(c, c->st);
    for (int q = 0; q < 2; ++q) {
        if (c->ulist[q]) dev_free(c, c->ulist[q]);
        c->ulist[q] = nullptr;
    }
    for (int q = 0; q < 3; ++q) {
        if (c->tu_tag[q]) dev_free(c, c->tu_tag[q]);
        if (c->tu_key[q]) dev_free(c, c->tu_key[q]);
        c->tu_tag[q] = nullptr;
        c->tu_key[q] = nullptr;
    }
    if (c->info) dev_free(c, c->info);
    c->info = nullptr;
    for (uint32_t **pp : {&c->counts1, &c->counts2, &c->partial}) {
        if (*pp) dev_free(c, *pp);
        *pp = nullptr;
    }
    c->cap_counts1 = c->cap_counts2 = c->cap_partial = 0;
    c->cap_tu = 0;
    c->tab = nullptr;
    c->sw_slot = nullptr;
    c->st = nullptr;
    c->cap_m = 0;
    c->tab_slots = 0;
}

// Bumped by every device allocation: a captured graph holds buffer addresses,
// so it is only replayed while no buffer has moved.
std::atomic<uint64_t> g_alloc_epoch{0};

// Device memory of a context: from the caller's allocator once one is set
// (gesmc_set_allocator), else hipMalloc.  Each buffer remembers the free
// function of the allocator that made it, so buffers from before and after a
// change are each returned to their own allocator.
gesmc_status dev_alloc(gesmc_ctx *c, void **p, size_t bytes) {
    if (alloc_forbidden()) return GESMC_E_INTERNAL;
    ++g_alloc_epoch;
    const size_t b = bytes ? bytes : 16;
    if (c && c->alloc_fn) {
        void *q = c->alloc_fn(b, c->alloc_user);
        *p = q;
        if (!q || ((uintptr_t)q & 255u)) {
            if (q) c->free_fn(q, c->alloc_user);
            *p = nullptr;
            set_error(q ? "the caller's allocator returned memory aligned below 256 bytes"
                        : "the caller's allocator returned no memory for %zu bytes",
                      b);
            return GESMC_E_NOMEM;
        }
        c->hooked[q] = HookedBuffer{c->free_fn, c->alloc_user};
        return GESMC_OK;
    }
    if (hipMalloc(p, b) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        set_error("hipMalloc of %zu bytes failed", bytes);
        return GESMC_E_NOMEM;
    }
    return GESMC_OK;
}

// Returns a device buffer to the allocator that made it.  The caller's free
// function runs only once the device has finished all queued work, since it
// may hand the memory to other work at once; hipFree waits by itself.
void dev_free(gesmc_ctx *c, void *p) {
    if (!p) return;
    if (c) {
        const auto it = c->hooked.find(p);
        if (it != c->hooked.end()) {
            const HookedBuffer h = it->second;
            c->hooked.erase(it);
            (void)hipDeviceSynchronize();
            h.free_fn(p, h.user);
            return;
        }
    }
    (void)hipFree(p);
}

uint64_t table_slots_for(uint64_t m) {
    // keys per superstep <= m sources + 2 * floor(m/2) targets <= 2m; load <= 1/2
    // (slot count a multiple of 8: whole 128-byte lines)
    return std::max<uint64_t>(1024, (4 * m + 7) / 8 * 8);
}

gesmc_status ensure_capacity(gesmc_ctx *c, uint64_t m, bool tuples = false) {
    const bool need_tab = c->strategy == 1;
    const bool need_tu = c->strategy == 0 || tuples;
    if (m <= c->cap_m && (!need_tab || c->tab) && (!need_tu || c->info)) return GESMC_OK;
    if (alloc_forbidden()) return GESMC_E_INTERNAL;
    free_buffers(c);
    const uint64_t cap = std::max<uint64_t>(m, 1024);
    gesmc_status s = GESMC_OK;
    for (int q = 0; q < 3 && s == GESMC_OK; ++q) {
        s = dev_alloc(c, (void **)&c->idx[q], cap * 4);
        if (s == GESMC_OK) s = dev_alloc(c, (void **)&c->key[q], cap * 8);
    }
    const uint64_t ts = need_tab ? table_slots_for(cap) : 0;
    if (s == GESMC_OK && need_tab) s = dev_alloc(c, (void **)&c->tab, ts * sizeof(Slot));
    const uint64_t ntu = 2 * cap + 8;  // 4 * floor(m/2) + 1 tuple slots
    for (int q = 0; q < 3 && s == GESMC_OK && need_tu; ++q) {
        s = dev_alloc(c, (void **)&c->tu_tag[q], ntu * 4);
        if (s == GESMC_OK) s = dev_alloc(c, (void **)&c->tu_key[q], ntu * 8);
    }
    if (s == GESMC_OK && need_tu) s = dev_alloc(c, (void **)&c->info, (cap + 8) * sizeof(uint2));
    if (s == GESMC_OK) c->cap_tu = need_tu ? ntu : 0;
    if (s == GESMC_OK) s = dev_alloc(c, (void **)&c->sw_slot, (cap / 2 + 1) * 8);
    if (s == GESMC_OK) s = dev_alloc(c, (void **)&c->st, cap / 2 + 64);
    for (int q = 0; q < 2 && s == GESMC_OK; ++q) s = dev_alloc(c, (void **)&c->ulist[q], (cap / 2 + 64) * 4);
    if (s != GESMC_OK) {
        free_buffers(c);
        return s;
    }
    c->cap_m = cap;
    c->tab_slots = ts;
    return GESMC_OK;
}

gesmc_status ensure_counters(gesmc_ctx *c, uint64_t r) {
    const uint64_t want = std::max<uint64_t>(r, 1);
    if ((want > c->ctr_cap || want > c->h_ctr_cap) && alloc_forbidden()) return GESMC_E_INTERNAL;
    if (want > c->ctr_cap) {
        if (c->ctr) dev_free(c, c->ctr);
        c->ctr = nullptr;
        c->ctr_cap = 0;
        gesmc_status s = dev_alloc(c, (void **)&c->ctr, want * sizeof(StepCounters));
        if (s != GESMC_OK) return s;
        c->ctr_cap = want;
    }
    if (want > c->h_ctr_cap) {
        if (c->h_ctr) (void)hipHostFree(c->h_ctr);
        c->h_ctr = nullptr;
        c->h_ctr_cap = 0;
        if (hipHostMalloc((void **)&c->h_ctr, want * sizeof(StepCounters), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipHostMalloc failed");
            return GESMC_E_NOMEM;
        }
        c->h_ctr_cap = want;
    }
    return GESMC_OK;
}

// ---- launch helper with optional per-launch event timing -------------------
hipEvent_t take_event(gesmc_ctx *c) {
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_used++];
}

template <typename Kern, typename... Args>
gesmc_status launch(gesmc_ctx *c, hipStream_t s, int kid, uint64_t items, Kern kern, dim3 grid, dim3 block,
                    size_t lds, Args... args) {
    hipEvent_t a = nullptr, b = nullptr;
    if (c->profile && !c->capturing && (c->profile_only < 0 || c->profile_only == kid)) {
        a = take_event(c);
        b = take_event(c);
        if (a) (void)hipEventRecord(a, s);
    }
    hipLaunchKernelGGL(kern, grid, block, lds, s, args...);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("launch of %s failed: %s", kKernelNames[kid], hipGetErrorString(e));
        return GESMC_E_DEVICE;
    }
    if (a && b) {
        (void)hipEventRecord(b, s);
        c->recs.push_back({kid, items, a, b});
    }
    return GESMC_OK;
}

#define GESMC_TRY(x)                      \
    do {                                  \
        gesmc_status _s = (x);            \
        if (_s != GESMC_OK) return _s;    \
    } while (0)

struct Plan {
    uint32_t m, ell, bbits, b1, b2, ncoarse, nfine, ntiles1, tile;
    uint32_t dig_in_key = 0;  // the permutation's scatters stage digits in the keys' top byte (SrcArgs)
    uint32_t tile2 = 0;       // second-level tile records (0: tile)
};

// Digits in the keys' top byte (SrcArgs::dig_in_key) when every vertex id is
// below 2^24 and both levels have at most 8 digit bits; 0 disables it.
#ifndef GESMC_DIGIT_IN_KEY
#define GESMC_DIGIT_IN_KEY 1
#endif
// Level-1 counts of the next superstep taken in the first decision round
// (k_decide_chain's NextCounts); 0 disables it.
#ifndef GESMC_COUNT_AHEAD
#define GESMC_COUNT_AHEAD 1
#endif

uint32_t digit_in_key(const Plan &p, uint32_t n) {
    return GESMC_DIGIT_IN_KEY && n <= (1u << 24) && p.b1 <= 8 && p.b2 <= 8 ? 1u : 0u;
}

uint32_t tile_for(uint32_t n) { return n >= kLargeTileRecords ? (uint32_t)kTileLarge : (uint32_t)kTileSmall; }

// Tiles per chunk of the level-1 column scan: a power of two in [8, 256]
// giving about 192 chunks.
#ifndef GESMC_SCAN_ROWS
#define GESMC_SCAN_ROWS 192
#endif
uint32_t scan_chunk(uint32_t ntiles) {
    uint32_t ch = 8;
    while (ch < 256 && ceil_div(ntiles, ch) > GESMC_SCAN_ROWS) ch <<= 1;
    return ch;
}

// Digit bits of the first level: an even split of B (so both levels write
// runs of similar length; from 17 bits on, an odd B gives the first level
// the smaller half, whose scatter then writes longer runs per digit, unless
// `ceil_half`: batch permutations, whose first level stages more per record,
// keep the larger half), or at most `cap` bits if the option sets one.
uint32_t level1_bits(uint32_t B, uint32_t cap, bool ceil_half = false) {
    if (cap == 0) return std::min<uint32_t>(kMaxCoarseBits, B >= 17 && !ceil_half ? B / 2 : (B + 1) / 2);
    // the second level keeps at most kMaxLevelBits (its LDS counters)
    return std::min<uint32_t>(B, std::max<uint32_t>(cap, B > kMaxLevelBits ? B - kMaxLevelBits : 0));
}

// Plan of a batch permutation: global buckets [0, nb) over m records.  The
// second level runs on 2048-record tiles at every size (its scatter stages
// 14 bytes per record: smaller workgroups, more of them per CU), the first
// on the size's usual tile; 0: both levels on the usual tile.
#ifndef GESMC_BATCH_LEVEL2_SMALL_TILES
#define GESMC_BATCH_LEVEL2_SMALL_TILES 1
#endif
Plan batch_plan(const gesmc_ctx *c, uint32_t m, uint64_t nb) {
    Plan p;
    p.m = m;
    p.ell = m / 2;
    uint32_t B = 0;
    while ((1ull << B) < nb) ++B;
    p.bbits = B;
    p.b1 = level1_bits(B, c->level1_cap, true);
    p.b2 = B - p.b1;
    p.ncoarse = 1u << p.b1;
    p.nfine = 1u << B;
    p.tile = tile_for(m);
    p.tile2 = GESMC_BATCH_LEVEL2_SMALL_TILES ? (uint32_t)kTileSmall : 0u;
    p.ntiles1 = std::max<uint32_t>(1, ceil_div(m, p.tile));
    return p;
}

// Radix plan for n records: B bucket bits (mean bucket <= bucket_avg), split
// into a coarse level (level1_bits) and a second level of the rest.
Plan make_plan(const gesmc_ctx *c, uint32_t m) {
    Plan p;
    p.m = m;
    p.ell = m / 2;
    uint32_t B = 0;
    while (B < kMaxFineBits && ((uint64_t)c->bucket_avg << B) < m) ++B;
    p.bbits = B;
    p.b1 = level1_bits(B, c->level1_cap);
    p.b2 = B - p.b1;
    p.ncoarse = 1u << p.b1;
    p.nfine = 1u << B;
    p.tile = tile_for(m);
    p.ntiles1 = std::max<uint32_t>(1, ceil_div(m, p.tile));
    return p;
}

// LDS of k_scatter: counters, staged indices (none for packed tuple
// words), keys and digits, and (batch level 1 only) staged global buckets.
// It bounds the workgroups per CU.
size_t scatter_lds_bytes(int dbits, uint32_t tile, bool buckets = true, bool idx = true, bool digits = true) {
    const size_t nd = (size_t)1 << dbits;
    size_t words = 3 * nd + scatter_threads((int)tile) / 64 + 1 + (idx ? tile : 0);
    words += words & 1;  // 8-byte alignment of the key stage
    return words * 4 + (size_t)tile * 8 + (digits ? (size_t)tile * 2 : 0) + (buckets ? (size_t)tile * 4 : 0);
}

// Every k_scatter instance may take more than 64 KiB of dynamic LDS (gfx950
// has 160 KiB per CU); a level has at most kMaxLevelBits digit bits.
template <int kTile, bool kOne>
void set_scatter_lds_limits_one() {
    for (const void *f : {(const void *)k_scatter<kSrcPerm, kTile, scatter_threads(kTile), kOne>,
                          (const void *)k_scatter<kSrcHash, kTile, scatter_threads(kTile), kOne>,
                          (const void *)k_scatter<kSrcBatch, kTile, scatter_threads(kTile), kOne>,
                          (const void *)k_scatter<kSrcBucket, kTile, scatter_threads(kTile), kOne>,
                          (const void *)k_scatter<kSrcEmit, kTile, scatter_threads(kTile), kOne>,
                          (const void *)k_scatter<kSrcHashed, kTile, scatter_threads(kTile), kOne>,
                          (const void *)k_scatter<kSrcEmitPacked, kTile, scatter_threads(kTile), kOne>,
                          (const void *)k_scatter<kSrcEmitPackedLocal, kTile, scatter_threads(kTile), kOne>,
                          (const void *)k_scatter<kSrcPacked, kTile, scatter_threads(kTile), kOne>,
                          (const void *)k_scatter<kSrcIdx, kTile, scatter_threads(kTile), kOne>})
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)scatter_lds_bytes(kMaxLevelBits, kTile));
}

template <int kTile>
void set_scatter_lds_limits() {
    set_scatter_lds_limits_one<kTile, true>();
    set_scatter_lds_limits_one<kTile, false>();
}

size_t sort_lds_bytes(uint32_t cap) {
    return ((size_t)(1u << kCellBits) + kBlock + 2) * 4 + (size_t)cap * 20;
}

// cells, scan words, keys, tags, list links; packed words with the cell
// lists keep their tags in the words
size_t resolve_lds_bytes(uint32_t cap, bool packed = false) {
    return ((size_t)(1u << kCellBits) + kBlock + 2) * 4 + (size_t)cap * (packed && GESMC_RESOLVE_LISTS ? 10 : 14);
}

// Workgroups of a persistent kernel: as many as can be resident at once
// (occupancy query for its LDS size), never more than the work units.
template <typename Kern>
uint32_t persistent_blocks(const gesmc_ctx *c, Kern kern, size_t lds, uint64_t units, int threads = kBlock) {
    if (c->persist_mult == 0) return (uint32_t)std::max<uint64_t>(1, units);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds) != hipSuccess || per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    const uint64_t want = (uint64_t)per_cu * c->num_cus * c->persist_mult;
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, units));
}

uint32_t grid_stride_blocks(const gesmc_ctx *c, uint64_t work) {
    const uint64_t want = (work + kBlock - 1) / kBlock;
    const uint64_t cap = (uint64_t)c->num_cus * 8;
    return (uint32_t)std::max<uint64_t>(1, std::min(want, cap));
}

// Grows a word buffer of the radix bookkeeping.
gesmc_status ensure_words(gesmc_ctx *c, uint32_t **p, uint64_t *cap, uint64_t want) {
    if (want <= *cap && *p) return GESMC_OK;
    if (alloc_forbidden()) return GESMC_E_INTERNAL;
    if (*p) dev_free(c, *p);
    *p = nullptr;
    *cap = 0;
    GESMC_TRY(dev_alloc(c, (void **)p, std::max<uint64_t>(want, 1024) * 4));
    *cap = std::max<uint64_t>(want, 1024);
    return GESMC_OK;
}

// Words of the radix bookkeeping of one two-level distribution with plan p:
// per-tile digit counts of both levels and the level-1 chunk sums.
struct RadixWords {
    uint64_t counts1, partial, counts2;
};

// An upper bound of the second level's tiles, less the coarse segment count
// (a segment's last tile may be partial).
uint64_t level2_tiles(const Plan &p) {
    const uint32_t t2 = p.tile2 ? p.tile2 : p.tile;
    return std::max<uint64_t>(1, ceil_div((uint64_t)p.m, t2));
}

RadixWords radix_words(const Plan &p) {
    const uint64_t nd1 = 1ull << p.b1, nd2 = 1ull << p.b2;
    const uint64_t nchunks = ceil_div(p.ntiles1, scan_chunk(p.ntiles1));
    return RadixWords{(uint64_t)p.ntiles1 * nd1, nchunks * nd1,
                      p.b2 > 0 ? ((uint64_t)level2_tiles(p) + p.ncoarse) * nd2 : 0};
}

// 1: with fused tuple passes, the emit runs inside the first tuple count pass
#ifndef GESMC_FUSE_EMIT_COUNTS
#define GESMC_FUSE_EMIT_COUNTS 1
#endif

// The emit's per-switch outputs, written by the first tuple count pass
// (k_emit_counts) when the tuples are computed from the pair records; its
// `grid` workgroups store their outcome counts in bslot[0, grid).
struct EmitOut {
    uint2 *info;
    uint8_t *st;
    uint32_t *out_idx;
    unsigned long long *out_key;
    uint4 *bslot;
    uint32_t *ucount;
    uint32_t grid;
};
constexpr uint32_t kEmitSlotsMax = 8192;  // workgroups of k_emit_counts (count slots)

// Two-level MSD radix distribution of the n records (idx/tag, key) in buffer
// set `src` into `dst` (one level) or via `mid` into `dst` (two levels), by
// the radix word of source kSrc1 (level 1) and kSrc2 (level 2), with the
// batch arguments ba1 / ba2 of those levels.  Leaves c->coarse_off /
// c->fine_off as the bucket boundaries; returns the buffer index holding the
// result in *out.
template <int kSrc1, int kSrc2, int kTile, int kTile2>
gesmc_status radix_distribute_t(gesmc_ctx *c, hipStream_t s, const Plan &p, uint32_t n, uint32_t t, uint32_t k0,
                              uint32_t k1, uint32_t *const *idx, unsigned long long *const *key, int src, int mid,
                              int dst, int *out, const uint32_t **bucket_off, uint32_t *nbuckets, int kid_counts1,
                              int kid_scatter1, int kid_counts2, int kid_scatter2, SrcArgs ba1, SrcArgs ba2,
                              const uint32_t *in_idx, const unsigned long long *in_key, const EmitOut *eo,
                              bool counts1_ready) {
    // level-1 input: buffer `src`, or the given arrays (the pair records of kSrcEmit)
    const uint32_t *src_i = in_idx ? in_idx : idx[src];
    const unsigned long long *src_k = in_key ? in_key : key[src];
    const uint32_t nd1 = 1u << p.b1;
    const uint32_t chunk = scan_chunk(p.ntiles1);
    const uint32_t nchunks = ceil_div(p.ntiles1, chunk);
    const uint32_t scan_threads = std::max<uint32_t>(64, std::min<uint32_t>(kBlock, nd1));
    const RadixWords rw = radix_words(p);
    GESMC_TRY(ensure_words(c, &c->counts1, &c->cap_counts1, rw.counts1));
    GESMC_TRY(ensure_words(c, &c->partial, &c->cap_partial, rw.partial));
    const int shift1 = p.b1 > 0 ? 64 - (int)p.b1 : 63;  // level 1: one segment [0, n), passed by value
    bool fused_emit = false;
    if constexpr (kSrc1 == kSrcEmit || src_emits_packed<kSrc1>()) {
        if (eo) {  // the emit's outputs in the same pass
            GESMC_TRY(launch(c, s, kid_counts1, n, k_emit_counts<kSrc1, kTile>, dim3(eo->grid), dim3(kBlock),
                             (size_t)nd1 * 4, src_i, src_k, t, k0, k1, shift1, (int)p.b1, n, c->counts1, ba1,
                             eo->info, eo->st, eo->out_idx, eo->out_key, eo->bslot, eo->ucount));
            fused_emit = true;
        }
    }
    if (eo && !fused_emit) {
        set_error("internal: emit outputs need a tuple source computed from the pair records");
        return GESMC_E_INTERNAL;
    }
    if (!fused_emit && !counts1_ready)  // (ready: counted by the previous superstep's first decision round)
        GESMC_TRY(launch(c, s, kid_counts1, n, k_tile_counts<kSrc1, kTile, true>,
                         dim3(persistent_blocks(c, k_tile_counts<kSrc1, kTile, true>, (size_t)nd1 * 4, p.ntiles1)),
                         dim3(kBlock), (size_t)nd1 * 4, src_i, src_k, t, k0, k1, shift1, (int)p.b1, 0u, n,
                         (const uint32_t *)nullptr, (const uint32_t *)nullptr, c->counts1, ba1));
    GESMC_TRY(launch(c, s, KID_SCAN, 0, k_colsum, dim3(nchunks), dim3(scan_threads), 0, c->counts1, p.ntiles1,
                     (int)p.b1, chunk, c->partial));
    GESMC_TRY(launch(c, s, KID_SCAN, 0, k_colscan_top, dim3(1), dim3(kTopThreads), 0, c->partial, nchunks, (int)p.b1,
                     c->coarse_off, c->tile_first, (uint32_t)kTile2));
    GESMC_TRY(launch(c, s, KID_SCAN, 0, k_colapply, dim3(nchunks), dim3(scan_threads), 0, c->counts1, p.ntiles1,
                     (int)p.b1, chunk, c->partial, c->coarse_off));
    const int lvl1_out = p.b2 > 0 ? mid : dst;
    const size_t lds1 =
        scatter_lds_bytes(p.b1, kTile, kSrc1 == kSrcBatch, !src_emits_packed<kSrc1>(), ba1.dig_in_key == 0);
    const size_t lds2 = scatter_lds_bytes(p.b2, kTile2, kSrc2 == kSrcBatch, kSrc2 != kSrcPacked,
                                          kSrc2 != kSrcPacked && kSrc2 != kSrcHashed && ba2.dig_in_key == 0);
    GESMC_TRY(launch(c, s, kid_scatter1, n, k_scatter<kSrc1, kTile, scatter_threads(kTile), true>,
                     dim3(persistent_blocks(c, k_scatter<kSrc1, kTile, scatter_threads(kTile), true>, lds1, p.ntiles1, scatter_threads(kTile))), dim3(scatter_threads(kTile)), lds1, src_i, src_k, idx[lvl1_out], key[lvl1_out], t, k0,
                     k1, shift1, (int)p.b1, 0u, n, (const uint32_t *)nullptr, (const uint32_t *)nullptr,
                     (const uint32_t *)c->counts1, c->err, ba1));
    if (p.b2 == 0) {
        *out = dst;
        *bucket_off = c->coarse_off;
        *nbuckets = p.ncoarse;
        return GESMC_OK;
    }
    const uint32_t nd2 = 1u << p.b2;
    const uint32_t tiles2 = (uint32_t)level2_tiles(p) + p.ncoarse;  // >= sum over segments of their tiles
    GESMC_TRY(ensure_words(c, &c->counts2, &c->cap_counts2, rw.counts2));
    // packed words lost the first level's bits: the second level's are on top
    const int shift2 = kSrc2 == kSrcPacked ? 64 - (int)p.b2 : 64 - (int)p.bbits;
    GESMC_TRY(launch(c, s, kid_counts2, n, k_tile_counts<kSrc2, kTile2, false>,
                     dim3(persistent_blocks(c, k_tile_counts<kSrc2, kTile2, false>, (size_t)nd2 * 4, tiles2)), dim3(kBlock),
                     (size_t)nd2 * 4, idx[mid], key[mid], t, k0, k1, shift2, (int)p.b2, p.ncoarse, 0u,
                     (const uint32_t *)c->coarse_off, (const uint32_t *)c->tile_first, c->counts2, ba2));
    GESMC_TRY(launch(c, s, KID_SCAN, 0, k_segscan, dim3(p.ncoarse), dim3(kBlock), ((size_t)nd2 + kBlock + 1) * 4,
                     c->counts2, (int)p.b2, p.ncoarse, c->coarse_off, c->tile_first, c->fine_off));
    GESMC_TRY(launch(c, s, kid_scatter2, n, k_scatter<kSrc2, kTile2, scatter_threads(kTile2), false>,
                     dim3(persistent_blocks(c, k_scatter<kSrc2, kTile2, scatter_threads(kTile2), false>, lds2, tiles2, scatter_threads(kTile2))), dim3(scatter_threads(kTile2)), lds2, idx[mid], key[mid], idx[dst], key[dst], t, k0, k1, shift2, (int)p.b2,
                     p.ncoarse, 0u, (const uint32_t *)c->coarse_off, (const uint32_t *)c->tile_first,
                     (const uint32_t *)c->counts2, c->err, ba2));
    *out = dst;
    *bucket_off = c->fine_off;
    *nbuckets = p.nfine;
    return GESMC_OK;
}

template <int kSrc1, int kSrc2>
gesmc_status radix_distribute(gesmc_ctx *c, hipStream_t s, const Plan &p, uint32_t n, uint32_t t, uint32_t k0,
                              uint32_t k1, uint32_t *const *idx, unsigned long long *const *key, int src, int mid,
                              int dst, int *out, const uint32_t **bucket_off, uint32_t *nbuckets, int kid_counts1,
                              int kid_scatter1, int kid_counts2, int kid_scatter2, SrcArgs ba1, SrcArgs ba2,
                              const uint32_t *in_idx = nullptr, const unsigned long long *in_key = nullptr,
                              const EmitOut *eo = nullptr, bool counts1_ready = false) {
#define GESMC_RADIX_T(T1, T2)                                                                                   \
    radix_distribute_t<kSrc1, kSrc2, T1, T2>(c, s, p, n, t, k0, k1, idx, key, src, mid, dst, out, bucket_off, nbuckets, \
                                             kid_counts1, kid_scatter1, kid_counts2, kid_scatter2, ba1, ba2, in_idx,  \
                                             in_key, eo, counts1_ready)
    const uint32_t t2 = p.tile2 ? p.tile2 : p.tile;
    if (p.tile == (uint32_t)kTileLarge)
        return t2 == (uint32_t)kTileLarge ? GESMC_RADIX_T(kTileLarge, kTileLarge) : GESMC_RADIX_T(kTileLarge, kTileSmall);
    return GESMC_RADIX_T(kTileSmall, kTileSmall);
#undef GESMC_RADIX_T
}

// One superstep of a batch: the graphs switched (ranks [0, ngraphs), a
// prefix of the rank order) and the per-position arrays of the batch.
struct BatchStep {
    const BatchGraph *gr;      // device, per rank
    uint32_t ngraphs;          // ranks switched in this superstep
    uint32_t step;             // batch superstep s (graph g runs its superstep t0_g + s)
    const uint32_t *pg;        // device: rank of the graph holding each position
    uint32_t *bk;              // device: global bucket of each record between the radix levels
    unsigned long long *acc;   // device: per-rank outcome counts (nullable)
    GraphErr ge;               // per-rank error attribution (gr = nullptr: none)
    uint64_t vend;             // vertex ids of the switched ranks are below this
    uint64_t dend;             // and so are the id offsets v - u of their edges (the largest n)
    uint64_t mmax;             // the largest record count of a graph (even: mpad)
};

// Sorts the records of [0, m) of buffer `src` by (K_i, i) of superstep t --
// per graph with its own keys if `bs` describes a batch (plan bits then
// number the global buckets).  Returns the buffer index holding the sorted
// records.
// counts1_ready: the first level's tile counts of superstep t are in
// c->counts1 already (k_decide_chain of superstep t - 1 wrote them).
gesmc_status permute(gesmc_ctx *c, hipStream_t s, const Plan &p, uint32_t t, uint32_t k0, uint32_t k1, int src,
                     int *sorted_out, bool clear_table, const BatchStep *bs = nullptr, bool counts1_ready = false) {
    const uint32_t m = p.m;
    const int X = (src + 1) % 3, Y = (src + 2) % 3;
    // the table strategy resets its table, statuses and list counters here;
    // the sorted-tuples emit writes every status and clears the counters itself
    if (clear_table) {
        const uint64_t tslots = c->tab_slots;
        GESMC_TRY(launch(c, s, KID_STEP_CLEAR, tslots, k_step_clear,
                         dim3(grid_stride_blocks(c, std::max<uint64_t>(p.ell, tslots) + 1)), dim3(kBlock), 0, c->tab,
                         tslots, c->st, p.ell, c->ucount));
    }
    const size_t sort_lds = sort_lds_bytes(c->sort_cap);
    if (p.bbits == 0) {
        // one bucket: sort src -> X (scratch keys in Y)
        GESMC_TRY(launch(c, s, KID_MISC, 0, k_setup_level1, dim3(1), dim3(64), 0, c->lvl1_seg, c->lvl1_tiles, m,
                         p.ntiles1));
        GESMC_TRY(launch(c, s, KID_SORT, m, k_sort_buckets, dim3(1), dim3(kBlock), sort_lds, c->idx[src], c->key[src],
                         c->idx[X], c->key[X], c->key[Y], t, k0, k1, 0, (const uint32_t *)c->lvl1_seg, 1u, m,
                         c->sort_cap, c->ctr_step, bs ? bs->gr : nullptr, bs ? bs->ngraphs : 0u,
                         bs ? bs->step : 0u));
        *sorted_out = X;
        return GESMC_OK;
    }
    int dist = 0;
    const uint32_t *boff = nullptr;
    uint32_t nb = 0;
    const int mid = X, dst = p.b2 > 0 ? Y : X;
    if (bs) {
        const SrcArgs ba1{bs->gr, bs->pg, bs->bk, bs->step, (int)p.bbits};
        const SrcArgs ba2{bs->gr, bs->bk, nullptr, bs->step, (int)p.bbits};
        GESMC_TRY((radix_distribute<kSrcBatch, kSrcBucket>(c, s, p, m, t, k0, k1, c->idx, c->key, src, mid, dst, &dist,
                                                           &boff, &nb, KID_COUNTS1, KID_SCATTER1, KID_COUNTS2,
                                                           KID_SCATTER2, ba1, ba2, nullptr, nullptr, nullptr,
                                                           counts1_ready)));
    } else {
        SrcArgs pa{};
        pa.dig_in_key = p.dig_in_key;
        GESMC_TRY((radix_distribute<kSrcPerm, kSrcPerm>(c, s, p, m, t, k0, k1, c->idx, c->key, src, mid, dst, &dist,
                                                        &boff, &nb, KID_COUNTS1, KID_SCATTER1, KID_COUNTS2,
                                                        KID_SCATTER2, pa, pa, nullptr, nullptr, nullptr,
                                                        counts1_ready)));
    }
    const int sorted = (dist == X) ? Y : X;  // sort into the buffer not holding the buckets
    GESMC_TRY(launch(c, s, KID_SORT, m, k_sort_buckets, dim3(persistent_blocks(c, k_sort_buckets, sort_lds, nb)),
                     dim3(kBlock), sort_lds, c->idx[dist], c->key[dist], c->idx[sorted], c->key[sorted], c->key[src],
                     t, k0, k1, (int)p.bbits, boff, nb, m, c->sort_cap, c->ctr_step, bs ? bs->gr : nullptr,
                     bs ? bs->ngraphs : 0u, bs ? bs->step : 0u));
    *sorted_out = sorted;
    return GESMC_OK;
}

// Partitions the tuples in tuple buffer 0 (nslots slots, empty keys dropped)
// by key hash and resolves every partition.
// Tuples come from tuple buffer 0 (validation), or -- with `emit` -- are
// computed from the pair records si / sk of a superstep in the first pass.
struct EmitSource {
    const uint32_t *si;
    const unsigned long long *sk;
    uint32_t t, k0, k1;
    SrcArgs sa;
};

// Bits of x - 1 (x >= 1): the width of the values [0, x).
int width_below(uint64_t x) {
    int b = 0;
    while (b < 64 && (x - 1) >> b) ++b;
    return b;
}

// Packed 8-byte tuple words (TuplePack) for nslots tuple slots of keys (u, v)
// with v below vend and v - u below dend, if the bits allow: the hash bits
// left after the first level plus the tag code fit 64 bits, and at least
// kCellBits hash bits remain below both levels for the resolve's cells.
// w = 0: 12-byte tuples.
TuplePack tuple_pack(const gesmc_ctx *c, const Plan &p, uint32_t nslots, uint64_t vend, uint64_t dend,
                     uint64_t mmax = 0) {
    TuplePack pk{0, 0, 0, 0, 0, 0};
    if (!c->pack_tuples || vend < 2 || dend < 2) return pk;
    const int vb = width_below(vend), db = width_below(std::min(dend, vend)), w = vb + db;
    int kb = std::max(1, width_below(2ull * (nslots / 4) + 1));  // 2 ell < 2^kb, so ell < 2^kb - 1
    int local = 0;
    if ((w - (int)p.b1 + kb + 1 > 64 || c->pack_tuples == 2) && mmax > 0) {
        // a batch (mmax: its largest even record count): tags local to each
        // graph, codes below mmax, so its switches k < mmax / 2 < 2^kb - 1
        kb = std::max(1, width_below(mmax + 1));
        local = 1;
    }
    if (w > 62 || w - (int)p.b1 + kb + 1 > 64 || w - (int)p.bbits < kCellBits) return pk;
    pk.w = w;
    pk.db = db;
    pk.kb = kb;
    pk.b1 = (int)p.b1;
    pk.b2 = (int)p.b2;
    pk.local = local;
    return pk;
}

gesmc_status partition_and_resolve(gesmc_ctx *c, hipStream_t s, uint32_t nslots, uint32_t dup_bit,
                                   GraphErr ge = GraphErr{nullptr, 0, nullptr}, const EmitSource *emit = nullptr,
                                   uint64_t vend = 0, uint64_t dend = 0, const EmitOut *eo = nullptr,
                                   uint64_t mmax = 0) {
    const Plan p = make_plan(c, nslots);
    int parts = 0;
    const uint32_t *poff = nullptr;
    uint32_t np = 0;
    // graph-local tags need the graphs (emit: their first switches; resolve: the key's graph)
    const TuplePack pk = emit ? tuple_pack(c, p, nslots, vend, dend, (ge.gr && emit->sa.pg) ? mmax : 0)
                              : TuplePack{0, 0, 0, 0, 0, 0};
    c->tuple_bytes = pk.w ? 8u : 12u;
    if (pk.w) {
        SrcArgs sa = emit->sa;
        sa.pk = pk;
        if (pk.local)
            GESMC_TRY((radix_distribute<kSrcEmitPackedLocal, kSrcPacked>(
                c, s, p, nslots, emit->t, emit->k0, emit->k1, c->tu_tag, c->tu_key, 0, 1, p.b2 > 0 ? 2 : 1, &parts,
                &poff, &np, KID_TCOUNTS1, KID_TSCATTER1, KID_TCOUNTS2, KID_TSCATTER2, sa, SrcArgs{}, emit->si,
                emit->sk, eo)));
        else
            GESMC_TRY((radix_distribute<kSrcEmitPacked, kSrcPacked>(
                c, s, p, nslots, emit->t, emit->k0, emit->k1, c->tu_tag, c->tu_key, 0, 1, p.b2 > 0 ? 2 : 1, &parts,
                &poff, &np, KID_TCOUNTS1, KID_TSCATTER1, KID_TCOUNTS2, KID_TSCATTER2, sa, SrcArgs{}, emit->si,
                emit->sk, eo)));
        const int scratch = parts == 2 ? 1 : 0;
        const size_t rlds = resolve_lds_bytes(c->sort_cap, true);
        GESMC_TRY(launch(c, s, KID_RESOLVE, nslots, k_resolve<true>,
                         dim3(persistent_blocks(c, k_resolve<true>, rlds, np)), dim3(kBlock), rlds, c->tu_tag[parts],
                         c->tu_key[parts], c->tu_tag[scratch], c->tu_key[scratch], (int)p.b2, poff, np, c->sort_cap,
                         c->info, c->err, dup_bit, c->ctr_step, ge, pk));
        return GESMC_OK;
    }
    if (emit)
        GESMC_TRY((radix_distribute<kSrcEmit, kSrcHashed>(c, s, p, nslots, emit->t, emit->k0, emit->k1, c->tu_tag,
                                                        c->tu_key, 0, 1, p.b2 > 0 ? 2 : 1, &parts, &poff, &np,
                                                        KID_TCOUNTS1, KID_TSCATTER1, KID_TCOUNTS2, KID_TSCATTER2,
                                                        emit->sa, SrcArgs{}, emit->si, emit->sk, eo)));
    else
        GESMC_TRY((radix_distribute<kSrcHash, kSrcHashed>(c, s, p, nslots, 0u, 0u, 0u, c->tu_tag, c->tu_key, 0, 1,
                                                        p.b2 > 0 ? 2 : 1, &parts, &poff, &np, KID_TCOUNTS1,
                                                        KID_TSCATTER1, KID_TCOUNTS2, KID_TSCATTER2, SrcArgs{},
                                                        SrcArgs{})));
    const int scratch = parts == 2 ? 1 : 0;
    const size_t rlds = resolve_lds_bytes(c->sort_cap);
    GESMC_TRY(launch(c, s, KID_RESOLVE, nslots, k_resolve<false>,
                     dim3(persistent_blocks(c, k_resolve<false>, rlds, np)), dim3(kBlock), rlds, c->tu_tag[parts],
                     c->tu_key[parts], c->tu_tag[scratch], c->tu_key[scratch], (int)p.bbits, poff, np, c->sort_cap,
                     c->info, c->err, dup_bit, c->ctr_step, ge, TuplePack{0, 0, 0, 0, 0, 0}));
    return GESMC_OK;
}

// One superstep with the partitioned resolution (state in buffer 0).
// vend bounds the vertex ids of the keys (a batch: bs->vend, bs->dend).
// counts1_ready: this superstep's first radix level was counted by the
// previous one; count_next: count superstep t + 1's in the first decision
// round (a plan with a first radix level; a batch passes its next step's
// plan, next_p, whose positions are a prefix of this step's).
gesmc_status superstep_partitioned(gesmc_ctx *c, hipStream_t s, const Plan &p, uint32_t t, uint32_t k0, uint32_t k1,
                                   uint32_t pl, uint32_t dup_bit, const BatchStep *bs = nullptr, uint64_t vend = 0,
                                   uint32_t cls = 0, bool counts1_ready = false, bool count_next = false,
                                   const Plan *next_p = nullptr) {
    int sorted = 0;
    GESMC_TRY(permute(c, s, p, t, k0, k1, 0, &sorted, false, bs, counts1_ready));
    const uint32_t *si = c->idx[sorted];
    const unsigned long long *sk = c->key[sorted];
    const uint32_t nslots = 4 * p.ell + (p.m & 1u);
    // per-block counts of emit and the first round go to slots [0, ge) and [ge, ge + gd);
    // with the tuples computed from the pair records, the emit runs inside the
    // first tuple count pass (k_emit_counts), one workgroup per tile up to
    // kEmitSlotsMax
    const bool fused = c->fuse_emit && GESMC_FUSE_EMIT_COUNTS;
    const uint32_t ge = fused ? std::min<uint32_t>(kEmitSlotsMax, make_plan(c, nslots).ntiles1)
                              : grid_stride_blocks(c, (uint64_t)p.ell + 1);
    const uint32_t gd = grid_stride_blocks(c, p.ell);
    SrcArgs sa{};
    sa.gr = bs ? bs->gr : nullptr;
    sa.pg = bs ? bs->pg : nullptr;
    sa.step = bs ? bs->step : 0u;
    sa.m = p.m;
    sa.pl = pl;
    sa.cls = cls;
    // directed keys (tail, head) do not fit the packed (u, v - u) coding
    if (cls & CLS_DIRECTED) vend = 0;
    if (!fused)
        GESMC_TRY(launch(c, s, KID_EMIT, p.ell, k_emit, dim3(ge), dim3(kBlock), 0, si, sk, t, k0, k1, sa, c->info,
                         c->st, c->idx[0], c->key[0], c->bslot, c->ucount));
    const EmitSource es{si, sk, t, k0, k1, sa};
    const EmitOut eo{c->info, c->st, c->idx[0], c->key[0], c->bslot, c->ucount, ge};
    if (!c->fuse_emit)
        GESMC_TRY(launch(c, s, KID_EMIT, nslots, k_emit_tuples, dim3(grid_stride_blocks(c, nslots)), dim3(kBlock), 0,
                         si, sk, t, k0, k1, sa, nslots, c->tu_tag[0], c->tu_key[0]));
    GESMC_TRY(partition_and_resolve(c, s, nslots, dup_bit, bs ? bs->ge : GraphErr{nullptr, 0, nullptr},
                                    c->fuse_emit ? &es : nullptr, bs ? bs->vend : vend, bs ? bs->dend : vend,
                                    fused ? &eo : nullptr, bs ? bs->mmax : 0));
    if (p.ell == 0) return GESMC_OK;
    NextCounts nc{};
    if (count_next) {
        const Plan &q = next_p ? *next_p : p;
        GESMC_TRY(ensure_words(c, &c->counts1, &c->cap_counts1, radix_words(q).counts1));
        nc = NextCounts{c->counts1, t + 1, k0, k1, 64 - (int)q.b1, (int)q.b1, q.tile, q.m,
                        bs ? bs->gr : nullptr, bs ? bs->pg : nullptr, bs ? bs->step + 1 : 0u, (int)q.bbits};
    }
    GESMC_TRY(launch(c, s, KID_DECIDE_CHAIN1, p.ell, k_decide_chain, dim3(gd), dim3(kBlock), 0, si, sk, p.ell,
                     c->info, c->st, c->idx[0], c->key[0], (const uint32_t *)nullptr,
                     (const uint32_t *)nullptr, c->ulist[0], &c->ucount[0], (uint32_t *)nullptr, c->bslot + ge,
                     c->ctr_step, cls, nc));
    const uint32_t rblocks = std::max<uint32_t>(1, std::min<uint32_t>(ceil_div(p.ell, kBlock), c->num_cus * 4));
    int j = 0;
    for (; j < c->fast_rounds; ++j) {
        GESMC_TRY(launch(c, s, KID_DECIDE_CHAIN, 0, k_decide_chain, dim3(rblocks), dim3(kBlock), 0, si, sk, p.ell,
                         c->info, c->st, c->idx[0], c->key[0], (const uint32_t *)c->ulist[j % 2],
                         (const uint32_t *)&c->ucount[j % 3], c->ulist[(j + 1) % 2], &c->ucount[(j + 1) % 3],
                         &c->ucount[(j + 2) % 3], (uint4 *)nullptr, c->ctr_step, cls, NextCounts{}));
    }
    GESMC_TRY(launch(c, s, KID_FINISH_CHAIN, 0, k_finish_chain, dim3(1), dim3(kFinishBlock), 0, si, sk, p.ell,
                     c->info, c->st, c->idx[0], c->key[0], c->ulist[j % 2], &c->ucount[j % 3],
                     c->ulist[(j + 1) % 2], &c->ucount[(j + 1) % 3], (const uint4 *)c->bslot, ge + gd,
                     c->ctr_step, c->err, c->round_limit, cls));
    if (bs && bs->acc)
        GESMC_TRY(launch(c, s, KID_MISC, 0, k_graph_stats, dim3(ceil_div(p.ell, kStatsChunk)), dim3(kBlock), 0,
                         (const uint8_t *)c->st, bs->gr, bs->ngraphs, p.ell, bs->acc));
    return GESMC_OK;
}

// One superstep of a multi-edge class (state in buffer 0): the permutation,
// then every switch decided from its own pair records (k_decide_local).
gesmc_status superstep_local(gesmc_ctx *c, hipStream_t s, const Plan &p, uint32_t t, uint32_t k0, uint32_t k1,
                             uint32_t pl, uint32_t cls) {
    int sorted = 0;
    GESMC_TRY(permute(c, s, p, t, k0, k1, 0, &sorted, false));
    GESMC_TRY(launch(c, s, KID_DECIDE_LOCAL, p.ell, k_decide_local, dim3(grid_stride_blocks(c, (uint64_t)p.ell + 1)),
                     dim3(kBlock), 0, c->idx[sorted], c->key[sorted], p.m, t, k0, k1, pl, cls, c->st, c->idx[0],
                     c->key[0], c->ctr_step));
    return GESMC_OK;
}

// One superstep t on the state records in buffer 0 (result back in buffer 0).
gesmc_status superstep(gesmc_ctx *c, hipStream_t s, const Plan &p, uint32_t t, uint32_t k0, uint32_t k1, uint32_t pl,
                       uint32_t dup_bit) {
    int sorted = 0;
    GESMC_TRY(permute(c, s, p, t, k0, k1, 0, &sorted, true));
    const uint32_t nslots = (uint32_t)c->tab_slots;
    const uint32_t *si = c->idx[sorted];
    const unsigned long long *sk = c->key[sorted];
    GESMC_TRY(launch(c, s, KID_BUILD, p.ell, k_build, dim3(ceil_div((uint64_t)p.ell + 1, kBlock)), dim3(kBlock), 0,
                     si, sk, p.m, t, k0, k1, pl, c->tab, nslots, c->sw_slot, c->st, c->idx[0], c->key[0], c->ctr_step,
                     c->err, dup_bit));
    if (p.ell == 0) return GESMC_OK;
    GESMC_TRY(launch(c, s, KID_DECIDE1, p.ell, k_decide_first, dim3(ceil_div(p.ell, kBlock)), dim3(kBlock), 0, si, sk,
                     p.ell, c->tab, c->sw_slot, c->st, c->idx[0], c->key[0], c->ulist[0], &c->ucount[0], c->ctr_step,
                     c->err));
    const uint32_t rblocks = std::max<uint32_t>(1, std::min<uint32_t>(ceil_div(p.ell, kBlock), c->num_cus * 4));
    int cur = 0;
    for (int rr = 0; rr < c->fast_rounds; ++rr) {
        const int nxt = 1 - cur;
        GESMC_TRY(launch(c, s, KID_ROUND_RESET, 0, k_round_reset, dim3(rblocks), dim3(kBlock), 0, c->ulist[cur],
                         &c->ucount[cur], p.ell, c->tab, c->sw_slot, &c->ucount[nxt]));
        GESMC_TRY(launch(c, s, KID_ROUND_CLAIM, 0, k_round_claim, dim3(rblocks), dim3(kBlock), 0, c->ulist[cur],
                         &c->ucount[cur], p.ell, c->tab, c->sw_slot));
        GESMC_TRY(launch(c, s, KID_ROUND_DECIDE, 0, k_round_decide, dim3(rblocks), dim3(kBlock), 0, si, sk, p.ell,
                         c->tab, c->sw_slot, c->st, c->idx[0], c->key[0], c->ulist[cur], &c->ucount[cur],
                         c->ulist[nxt], &c->ucount[nxt], c->ctr_step, c->err));
        cur = nxt;
    }
    GESMC_TRY(launch(c, s, KID_FINISH, 0, k_finish, dim3(1), dim3(kFinishBlock), 0, si, sk, p.ell, c->tab,
                     c->sw_slot, c->st, c->idx[0], c->key[0], c->ulist[cur], &c->ucount[cur], c->ulist[1 - cur],
                     &c->ucount[1 - cur], c->ctr_step, c->err));
    return GESMC_OK;
}

// Writes the state records of buffer 0 (idx, key) to out[idx].  From
// 2^20 records on, a one-level distribution by the index's top bits
// (kSrcIdx, buffer 0 -> 1) first gathers consecutive indices into buckets
// of at most 2^17 records, which k_unpermute_buckets writes back XCD by XCD
// (2.12 -> 1.65 ms at 2^26 edges: each XCD's scattered stores stay in a
// 1 MB window at a time).
constexpr uint32_t kUnpermuteBuckets = 1u << 20;  // records from which the buckets pay
gesmc_status unpermute(gesmc_ctx *c, hipStream_t s, uint32_t m, unsigned long long *out) {
    if (m < kUnpermuteBuckets || !c->unpermute_buckets || alloc_forbidden()) {
        return launch(c, s, KID_UNPERMUTE, m, k_unpermute, dim3(grid_stride_blocks(c, m)), dim3(kBlock), 0,
                      c->idx[0], c->key[0], m, out, c->err);
    }
    const int W = width_below(m);  // every index < 2^W
    Plan p;
    p.m = m;
    p.ell = m / 2;
    p.bbits = (uint32_t)std::min<int>((int)kMaxCoarseBits, std::max(1, W - 17));
    p.b1 = p.bbits;
    p.b2 = 0;
    p.ncoarse = p.nfine = 1u << p.bbits;
    p.tile = tile_for(m);
    p.ntiles1 = std::max<uint32_t>(1, ceil_div(m, p.tile));
    SrcArgs sa{};
    sa.ishift = 64u - (uint32_t)W;
    int dist = 0;
    const uint32_t *boff = nullptr;
    uint32_t nb = 0;
    GESMC_TRY((radix_distribute<kSrcIdx, kSrcIdx>(c, s, p, m, 0u, 0u, 0u, c->idx, c->key, 0, 1, 1, &dist, &boff, &nb,
                                                  KID_UNPERMUTE, KID_UNPERMUTE, KID_UNPERMUTE, KID_UNPERMUTE, sa,
                                                  SrcArgs{})));
    const uint32_t per_xcd = std::max<uint32_t>(1, c->num_cus / 8) * 4;
    return launch(c, s, KID_UNPERMUTE, m, k_unpermute_buckets, dim3(8 * per_xcd), dim3(kBlock), 0,
                  (const uint32_t *)c->idx[dist], (const unsigned long long *)c->key[dist], boff, nb, m, out,
                  (const uint32_t *)c->err);
}

gesmc_status check_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return GESMC_OK;
    set_error("%s: %s", what, hipGetErrorString(e));
    return GESMC_E_DEVICE;
}

gesmc_status collect_profile(gesmc_ctx *c) {
    for (const auto &r : c->recs) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            c->prof_ms[r.kid] += ms;
            c->prof_launch[r.kid] += 1;
            c->prof_items[r.kid] += r.items;
        } else {
            (void)hipGetLastError();
        }
    }
    c->recs.clear();
    c->ev_used = 0;
    return GESMC_OK;
}

gesmc_status map_err(uint32_t e) {
    if (e & (ERR_LOOP | ERR_DUP)) {
        set_error("input is not a graph of the requested class (%s)", (e & ERR_LOOP) ? "loop" : "duplicate edge");
        return GESMC_E_NOT_SIMPLE;
    }
    if (e & ERR_RANGE) {
        set_error("vertex id out of range");
        return GESMC_E_RANGE;
    }
    if (e & ERR_ROUNDS) {
        set_error("a superstep needed more decision rounds than GESMC_OPT_ROUND_LIMIT allows");
        return GESMC_E_ROUNDS;
    }
    if (e) {
        set_error("internal consistency check failed (error bits 0x%x)", e);
        return GESMC_E_INTERNAL;
    }
    return GESMC_OK;
}

// The plain form on a graph that fits one workgroup's LDS: per piece of at
// most kSmallPiSteps supersteps, their permutations in parallel
// (k_small_perm, one workgroup each; the first also clears the error word
// and the counts), then the chain itself on one workgroup (k_small_plain),
// which resumes from the previous piece's output.  The counts (legal, loop,
// exists, P_L) go to error words 8 .. 15, so one copy brings back both; no
// rounds are recorded.
template <uint32_t kMax, uint32_t kThreads, bool kCompact>
gesmc_status run_small_pieces(gesmc_ctx *c, hipStream_t s, int kid, const unsigned long long *in,
                              unsigned long long *out, uint32_t m, uint32_t n, uint32_t t0, uint32_t r, uint32_t pl,
                              uint32_t k0, uint32_t k1, unsigned long long *acc) {
    static_assert(kMax <= kCmpMax, "permutation rows of the small-graph path hold kCmpMax entries");
    for (uint32_t done = 0; done < r;) {
        const uint32_t rr = std::min<uint32_t>(r - done, kSmallPiSteps);
        GESMC_TRY(launch(c, s, KID_SMALL_PERM, (uint64_t)rr * m, k_small_perm<kMax, kThreads, kCompact>, dim3(rr),
                         dim3(kThreads), 0, m, t0 + done, k0, k1, c->small_pi, done ? nullptr : c->err));
        GESMC_TRY(launch(c, s, kid, m, k_small_plain<kMax, kThreads, kCompact>, dim3(1), dim3(kThreads), 0,
                         done ? (const unsigned long long *)out : in, out, m, n, t0 + done, rr, pl, k0, k1, acc,
                         c->err, (const uint16_t *)c->small_pi));
        done += rr;
    }
    return GESMC_OK;
}

gesmc_status run_small_impl(gesmc_ctx *c, hipStream_t s, const uint64_t *d_in, uint64_t *d_out, uint32_t m,
                            uint32_t n, uint64_t seed, uint32_t t0, uint32_t r, uint32_t pl, gesmc_stats *stats) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    unsigned long long *acc = (unsigned long long *)(c->err + 8);  // legal, loop, exists, P_L
    const auto *in = (const unsigned long long *)d_in;
    auto *out = (unsigned long long *)d_out;
    if (!c->small_pi) GESMC_TRY(dev_alloc(c, (void **)&c->small_pi, kSmallPiBytes));
    GESMC_TRY(check_hip(hipEventRecord(c->call_a, s), "hipEventRecord"));
    if (m <= kSmallMax)
        GESMC_TRY((run_small_pieces<kSmallMax, kSmallThreads, false>(c, s, KID_SMALL, in, out, m, n, t0, r, pl, k0,
                                                                     k1, acc)));
    else if (m <= kMidMax)
        GESMC_TRY((run_small_pieces<kMidMax, kMidThreads, false>(c, s, KID_SMALL_MID, in, out, m, n, t0, r, pl, k0,
                                                                 k1, acc)));
    else
        GESMC_TRY((run_small_pieces<kCmpMax, kCmpThreads, true>(c, s, KID_SMALL_CMP, in, out, m, n, t0, r, pl, k0,
                                                                k1, acc)));
    GESMC_TRY(check_hip(hipEventRecord(c->call_b, s), "hipEventRecord"));
    GESMC_TRY(check_hip(hipMemcpyAsync(c->h_err, c->err, 64, hipMemcpyDeviceToHost, s), "hipMemcpyAsync"));
    GESMC_TRY(check_hip(hipStreamSynchronize(s), "hipStreamSynchronize"));
    if (c->profile) collect_profile(c);
    GESMC_TRY(map_err(*c->h_err));
    if (stats) {
        uint64_t h[4];
        memcpy(h, c->h_err + 8, sizeof(h));
        memset(stats, 0, sizeof(*stats));
        stats->supersteps = r;
        stats->attempts = (uint64_t)r * (m / 2);
        stats->legal = h[0];
        stats->rej_loop = h[1];
        stats->rej_exists = h[2];
        stats->rej_pl = h[3];
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->call_a, c->call_b) == hipSuccess)
            stats->ms_device = ms;
        else
            (void)hipGetLastError();
    }
    return GESMC_OK;
}

// Adaptive multi-workgroup rounds of plain calls: after a call whose
// supersteps took more than kAdaptRoundsAbove decision rounds, the next
// plain call of the context runs kAdaptRoundsMany (power-law gamma = 2.01,
// n = 2^20: 2.4e8 -> 3.4e8 attempts/s), else kAdaptRoundsFew (each extra
// round is a launch, most of them empty on graphs without hubs).
constexpr uint64_t kAdaptRoundsAbove = 16;
constexpr int kAdaptRoundsMany = 128, kAdaptRoundsFew = 2;

gesmc_status run_impl(gesmc_ctx *c, void *stream, const uint64_t *d_in, uint64_t *d_out, uint64_t m64, uint32_t n,
                      uint64_t seed, uint32_t t0, uint32_t r, uint32_t pl, gesmc_stats *stats,
                      gesmc_step_stats *steps, uint8_t *d_outcome, uint32_t cls = 0) {
    if (!c) {
        set_error("null context");
        return GESMC_E_INVAL;
    }
    if (m64 > 0 && (!d_in || !d_out)) {
        set_error("null edge pointer");
        return GESMC_E_INVAL;
    }
    if (m64 >= kMaxEdges) {
        set_error("m = %llu exceeds the limit 2^30 - 1", (unsigned long long)m64);
        return GESMC_E_RANGE;
    }
    if ((uint64_t)t0 + r > 0x100000000ull) {
        set_error("superstep counter t0 + r overflows 32 bits");
        return GESMC_E_INVAL;
    }
    GESMC_TRY(check_hip(hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    const uint32_t m = (uint32_t)m64;
    // small graphs (Sec. 7's base case): every superstep in one workgroup's LDS
    // (the permutations computed ahead), when no per-superstep records or
    // outcome codes are asked for
    if (cls > CLS_ALL) {
        set_error("graph class %u has bits other than loops (1), multi-edges (2) and directed (4)", cls);
        return GESMC_E_INVAL;
    }
    if (cls == 0 && c->small_graphs && c->strategy == 0 && m >= 2 && r > 0 && !steps && !d_outcome &&
        (m <= kMidMax || (m <= kCmpMax && n <= kCmpMaxN)))
        return run_small_impl(c, s, d_in, d_out, m, n, seed, t0, r, pl, stats);
    GESMC_TRY(ensure_capacity(c, m, cls != 0 && !(cls & CLS_MULTI)));
    // the multi-workgroup decision rounds of this call (restored on return)
    struct FastRounds {
        gesmc_ctx *c;
        int saved;
        ~FastRounds() { c->fast_rounds = saved; }
    } fast_rounds_guard{c, c->fast_rounds};
    if (c->fast_rounds_auto) c->fast_rounds = c->adapt_rounds;
    GESMC_TRY(ensure_counters(c, r));
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    c->tuple_bytes = 0;
    GESMC_TRY(check_hip(hipEventRecord(c->call_a, s), "hipEventRecord"));
    const uint64_t zero_words = 64 + (uint64_t)std::max<uint32_t>(r, 1) * (sizeof(StepCounters) / 4);
    GESMC_TRY(launch(c, s, KID_MISC, 0, k_zero_words, dim3(4), dim3(256), 0, c->err, (uint64_t)64));
    GESMC_TRY(launch(c, s, KID_MISC, 0, k_zero_words, dim3(16), dim3(256), 0, (uint32_t *)c->ctr,
                     zero_words - 64));
    if (m > 0)
        GESMC_TRY(launch(c, s, KID_LOAD, m, k_load, dim3(grid_stride_blocks(c, m)), dim3(kBlock), 0,
                         (const unsigned long long *)d_in, m, n, c->idx[0], c->key[0], c->err, cls));
    Plan p = make_plan(c, m);
    p.dig_in_key = digit_in_key(p, n);
    const uint32_t nslots = (uint32_t)c->tab_slots;
    // the graph classes run on the sorted tuples only (multi-edge classes
    // have no dependencies at all)
    const bool table = c->strategy == 1 && cls == 0;
    if (m >= 2 && r == 0 && !(cls & CLS_MULTI)) {
        c->ctr_step = c->ctr;
        if (table) {
            GESMC_TRY(launch(c, s, KID_STEP_CLEAR, c->tab_slots, k_step_clear,
                             dim3(grid_stride_blocks(c, c->tab_slots)), dim3(kBlock), 0, c->tab, c->tab_slots, c->st,
                             0u, c->ucount));
            GESMC_TRY(launch(c, s, KID_VALIDATE, m, k_validate, dim3(grid_stride_blocks(c, m)), dim3(kBlock), 0,
                             c->key[0], m, c->tab, nslots, c->err));
        } else {
            GESMC_TRY(launch(c, s, KID_EMIT, m, k_emit_sources, dim3(grid_stride_blocks(c, m)), dim3(kBlock), 0,
                             (const unsigned long long *)c->key[0], m, c->tu_tag[0], c->tu_key[0]));
            GESMC_TRY(partition_and_resolve(c, s, m, ERR_DUP));
        }
    }
    if (m >= 2) {
        // supersteps after the first take their first radix level's counts
        // from the previous superstep's first decision round
        const bool chain_counts = GESMC_COUNT_AHEAD && p.bbits > 0 && p.b1 > 0 && p.ell > 0;
        for (uint32_t q = 0; q < r; ++q) {
            c->ctr_step = c->ctr + q;
            const uint32_t dup = q == 0 ? ERR_DUP : ERR_INTERNAL;
            if (cls & CLS_MULTI)
                GESMC_TRY(superstep_local(c, s, p, t0 + q, k0, k1, pl, cls));
            else if (table)
                GESMC_TRY(superstep(c, s, p, t0 + q, k0, k1, pl, dup));
            else
                GESMC_TRY(superstep_partitioned(c, s, p, t0 + q, k0, k1, pl, dup, nullptr, n, cls,
                                                chain_counts && q > 0, chain_counts && q + 1 < r));
        }
    }
    if (d_outcome && p.ell > 0)
        GESMC_TRY(launch(c, s, KID_MISC, 0, k_copy_bytes, dim3(grid_stride_blocks(c, p.ell)), dim3(kBlock), 0,
                         (const uint8_t *)c->st, d_outcome, (uint64_t)p.ell));
    if (m > 0)
        GESMC_TRY(unpermute(c, s, m, (unsigned long long *)d_out));
    GESMC_TRY(check_hip(hipEventRecord(c->call_b, s), "hipEventRecord"));
    GESMC_TRY(check_hip(hipMemcpyAsync(c->h_err, c->err, 4, hipMemcpyDeviceToHost, s), "hipMemcpyAsync"));
    if (r > 0)
        GESMC_TRY(check_hip(hipMemcpyAsync(c->h_ctr, c->ctr, sizeof(StepCounters) * r, hipMemcpyDeviceToHost, s),
                            "hipMemcpyAsync"));
    GESMC_TRY(check_hip(hipStreamSynchronize(s), "hipStreamSynchronize"));
    if (c->profile) collect_profile(c);
    const gesmc_status st = map_err(*c->h_err);
    if (st != GESMC_OK) return st;
    if (c->fast_rounds_auto && m >= 2 && r > 0) {
        // supersteps with long dependency chains (hub edges) finish faster
        // with many multi-workgroup rounds before the one-workgroup finisher;
        // short ones would only pay empty launches
        uint64_t maxr = 0;
        for (uint32_t q = 0; q < r; ++q) maxr = std::max<uint64_t>(maxr, c->h_ctr[q].rounds);
        c->adapt_rounds = maxr > kAdaptRoundsAbove ? kAdaptRoundsMany : kAdaptRoundsFew;
    }
    const uint64_t att = (m >= 2) ? p.ell : 0;
    if (steps) {
        for (uint32_t q = 0; q < r; ++q) {
            const StepCounters &h = c->h_ctr[q];
            steps[q] = gesmc_step_stats{att, h.legal, h.rej_loop, h.rej_exists, h.rej_pl, h.rounds,
                                        h.undecided_round1, h.fallback_buckets};
        }
    }
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->supersteps = r;
        for (uint32_t q = 0; q < r; ++q) {
            const StepCounters &h = c->h_ctr[q];
            stats->attempts += att;
            stats->legal += h.legal;
            stats->rej_loop += h.rej_loop;
            stats->rej_exists += h.rej_exists;
            stats->rej_pl += h.rej_pl;
            stats->rounds_sum += h.rounds;
            stats->rounds_max = std::max<uint32_t>(stats->rounds_max, (uint32_t)h.rounds);
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->call_a, c->call_b) == hipSuccess)
            stats->ms_device = ms;
        else
            (void)hipGetLastError();
        stats->tuple_bytes = c->tuple_bytes;
    }
    return GESMC_OK;
}

// ---------------------------------------------------------------------------
// gesmc_run_noalloc: gesmc_run with every per-call device buffer carved from
// `scratch` instead of the context's own allocations.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)GESMC_NOALLOC_SCRATCH_MIB << 20;
constexpr int kMaxDevices = 64;
constexpr uint32_t kNoAllocChunk = 64;  // supersteps per internal run: the context's counter records

std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (which must be current), looked
// up once per device with hipGetSymbolAddress: each device holds its own copy
// of the array.  *out may be null (look-up only).
gesmc_status noalloc_scratch_ptr(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d beyond the %d devices the no-allocation entry point supports", dev, kMaxDevices);
        return GESMC_E_DEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            set_error("hipGetSymbolAddress of the no-allocation scratch failed: %s", hipGetErrorString(e));
            return GESMC_E_DEVICE;
        }
        g_scratch_dev[dev] = p;
    }
    if (out) *out = g_scratch_dev[dev];
    return GESMC_OK;
}

// Every per-call device buffer of a plain sorted-tuples run, with its capacity.
struct RunBuffers {
    uint32_t *idx[3];
    unsigned long long *key[3];
    uint32_t *tu_tag[3];
    unsigned long long *tu_key[3];
    uint2 *info;
    uint32_t *sw_slot;
    uint8_t *st;
    uint32_t *ulist[2];
    Slot *tab;
    uint64_t cap_m, cap_tu, tab_slots;
    uint32_t *counts1, *counts2, *partial;
    uint64_t cap_counts1, cap_counts2, cap_partial;
    uint32_t *small;
    uint16_t *small_pi;
    uint4 *bslot;
    StepCounters *ctr;
    uint64_t ctr_cap;
    uint32_t *err, *ucount, *coarse_off, *tile_first, *lvl1_seg, *lvl1_tiles, *fine_off;
};

RunBuffers take_buffers(const gesmc_ctx *c) {
    RunBuffers b;
    for (int q = 0; q < 3; ++q) {
        b.idx[q] = c->idx[q];
        b.key[q] = c->key[q];
        b.tu_tag[q] = c->tu_tag[q];
        b.tu_key[q] = c->tu_key[q];
    }
    b.info = c->info;
    b.sw_slot = c->sw_slot;
    b.st = c->st;
    b.ulist[0] = c->ulist[0];
    b.ulist[1] = c->ulist[1];
    b.tab = c->tab;
    b.cap_m = c->cap_m;
    b.cap_tu = c->cap_tu;
    b.tab_slots = c->tab_slots;
    b.counts1 = c->counts1;
    b.counts2 = c->counts2;
    b.partial = c->partial;
    b.cap_counts1 = c->cap_counts1;
    b.cap_counts2 = c->cap_counts2;
    b.cap_partial = c->cap_partial;
    b.small = c->small;
    b.small_pi = c->small_pi;
    b.bslot = c->bslot;
    b.ctr = c->ctr;
    b.ctr_cap = c->ctr_cap;
    b.err = c->err;
    b.ucount = c->ucount;
    b.coarse_off = c->coarse_off;
    b.tile_first = c->tile_first;
    b.lvl1_seg = c->lvl1_seg;
    b.lvl1_tiles = c->lvl1_tiles;
    b.fine_off = c->fine_off;
    return b;
}

void put_buffers(gesmc_ctx *c, const RunBuffers &b) {
    for (int q = 0; q < 3; ++q) {
        c->idx[q] = b.idx[q];
        c->key[q] = b.key[q];
        c->tu_tag[q] = b.tu_tag[q];
        c->tu_key[q] = b.tu_key[q];
    }
    c->info = b.info;
    c->sw_slot = b.sw_slot;
    c->st = b.st;
    c->ulist[0] = b.ulist[0];
    c->ulist[1] = b.ulist[1];
    c->tab = b.tab;
    c->cap_m = b.cap_m;
    c->cap_tu = b.cap_tu;
    c->tab_slots = b.tab_slots;
    c->counts1 = b.counts1;
    c->counts2 = b.counts2;
    c->partial = b.partial;
    c->cap_counts1 = b.cap_counts1;
    c->cap_counts2 = b.cap_counts2;
    c->cap_partial = b.cap_partial;
    c->small = b.small;
    c->small_pi = b.small_pi;
    c->bslot = b.bslot;
    c->ctr = b.ctr;
    c->ctr_cap = b.ctr_cap;
    c->err = b.err;
    c->ucount = b.ucount;
    c->coarse_off = b.coarse_off;
    c->tile_first = b.tile_first;
    c->lvl1_seg = b.lvl1_seg;
    c->lvl1_tiles = b.lvl1_tiles;
    c->fine_off = b.fine_off;
}

// Lays out the buffers of a run over m edges from `base` (256-byte aligned
// pieces) and returns the bytes they take; base = nullptr only measures.
// Sizes follow ensure_capacity, the radix plans of the permutation (m
// records) and of the tuple partition (4 floor(m/2) + (m & 1) slots, or m
// for a validation-only call), and the fixed areas of gesmc_create.
uint64_t carve_buffers(const gesmc_ctx *c, unsigned char *base, uint64_t m, RunBuffers *out) {
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) -> void * {
        off = (off + 255) & ~255ull;
        void *p = base ? (void *)(base + off) : nullptr;
        off += bytes;
        return p;
    };
    RunBuffers b{};
    const uint64_t cap = std::max<uint64_t>(m, 1024), ntu = 2 * cap + 8;
    for (int q = 0; q < 3; ++q) {
        b.idx[q] = (uint32_t *)take(cap * 4);
        b.key[q] = (unsigned long long *)take(cap * 8);
    }
    for (int q = 0; q < 3; ++q) {
        b.tu_tag[q] = (uint32_t *)take(ntu * 4);
        b.tu_key[q] = (unsigned long long *)take(ntu * 8);
    }
    b.info = (uint2 *)take((cap + 8) * sizeof(uint2));
    b.st = (uint8_t *)take(cap / 2 + 64);
    for (int q = 0; q < 2; ++q) b.ulist[q] = (uint32_t *)take((cap / 2 + 64) * 4);
    b.sw_slot = nullptr;  // the table strategy only
    b.tab = nullptr;
    b.cap_m = cap;
    b.cap_tu = ntu;
    b.tab_slots = 0;
    uint64_t w1 = 1024, wp = 1024, w2 = 1024, nfine = 1;
    const uint64_t nslots = 4 * (m / 2) + (m & 1);
    for (uint64_t nrec : {m, nslots}) {
        if (nrec == 0) continue;
        const Plan p = make_plan(c, (uint32_t)nrec);
        const RadixWords rw = radix_words(p);
        w1 = std::max(w1, rw.counts1);
        wp = std::max(wp, rw.partial);
        w2 = std::max(w2, rw.counts2);
        nfine = std::max<uint64_t>(nfine, p.nfine);
    }
    b.counts1 = (uint32_t *)take(w1 * 4);
    b.partial = (uint32_t *)take(wp * 4);
    b.counts2 = (uint32_t *)take(w2 * 4);
    b.cap_counts1 = w1;
    b.cap_partial = wp;
    b.cap_counts2 = w2;
    const uint64_t nc = ((uint64_t)1 << kMaxCoarseBits) + 8;
    b.small = (uint32_t *)take((16 + 16 + 2 * nc + 8 + nfine + 8) * 4);
    b.small_pi = (uint16_t *)take(kSmallPiBytes);
    b.bslot = (uint4 *)take((kEmitSlotsMax + 2 * (uint64_t)grid_stride_blocks(c, ~0ull >> 1)) * sizeof(uint4));
    b.ctr = (StepCounters *)take(kNoAllocChunk * sizeof(StepCounters));
    b.ctr_cap = kNoAllocChunk;
    if (base) {
        uint32_t *w = b.small;
        b.err = w;
        b.ucount = w + 16;
        b.coarse_off = w + 32;
        b.tile_first = w + 32 + nc;
        b.lvl1_seg = w + 32 + 2 * nc;
        b.lvl1_tiles = w + 32 + 2 * nc + 4;
        b.fine_off = w + 32 + 2 * nc + 8;
    }
    if (out) *out = b;
    return off;
}

gesmc_status run_noalloc_impl(gesmc_ctx *c, void *stream, const uint64_t *d_in, uint64_t *d_out, uint64_t m,
                              uint32_t n, uint64_t seed, uint32_t t0, uint32_t r, uint32_t pl, gesmc_stats *stats) {
    if (!c) {
        set_error("null context");
        return GESMC_E_INVAL;
    }
    if (c->strategy != 0) {
        set_error("gesmc_run_noalloc needs the sorted-tuples strategy (GESMC_OPT_STRATEGY 0)");
        return GESMC_E_INVAL;
    }
    if (m > GESMC_NOALLOC_MAX_EDGES) {
        set_error("m = %llu exceeds the no-allocation limit of %llu edges (a %u MiB device array)",
                  (unsigned long long)m, (unsigned long long)GESMC_NOALLOC_MAX_EDGES, (unsigned)GESMC_NOALLOC_SCRATCH_MIB);
        return GESMC_E_RANGE;
    }
    if (m > 0 && (!d_in || !d_out)) {
        set_error("null edge pointer");
        return GESMC_E_INVAL;
    }
    if ((uint64_t)t0 + r > 0x100000000ull) {
        set_error("superstep counter t0 + r overflows 32 bits");
        return GESMC_E_INVAL;
    }
    GESMC_TRY(check_hip(hipSetDevice(c->device), "hipSetDevice"));
    void *base = nullptr;
    GESMC_TRY(noalloc_scratch_ptr(c->device, &base));
    const uint64_t need = carve_buffers(c, nullptr, m, nullptr);
    if (need > kScratchBytes) {
        set_error("internal: %llu scratch bytes needed for m = %llu, %llu held", (unsigned long long)need,
                  (unsigned long long)m, (unsigned long long)kScratchBytes);
        return GESMC_E_INTERNAL;
    }
    RunBuffers carved;
    carve_buffers(c, (unsigned char *)base, m, &carved);
    const RunBuffers saved = take_buffers(c);
    const bool prof = c->profile;
    c->profile = false;
    put_buffers(c, carved);
    t_no_alloc = true;
    gesmc_stats tot{};
    gesmc_status st = GESMC_OK;
    const uint64_t *src = d_in;
    uint32_t done = 0;
    do {  // pieces of at most kNoAllocChunk supersteps, each resuming where the last ended
        const uint32_t rr = std::min<uint32_t>(r - done, kNoAllocChunk);
        gesmc_stats part{};
        st = run_impl(c, stream, src, d_out, m, n, seed, t0 + done, rr, pl, &part, nullptr, nullptr);
        if (st != GESMC_OK) break;
        tot.attempts += part.attempts;
        tot.legal += part.legal;
        tot.rej_loop += part.rej_loop;
        tot.rej_exists += part.rej_exists;
        tot.rej_pl += part.rej_pl;
        tot.rounds_sum += part.rounds_sum;
        tot.rounds_max = std::max(tot.rounds_max, part.rounds_max);
        tot.ms_device += part.ms_device;
        tot.tuple_bytes = part.tuple_bytes;
        src = d_out;
        done += rr;
    } while (done < r);
    t_no_alloc = false;
    put_buffers(c, saved);
    c->profile = prof;
    if (st != GESMC_OK) return st;
    tot.supersteps = r;
    if (stats) *stats = tot;
    return GESMC_OK;
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
// Appends the position chunks of rank q's segment [poff, poff + len).
void add_chunks(std::vector<uint4> &v, uint32_t q, uint32_t poff, uint32_t len, uint32_t aux = 0) {
    for (uint32_t b = 0; b < len; b += kChunkPos)
        v.push_back(make_uint4(q, poff + b, poff + std::min<uint32_t>(len, b + kChunkPos), aux));
}

// Pinned staging of a call's small host -> device uploads (graph records,
// offsets, rank lists, chunks).  A copy from pageable memory may be carried
// out before hipMemcpyAsync returns, which holds back the launches queued
// after it; from pinned memory it is a DMA in stream order.  One arena per
// context: up_begin sizes it for the call (after the previous call's uploads
// have left it), up_copy stages and queues one upload, up_end marks the end.
gesmc_status up_begin(gesmc_ctx *c, uint64_t bytes, uint32_t copies) {
    if (c->up_pending) {
        GESMC_TRY(check_hip(hipEventSynchronize(c->up_ev), "hipEventSynchronize"));
        c->up_pending = false;
    }
    const uint64_t need = bytes + 64ull * copies;
    if (need > c->up_cap) {
        if (c->h_up) (void)hipHostFree(c->h_up);
        c->h_up = nullptr;
        c->up_cap = 0;
        const uint64_t cap = std::max<uint64_t>(need + need / 2, 1u << 16);
        if (hipHostMalloc((void **)&c->h_up, cap, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipHostMalloc of %llu bytes failed", (unsigned long long)cap);
            return GESMC_E_NOMEM;
        }
        c->up_cap = cap;
    }
    c->up_used = 0;
    return GESMC_OK;
}

gesmc_status up_copy(gesmc_ctx *c, hipStream_t s, void *dst, const void *src, uint64_t bytes) {
    if (bytes == 0) return GESMC_OK;
    const uint64_t off = (c->up_used + 63) & ~63ull;
    if (off + bytes > c->up_cap) {
        set_error("upload staging too small");
        return GESMC_E_INTERNAL;
    }
    memcpy(c->h_up + off, src, bytes);
    c->up_used = off + bytes;
    return check_hip(hipMemcpyAsync(dst, c->h_up + off, bytes, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
}

gesmc_status up_end(gesmc_ctx *c, hipStream_t s) {
    GESMC_TRY(check_hip(hipEventRecord(c->up_ev, s), "hipEventRecord"));
    c->up_pending = true;
    return GESMC_OK;
}

// Device room for c->h_chunks (grown if needed; the copy goes through up_copy).
gesmc_status ensure_chunks(gesmc_ctx *c) {
    const uint64_t n = c->h_chunks.size();
    if (n > c->chunk_cap) {
        if (c->chunks) dev_free(c, c->chunks);
        c->chunks = nullptr;
        c->chunk_cap = 0;
        const uint64_t cap = std::max<uint64_t>(n + n / 2, 1024);
        GESMC_TRY(dev_alloc(c, (void **)&c->chunks, cap * sizeof(uint4)));
        c->chunk_cap = cap;
    }
    return GESMC_OK;
}

gesmc_status ensure_batch(gesmc_ctx *c, uint64_t G, uint64_t npos) {
    if (G > c->cap_g) {
        for (void **q : {(void **)&c->gr, (void **)&c->in_off, (void **)&c->rank_of, (void **)&c->gacc,
                         (void **)&c->gerr, (void **)&c->small_list, (void **)&c->rrank}) {
            if (*q) dev_free(c, *q);
            *q = nullptr;
        }
        if (c->h_gacc) (void)hipHostFree(c->h_gacc);
        if (c->h_gerr) (void)hipHostFree(c->h_gerr);
        c->h_gacc = nullptr;
        c->h_gerr = nullptr;
        c->cap_g = 0;
        const uint64_t cap = std::max<uint64_t>(G, 64);
        GESMC_TRY(dev_alloc(c, (void **)&c->gr, cap * sizeof(BatchGraph)));
        GESMC_TRY(dev_alloc(c, (void **)&c->in_off, (cap + 1) * 8));
        GESMC_TRY(dev_alloc(c, (void **)&c->rank_of, cap * 4));
        GESMC_TRY(dev_alloc(c, (void **)&c->gacc, cap * 4 * 8));
        GESMC_TRY(dev_alloc(c, (void **)&c->gerr, cap * 4));
        GESMC_TRY(dev_alloc(c, (void **)&c->small_list, cap * 4));
        GESMC_TRY(dev_alloc(c, (void **)&c->rrank, cap * 4));
        if (hipHostMalloc((void **)&c->h_gacc, cap * 4 * 8, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&c->h_gerr, cap * 4, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipHostMalloc failed");
            return GESMC_E_NOMEM;
        }
        c->cap_g = cap;
    }
    if (npos > c->cap_pos) {
        for (void **q : {(void **)&c->pg, (void **)&c->bk}) {
            if (*q) dev_free(c, *q);
            *q = nullptr;
        }
        c->cap_pos = 0;
        const uint64_t cap = std::max<uint64_t>(npos, 1024);
        GESMC_TRY(dev_alloc(c, (void **)&c->pg, cap * 4));
        GESMC_TRY(dev_alloc(c, (void **)&c->bk, cap * 4));
        c->cap_pos = cap;
    }
    return GESMC_OK;
}

gesmc_status run_batch_impl(gesmc_ctx *c, void *stream, uint32_t G, const uint64_t *d_in, uint64_t *d_out,
                            const uint64_t *offsets, const uint32_t *nv, const uint64_t *seed, const uint32_t *t0v,
                            const uint32_t *rv, uint32_t pl, gesmc_stats *stats, gesmc_stats *total) {
    if (!c) {
        set_error("null context");
        return GESMC_E_INVAL;
    }
    if (G == 0) {
        if (total) memset(total, 0, sizeof(*total));
        return GESMC_OK;
    }
    if (!offsets || !nv || !seed || !rv) {
        set_error("null per-graph array");
        return GESMC_E_INVAL;
    }
    if (G > (1u << kMaxFineBits)) {
        set_error("G = %u exceeds the limit 2^%u", G, kMaxFineBits);
        return GESMC_E_RANGE;
    }
    if (offsets[0] != 0) {
        set_error("offsets[0] must be 0");
        return GESMC_E_INVAL;
    }
    uint64_t vsum = 0;
    for (uint32_t g = 0; g < G; ++g) {
        if (offsets[g + 1] < offsets[g]) {
            set_error("offsets decrease at graph %u", g);
            return GESMC_E_INVAL;
        }
        const uint32_t t0 = t0v ? t0v[g] : 0u;
        if ((uint64_t)t0 + rv[g] > 0x100000000ull) {
            set_error("graph %u: superstep counter t0 + r overflows 32 bits", g);
            return GESMC_E_INVAL;
        }
        vsum += nv[g];
    }
    const uint64_t total_m = offsets[G];
    if (total_m + G >= kMaxEdges) {
        set_error("batch of %llu edges exceeds the limit 2^30 - G", (unsigned long long)total_m);
        return GESMC_E_RANGE;
    }
    if (vsum > 0xFFFFFFFEull) {
        set_error("batch vertex count %llu exceeds 2^32 - 2", (unsigned long long)vsum);
        return GESMC_E_RANGE;
    }
    if (total_m > 0 && (!d_in || !d_out)) {
        set_error("null edge pointer");
        return GESMC_E_INVAL;
    }
    GESMC_TRY(check_hip(hipSetDevice(c->device), "hipSetDevice"));
    if (c->strategy != 0) {
        set_error("batches need the sorted-tuples strategy (GESMC_OPT_STRATEGY 0)");
        return GESMC_E_INVAL;
    }
    hipStream_t s = (hipStream_t)stream;

    // rank order: graphs switched by the multi-kernel supersteps (m >= 2, r >= 1,
    // not small) by r descending, then the small ones (k_small_chain), then the rest
    auto m_of = [&](uint32_t g) { return offsets[g + 1] - offsets[g]; };
    auto r_eff = [&](uint32_t g) { return m_of(g) >= 2 ? rv[g] : 0u; };
    // LDS classes: m <= 4096, or m <= 6144 with vertex ids below 2^16 (compact keys)
    auto is_cmp = [&](uint32_t g) { return m_of(g) > kMidMax && m_of(g) <= kCmpMax && nv[g] <= kCmpMaxN; };
    auto is_small = [&](uint32_t g) {
        return c->small_graphs && r_eff(g) > 0 && (m_of(g) <= kMidMax || is_cmp(g));
    };
    auto r_pipe = [&](uint32_t g) { return is_small(g) ? 0u : r_eff(g); };
    auto rank_class = [&](uint32_t g) { return r_pipe(g) > 0 ? 0 : (is_small(g) ? 1 : 2); };
    std::vector<uint32_t> &order = c->h_order;
    order.resize(G);
    for (uint32_t g = 0; g < G; ++g) order[g] = g;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        const int ca = rank_class(a), cb = rank_class(b);
        return ca != cb ? ca < cb : r_pipe(a) > r_pipe(b);
    });
    std::vector<BatchGraph> &gr = c->h_gr;
    gr.assign(G, BatchGraph{});
    c->h_rank_of.assign(G, 0);
    c->h_small.clear();
    c->h_mid.clear();
    c->h_cmp.clear();
    c->h_rrank.assign(G, 0);
    uint64_t poff = 0, vbase = 0, bbase = 0, nmax = 0, mmax = 0;
    uint32_t nactive = 0, rmax = 0;
    bool need_validation = false;
    for (uint32_t q = 0; q < G; ++q) {
        const uint32_t g = order[q];
        const uint64_t m = m_of(g);
        const bool active = r_pipe(g) > 0;
        c->h_rrank[q] = r_eff(g);
        if (is_small(g)) (m <= kSmallMax ? c->h_small : m <= kMidMax ? c->h_mid : c->h_cmp).push_back(q);
        BatchGraph &b = gr[q];
        b.poff = (uint32_t)poff;
        b.mpad = (uint32_t)(m + (active ? (m & 1) : 0));
        b.goff = (uint32_t)offsets[g];
        b.vbase = (uint32_t)vbase;
        b.k0 = (uint32_t)seed[g];
        b.k1 = (uint32_t)(seed[g] >> 32);
        b.t0 = t0v ? t0v[g] : 0u;
        b.nb = active ? (uint32_t)std::max<uint64_t>(1, ceil_div((uint32_t)b.mpad, c->bucket_avg)) : 0u;
        b.bbase = (uint32_t)bbase;
        b.m = (uint32_t)m;
        b.n = nv[g];
        b.pl = pl;
        c->h_rank_of[g] = q;
        poff += b.mpad;
        vbase += nv[g];
        nmax = std::max<uint64_t>(nmax, nv[g]);
        mmax = std::max<uint64_t>(mmax, b.mpad);
        bbase += b.nb;
        if (active) {
            ++nactive;
            rmax = std::max(rmax, rv[g]);
        } else if (m >= 2 && !is_small(g)) {
            need_validation = true;  // never switched: duplicates are checked up front
        }
    }
    if (bbase > (1ull << kMaxFineBits)) {
        set_error("batch needs %llu permutation buckets (limit 2^%u): raise GESMC_OPT_BUCKET_AVG",
                  (unsigned long long)bbase, kMaxFineBits);
        return GESMC_E_RANGE;
    }
    const uint32_t npos = (uint32_t)poff;
    GESMC_TRY(ensure_capacity(c, npos));
    GESMC_TRY(ensure_counters(c, rmax));
    GESMC_TRY(ensure_batch(c, G, npos));
    c->h_chunks.clear();
    for (uint32_t q = 0; q < G; ++q) add_chunks(c->h_chunks, q, gr[q].poff, gr[q].mpad);
    const uint32_t nchunks = (uint32_t)c->h_chunks.size();
    GESMC_TRY(ensure_chunks(c));
    // uploads through the pinned arena: records, offsets, rank lists, chunks
    const uint64_t up_bytes = G * (sizeof(BatchGraph) + 8 + 4 + 4) + 8 +
                              (c->h_small.size() + c->h_mid.size() + c->h_cmp.size()) * 4ull +
                              (uint64_t)nchunks * sizeof(uint4);
    GESMC_TRY(up_begin(c, up_bytes, 6));
    GESMC_TRY(up_copy(c, s, c->gr, gr.data(), G * sizeof(BatchGraph)));
    GESMC_TRY(up_copy(c, s, c->in_off, offsets, (G + 1) * 8ull));
    const uint32_t nsm1 = (uint32_t)c->h_small.size(), nsm2 = (uint32_t)c->h_mid.size(),
                   nsm3 = (uint32_t)c->h_cmp.size();
    // the m <= 1024 list, then m <= 4096, then the compact class
    c->h_small.insert(c->h_small.end(), c->h_mid.begin(), c->h_mid.end());
    c->h_small.insert(c->h_small.end(), c->h_cmp.begin(), c->h_cmp.end());
    const uint32_t nsmall = nsm1 + nsm2 + nsm3;
    const bool need_acc = stats != nullptr || nsmall > 0;  // small graphs count per graph
    if (nsmall) {
        GESMC_TRY(up_copy(c, s, c->small_list, c->h_small.data(), nsmall * 4ull));
        GESMC_TRY(up_copy(c, s, c->rrank, c->h_rrank.data(), G * 4ull));
    }
    GESMC_TRY(up_copy(c, s, c->rank_of, c->h_rank_of.data(), G * 4ull));
    GESMC_TRY(up_copy(c, s, c->chunks, c->h_chunks.data(), (uint64_t)nchunks * sizeof(uint4)));
    GESMC_TRY(up_end(c, s));
    // The device work of the call.  In graph mode (GESMC_OPT_GRAPH) it is captured
    // into a hipGraph on the second call of a shape and replayed afterwards: the
    // per-call data (seeds, t0, n) live in the per-graph records uploaded above,
    // so a replay may use new seeds.  Uploads, events and result copies stay
    // outside the graph; the first call of a shape runs eagerly, so every
    // buffer is sized before a capture.
    auto device_work = [&]() -> gesmc_status {
        c->tuple_bytes = 0;
        const uint64_t zero_words = 64 + (uint64_t)std::max<uint32_t>(rmax, 1) * (sizeof(StepCounters) / 4);
        GESMC_TRY(launch(c, s, KID_MISC, 0, k_zero_words, dim3(4), dim3(256), 0, c->err, (uint64_t)64));
        GESMC_TRY(launch(c, s, KID_MISC, 0, k_zero_words, dim3(16), dim3(256), 0, (uint32_t *)c->ctr, zero_words - 64));
        if (need_acc)
            GESMC_TRY(launch(c, s, KID_MISC, 0, k_zero_words, dim3(16), dim3(256), 0, (uint32_t *)c->gacc,
                             (uint64_t)G * 8));
        GESMC_TRY(launch(c, s, KID_MISC, 0, k_zero_words, dim3(16), dim3(256), 0, c->gerr, (uint64_t)G));
        const GraphErr ge_all{c->gr, G, c->gerr};
        uint32_t *bad_pos = c->err + 4;
        if (total_m > 0) {
            GESMC_TRY(launch(c, s, KID_LOAD, total_m, k_load_batch, dim3(grid_stride_blocks(c, total_m)), dim3(kBlock), 0,
                             (const unsigned long long *)d_in, (uint32_t)total_m, (const uint64_t *)c->in_off, G,
                             (const uint32_t *)c->rank_of, (const BatchGraph *)c->gr, c->idx[0], c->key[0], c->err,
                             bad_pos, c->gerr));
            GESMC_TRY(launch(c, s, KID_MISC, 0, k_fill_pg, dim3(nchunks), dim3(kBlock), 0, (const uint4 *)c->chunks,
                             c->pg));
        }
        if (need_validation) {
            c->ctr_step = c->ctr;
            GESMC_TRY(launch(c, s, KID_EMIT, npos, k_emit_sources, dim3(grid_stride_blocks(c, npos)), dim3(kBlock), 0,
                             (const unsigned long long *)c->key[0], npos, c->tu_tag[0], c->tu_key[0]));
            GESMC_TRY(partition_and_resolve(c, s, npos, ERR_DUP, ge_all));
        }
        // small graphs: every superstep of each in one workgroup, in LDS.  Each
        // size class runs on a side stream beside the multi-kernel supersteps
        // of the other graphs (their records, counts and error words are
        // disjoint) and is joined back before the unpermute.  A lone class
        // with nothing beside it stays on the call's stream.
        const bool fork = (nsm1 > 0) + (nsm2 + nsm3 > 0) + (nactive > 0) > 1;
        if (fork) GESMC_TRY(check_hip(hipEventRecord(c->fork_ev, s), "hipEventRecord"));
        hipStream_t s1 = s, s2 = s;
        if (fork && nsm1) {
            s1 = c->side[0];
            GESMC_TRY(check_hip(hipStreamWaitEvent(s1, c->fork_ev, 0), "hipStreamWaitEvent"));
        }
        if (fork && nsm2 + nsm3) {
            s2 = c->side[1];
            GESMC_TRY(check_hip(hipStreamWaitEvent(s2, c->fork_ev, 0), "hipStreamWaitEvent"));
        }
        if (nsm1)
            GESMC_TRY(launch(c, s1, KID_SMALL, nsm1, k_small_chain<kSmallMax, kSmallThreads, false>, dim3(nsm1),
                             dim3(kSmallThreads), 0, (const uint32_t *)c->small_list, (const BatchGraph *)c->gr,
                             (const uint32_t *)c->rrank, c->key[0], c->gacc, c->gerr, c->err));
        if (nsm2)
            GESMC_TRY(launch(c, s2, KID_SMALL_MID, nsm2, k_small_chain<kMidMax, kMidThreads, false>, dim3(nsm2),
                             dim3(kMidThreads), 0, (const uint32_t *)c->small_list + nsm1, (const BatchGraph *)c->gr,
                             (const uint32_t *)c->rrank, c->key[0], c->gacc, c->gerr, c->err));
        if (nsm3)  // after the 4096-edge class on the same stream (one workgroup per CU either way)
            GESMC_TRY(launch(c, s2, KID_SMALL_CMP, nsm3, k_small_chain<kCmpMax, kCmpThreads, true>, dim3(nsm3),
                             dim3(kCmpThreads), 0, (const uint32_t *)c->small_list + nsm1 + nsm2,
                             (const BatchGraph *)c->gr, (const uint32_t *)c->rrank, c->key[0], c->gacc, c->gerr,
                             c->err));
        if (s1 != s) GESMC_TRY(check_hip(hipEventRecord(c->join_ev[0], s1), "hipEventRecord"));
        if (s2 != s) GESMC_TRY(check_hip(hipEventRecord(c->join_ev[1], s2), "hipEventRecord"));
        // superstep s switches the ranks [0, active_s): those with r > s
        // (each step after the first takes its first radix level's counts from
        // the previous step's first decision round)
        auto active = [&](uint32_t st, uint32_t q) {
            while (q > 0 && r_pipe(order[q - 1]) <= st) --q;
            return q;
        };
        auto step_plan = [&](uint32_t q) {
            return batch_plan(c, q < G ? gr[q].poff : npos, q < G ? gr[q].bbase : (uint32_t)bbase);
        };
        auto counts_ahead = [&](const Plan &q) { return GESMC_COUNT_AHEAD && q.bbits > 0 && q.b1 > 0 && q.m >= 2; };
        uint32_t qa = nactive;
        bool ready = false;
        for (uint32_t st = 0; st < rmax; ++st) {
            qa = active(st, qa);
            const Plan p = step_plan(qa);
            const uint32_t qn = st + 1 < rmax ? active(st + 1, qa) : 0;
            const Plan pn = step_plan(qn);
            const bool next = qn > 0 && counts_ahead(p) && counts_ahead(pn);
            BatchStep bs{c->gr, qa, st, c->pg, c->bk, stats ? c->gacc : nullptr, ge_all, vbase, nmax, mmax};
            c->ctr_step = c->ctr + st;
            GESMC_TRY(superstep_partitioned(c, s, p, 0u, 0u, 0u, pl, st == 0 ? ERR_DUP : ERR_INTERNAL, &bs, 0, 0,
                                            ready, next, &pn));
            ready = next;
        }
        if (s1 != s) GESMC_TRY(check_hip(hipStreamWaitEvent(s, c->join_ev[0], 0), "hipStreamWaitEvent"));
        if (s2 != s) GESMC_TRY(check_hip(hipStreamWaitEvent(s, c->join_ev[1], 0), "hipStreamWaitEvent"));
        if (total_m > 0)
            GESMC_TRY(launch(c, s, KID_UNPERMUTE, npos, k_unpermute_batch, dim3(grid_stride_blocks(c, npos)), dim3(kBlock),
                             0, (const uint32_t *)c->idx[0], (const unsigned long long *)c->key[0],
                             (const uint32_t *)c->pg, (const BatchGraph *)c->gr, npos, (unsigned long long *)d_out,
                             (const uint32_t *)c->err));
        return GESMC_OK;
    };
    GESMC_TRY(check_hip(hipEventRecord(c->call_a, s), "hipEventRecord"));
    if (c->use_graph && s != nullptr) {
        uint64_t key = 1469598103934665603ull;
        auto mix = [&](uint64_t v) { key = (key ^ v) * 1099511628211ull; };
        mix(G);
        mix((uint64_t)(uintptr_t)d_in);
        mix((uint64_t)(uintptr_t)d_out);
        mix(stats != nullptr);
        mix(pl);
        for (uint32_t g = 0; g <= G; ++g) mix(offsets[g]);
        for (uint32_t g = 0; g < G; ++g) mix(rv[g]);
        mix(c->bucket_avg);
        mix(c->sort_cap);
        mix((uint64_t)c->fast_rounds);
        mix(c->level1_cap);
        mix(c->fuse_emit);
        mix(c->small_graphs);
        mix(c->pack_tuples);
        mix(vbase);  // the tuple layout depends on the vertex id widths (n may change between replays)
        mix(nmax);
        mix((uint64_t)c->persist_mult);
        mix(g_alloc_epoch.load());
        mix((uint64_t)(uintptr_t)s);
        if (c->graph_exec && key == c->graph_key) {
            GESMC_TRY(check_hip(hipGraphLaunch(c->graph_exec, s), "hipGraphLaunch"));
            ++c->graph_replays;
        } else if (key == c->graph_last_key) {
            if (c->graph_exec) {
                (void)hipGraphExecDestroy(c->graph_exec);
                c->graph_exec = nullptr;
            }
            hipGraph_t graph = nullptr;
            c->capturing = true;
            gesmc_status st = check_hip(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal),
                                        "hipStreamBeginCapture");
            if (st == GESMC_OK) {
                st = device_work();
                const hipError_t e = hipStreamEndCapture(s, &graph);
                if (st == GESMC_OK) st = check_hip(e, "hipStreamEndCapture");
            }
            c->capturing = false;
            if (st == GESMC_OK)
                st = check_hip(hipGraphInstantiate(&c->graph_exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
            if (graph) (void)hipGraphDestroy(graph);
            if (st != GESMC_OK) {
                c->graph_exec = nullptr;
                return st;
            }
            c->graph_key = key;
            GESMC_TRY(check_hip(hipGraphLaunch(c->graph_exec, s), "hipGraphLaunch"));
        } else {
            c->graph_last_key = key;
            GESMC_TRY(device_work());
        }
    } else {
        GESMC_TRY(device_work());
    }
    GESMC_TRY(check_hip(hipEventRecord(c->call_b, s), "hipEventRecord"));
    GESMC_TRY(check_hip(hipMemcpyAsync(c->h_err, c->err, 32, hipMemcpyDeviceToHost, s), "hipMemcpyAsync"));
    if (rmax > 0)
        GESMC_TRY(check_hip(hipMemcpyAsync(c->h_ctr, c->ctr, sizeof(StepCounters) * rmax, hipMemcpyDeviceToHost, s),
                            "hipMemcpyAsync"));
    if (need_acc)
        GESMC_TRY(check_hip(hipMemcpyAsync(c->h_gacc, c->gacc, (size_t)G * 32, hipMemcpyDeviceToHost, s),
                            "hipMemcpyAsync"));
    GESMC_TRY(check_hip(hipMemcpyAsync(c->h_gerr, c->gerr, (size_t)G * 4, hipMemcpyDeviceToHost, s),
                        "hipMemcpyAsync"));
    GESMC_TRY(check_hip(hipStreamSynchronize(s), "hipStreamSynchronize"));
    if (c->profile) collect_profile(c);
    const uint32_t e = c->h_err[0];
    if (e) {
        const gesmc_status st = map_err(e);
        const uint32_t bp = c->h_err[4];
        if (bp && (e & (ERR_LOOP | ERR_RANGE))) {
            const uint64_t pos = ~bp;
            const uint32_t g = (uint32_t)(std::upper_bound(offsets, offsets + G + 1, pos) - offsets) - 1;
            set_error("graph %u, edge %llu: %s", g, (unsigned long long)(pos - offsets[g]),
                      st == GESMC_E_RANGE ? "vertex id out of range" : "input is not a simple graph (loop)");
        } else if (e & ERR_DUP) {
            uint32_t g = 0;
            while (g < G && !(c->h_gerr[c->h_rank_of[g]] & ERR_DUP)) ++g;
            if (g < G)
                set_error("graph %u: input is not a simple graph (duplicate edge)", g);
            else
                set_error("a graph of the batch is not simple (duplicate edge)");
        }
        return st;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->call_a, c->call_b) != hipSuccess) {
        (void)hipGetLastError();
        ms = 0.f;
    }
    if (stats) {
        for (uint32_t g = 0; g < G; ++g) {
            const uint32_t q = c->h_rank_of[g];
            gesmc_stats &o = stats[g];
            memset(&o, 0, sizeof(o));
            const uint32_t rg = r_eff(g);
            o.supersteps = rv[g];
            o.attempts = (uint64_t)rg * (m_of(g) / 2);
            o.legal = c->h_gacc[4 * (size_t)q + 0];
            o.rej_loop = c->h_gacc[4 * (size_t)q + 1];
            o.rej_exists = c->h_gacc[4 * (size_t)q + 2];
            o.rej_pl = c->h_gacc[4 * (size_t)q + 3];
            for (uint32_t st = 0; st < r_pipe(g); ++st) {  // rounds of the multi-kernel supersteps
                o.rounds_sum += c->h_ctr[st].rounds;
                o.rounds_max = std::max<uint32_t>(o.rounds_max, (uint32_t)c->h_ctr[st].rounds);
            }
            o.ms_device = ms;
            o.tuple_bytes = r_pipe(g) > 0 ? c->tuple_bytes : 0u;
        }
    }
    if (total) {
        memset(total, 0, sizeof(*total));
        total->supersteps = rmax;
        for (uint32_t g = 0; g < G; ++g) total->attempts += (uint64_t)r_eff(g) * (m_of(g) / 2);
        for (uint32_t st = 0; st < rmax; ++st) {
            const StepCounters &h = c->h_ctr[st];
            total->legal += h.legal;
            total->rej_loop += h.rej_loop;
            total->rej_exists += h.rej_exists;
            total->rej_pl += h.rej_pl;
            total->rounds_sum += h.rounds;
            total->rounds_max = std::max<uint32_t>(total->rounds_max, (uint32_t)h.rounds);
        }
        for (uint32_t q : c->h_small) {  // small graphs count per graph only
            total->legal += c->h_gacc[4 * (size_t)q + 0];
            total->rej_loop += c->h_gacc[4 * (size_t)q + 1];
            total->rej_exists += c->h_gacc[4 * (size_t)q + 2];
            total->rej_pl += c->h_gacc[4 * (size_t)q + 3];
            total->supersteps = std::max(total->supersteps, c->h_rrank[q]);
        }
        total->ms_device = ms;
        total->tuple_bytes = c->tuple_bytes;
    }
    return GESMC_OK;
}

}  // namespace

extern "C" {

const char *gesmc_last_error(void) { return g_last_error; }

gesmc_status gesmc_create(int hip_device, gesmc_ctx **out) {
    if (!out) {
        set_error("null output pointer");
        return GESMC_E_INVAL;
    }
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) {
        (void)hipGetLastError();
        set_error("no HIP device %d", hip_device);
        return GESMC_E_DEVICE;
    }
    GESMC_TRY(check_hip(hipSetDevice(hip_device), "hipSetDevice"));
    gesmc_ctx *c = new gesmc_ctx();
    c->device = hip_device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess) {
        if (prop.multiProcessorCount > 0) c->num_cus = prop.multiProcessorCount;
        char key[128];
        snprintf(key, sizeof(key), "%.32s:%04x:%02x:%02x", prop.gcnArchName, (unsigned)prop.pciDomainID,
                 (unsigned)prop.pciBusID, (unsigned)prop.pciDeviceID);
        c->device_key = key;
    } else {
        (void)hipGetLastError();
        c->device_key = "device" + std::to_string(hip_device);
    }
    // fixed-size area: err[16], ucount[16], coarse offsets / tile map, level-1 segment, fine offsets
    const size_t nf = (size_t)1 << kMaxFineBits;
    const size_t nc = ((size_t)1 << kMaxCoarseBits) + 8;
    const size_t words = 16 + 16 + 2 * nc + 8 + (nf + 8);
    if (dev_alloc(c, (void **)&c->small, words * 4) != GESMC_OK ||
        dev_alloc(c, (void **)&c->ctr, 64 * sizeof(StepCounters)) != GESMC_OK ||
        dev_alloc(c, (void **)&c->bslot, (kEmitSlotsMax + 2 * (size_t)grid_stride_blocks(c, ~0ull >> 1)) * sizeof(uint4)) !=
            GESMC_OK) {
        gesmc_destroy(c);
        return GESMC_E_NOMEM;
    }
    c->ctr_cap = 64;
    uint32_t *w = c->small;
    c->err = w;
    w += 16;
    c->ucount = w;
    w += 16;
    c->coarse_off = w;
    w += nc;
    c->tile_first = w;
    w += nc;
    c->lvl1_seg = w;
    w += 4;
    c->lvl1_tiles = w;
    w += 4;
    c->fine_off = w;
    // kernels whose dynamic LDS can exceed 64 KiB (gfx950 has 160 KiB per CU)
    (void)hipFuncSetAttribute((const void *)k_sort_buckets, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)sort_lds_bytes(kLdsCap));
    set_scatter_lds_limits<kTileSmall>();
    set_scatter_lds_limits<kTileLarge>();
    for (const void *f : {(const void *)k_resolve<false>, (const void *)k_resolve<true>})
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)resolve_lds_bytes(kLdsCap));
    (void)hipGetLastError();
    if (hipMemset(c->small, 0, words * 4) != hipSuccess ||
        hipHostMalloc((void **)&c->h_err, 64, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&c->h_ctr, 64 * sizeof(StepCounters), hipHostMallocDefault) != hipSuccess ||
        hipEventCreate(&c->call_a) != hipSuccess || hipEventCreate(&c->call_b) != hipSuccess ||
        hipStreamCreateWithFlags(&c->side[0], hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&c->side[1], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->join_ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->join_ev[1], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->up_ev, hipEventDisableTiming) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        (void)hipGetLastError();
        set_error("context initialisation failed");
        gesmc_destroy(c);
        return GESMC_E_DEVICE;
    }
    c->h_ctr_cap = 64;
    const gesmc_status sc = noalloc_scratch_ptr(hip_device, nullptr);
    if (sc != GESMC_OK) {
        gesmc_destroy(c);
        return sc;
    }
    *out = c;
    return GESMC_OK;
}

void gesmc_destroy(gesmc_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    free_buffers(c);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->small) dev_free(c, c->small);
    if (c->small_pi) dev_free(c, c->small_pi);
    if (c->bslot) dev_free(c, c->bslot);
    for (void *q : {(void *)c->gr, (void *)c->in_off, (void *)c->rank_of, (void *)c->gacc, (void *)c->pg,
                    (void *)c->bk, (void *)c->gerr, (void *)c->small_list, (void *)c->rrank, (void *)c->chunks})
        if (q) dev_free(c, q);
    if (c->h_gacc) (void)hipHostFree(c->h_gacc);
    if (c->h_gerr) (void)hipHostFree(c->h_gerr);
    if (c->ctr) dev_free(c, c->ctr);
    if (c->h_err) (void)hipHostFree(c->h_err);
    if (c->h_ctr) (void)hipHostFree(c->h_ctr);
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->call_a) (void)hipEventDestroy(c->call_a);
    if (c->call_b) (void)hipEventDestroy(c->call_b);
    if (c->h_up) (void)hipHostFree(c->h_up);
    if (c->h_hr) (void)hipHostFree(c->h_hr);
    for (void *q : {(void *)c->es_E, (void *)c->es_H, (void *)c->es_slot, (void *)c->es_ctr})
        if (q) dev_free(c, q);
    if (c->h_es_ctr) (void)hipHostFree(c->h_es_ctr);
    if (c->hr_dev) dev_free(c, c->hr_dev);
    for (hipEvent_t e : {c->fork_ev, c->join_ev[0], c->join_ev[1], c->up_ev})
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t q : c->side)
        if (q) (void)hipStreamDestroy(q);
    delete c;
}

gesmc_status gesmc_run_batch(gesmc_ctx *ctx, void *stream, uint32_t G, const uint64_t *d_in, uint64_t *d_out,
                             const uint64_t *offsets, const uint32_t *n, const uint64_t *seed, const uint32_t *t0,
                             const uint32_t *r, uint32_t pl, uint32_t flags, gesmc_stats *stats, gesmc_stats *total) {
    if (flags != 0) {
        set_error("flags must be 0");
        return GESMC_E_INVAL;
    }
    return run_batch_impl(ctx, stream, G, d_in, d_out, offsets, n, seed, t0, r, pl, stats, total);
}

}  // extern "C"

namespace {

// Tuning choices per device and shape class: key "device|mode|m|n|g" (the
// device's architecture and PCI address; the form; log2 of the edge count, of
// the largest vertex count and of the graph count).  Shared by every context
// of the process; gesmc_tune_cache_save / _load keep it in a file.
std::mutex g_tune_mu;
std::map<std::string, gesmc_tuning> g_tune;

int log2_class(uint64_t x) {
    int b = 0;
    while (b < 63 && (1ull << (b + 1)) <= x) ++b;
    return b;
}

std::string tune_key(const gesmc_ctx *c, const char *mode, uint64_t m, uint64_t nmax, uint64_t G) {
    char buf[256];
    snprintf(buf, sizeof(buf), "%s|%s|%d|%d|%d", c->device_key.c_str(), mode, log2_class(m), log2_class(nmax),
             log2_class(G));
    return buf;
}

// Times every candidate setting with `trial` (device ms of one call; the
// first call of a setting warms it up, the second is timed) and leaves the
// fastest set.  Candidates: bucket mean 1/2 or 3/4 of the LDS capacity, an
// even level split or an 8-bit first level, fused or unfused tuple pass.
// With the cache on (GESMC_OPT_TUNE_CACHE), a choice already made for this
// device and shape class is set instead, and a new choice is kept.
template <typename Trial>
gesmc_status autotune_impl(gesmc_ctx *c, Trial trial, gesmc_tuning *out, const std::string &key) {
    if (c->strategy != 0) {
        set_error("the autotuner needs the sorted-tuples strategy (GESMC_OPT_STRATEGY 0)");
        return GESMC_E_INVAL;
    }
    if (c->tune_cache) {  // a choice made before for this device and shape class
        std::lock_guard<std::mutex> lk(g_tune_mu);
        const auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            c->bucket_avg = it->second.bucket_avg;
            c->level1_cap = it->second.level1_bits;
            c->fuse_emit = it->second.fuse_emit != 0;
            if (out) {
                *out = it->second;
                out->candidates = 0;  // nothing timed
            }
            return GESMC_OK;
        }
    }
    const uint32_t avgs[2] = {3 * kLdsCap / 4, kLdsCap / 2};
    const uint32_t l1s[2] = {0, 8};
    const bool fuses[2] = {true, false};
    const uint32_t save_avg = c->bucket_avg, save_l1 = c->level1_cap;
    const bool save_fuse = c->fuse_emit, save_prof = c->profile;
    c->profile = false;
    double best = 1e300, dflt = 0;
    uint32_t best_avg = save_avg, best_l1 = save_l1, ncand = 0;
    bool best_fuse = save_fuse;
    gesmc_status st = GESMC_OK;
    for (uint32_t a : avgs)
        for (uint32_t l : l1s)
            for (bool f : fuses) {
                c->bucket_avg = a;
                c->level1_cap = l;
                c->fuse_emit = f;
                double ms = 0;
                st = trial(&ms);  // warm-up
                if (st == GESMC_OK) st = trial(&ms);
                if (st != GESMC_OK) break;
                ++ncand;
                if (a == avgs[0] && l == 0 && f) dflt = ms;
                if (ms < best) {
                    best = ms;
                    best_avg = a;
                    best_l1 = l;
                    best_fuse = f;
                }
            }
    c->profile = save_prof;
    if (st != GESMC_OK) {
        c->bucket_avg = save_avg;
        c->level1_cap = save_l1;
        c->fuse_emit = save_fuse;
        return st;
    }
    c->bucket_avg = best_avg;
    c->level1_cap = best_l1;
    c->fuse_emit = best_fuse;
    const gesmc_tuning t{best_avg, best_l1, best_fuse ? 1u : 0u, ncand, best, dflt};
    if (out) *out = t;
    if (c->tune_cache) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = t;
    }
    return GESMC_OK;
}

}  // namespace

extern "C" {

gesmc_status gesmc_autotune(gesmc_ctx *c, void *stream, const uint64_t *d_in, uint64_t m, uint32_t n, uint64_t seed,
                            uint32_t supersteps, gesmc_tuning *out) {
    if (!c || (m > 0 && !d_in)) {
        set_error("null argument");
        return GESMC_E_INVAL;
    }
    GESMC_TRY(check_hip(hipSetDevice(c->device), "hipSetDevice"));
    uint64_t *tmp = nullptr;
    GESMC_TRY(dev_alloc(c, (void **)&tmp, std::max<uint64_t>(m, 1) * 8));
    const gesmc_status st = autotune_impl(
        c,
        [&](double *ms) {
            gesmc_stats stt{};
            const gesmc_status s = run_impl(c, stream, d_in, tmp, m, n, seed, 0, std::max(supersteps, 1u), 0, &stt,
                                            nullptr, nullptr);
            *ms = stt.ms_device;
            return s;
        },
        out, tune_key(c, "plain", m, n, 1));
    (void)hipStreamSynchronize((hipStream_t)stream);
    dev_free(c, tmp);
    return st;
}

gesmc_status gesmc_autotune_batch(gesmc_ctx *c, void *stream, uint32_t G, const uint64_t *d_in,
                                  const uint64_t *offsets, const uint32_t *n, const uint64_t *seed,
                                  uint32_t supersteps, gesmc_tuning *out) {
    if (!c || !offsets || G == 0) {
        set_error("null argument");
        return GESMC_E_INVAL;
    }
    GESMC_TRY(check_hip(hipSetDevice(c->device), "hipSetDevice"));
    const uint64_t total = offsets[G];
    uint64_t *tmp = nullptr;
    GESMC_TRY(dev_alloc(c, (void **)&tmp, std::max<uint64_t>(total, 1) * 8));
    std::vector<uint32_t> rs(G, std::max(supersteps, 1u));
    const gesmc_status st = autotune_impl(
        c,
        [&](double *ms) {
            gesmc_stats tot{};
            const gesmc_status s = run_batch_impl(c, stream, G, d_in, tmp, offsets, n, seed, nullptr, rs.data(), 0,
                                                  nullptr, &tot);
            *ms = tot.ms_device;
            return s;
        },
        out, tune_key(c, "batch", total, n ? *std::max_element(n, n + G) : 0, G));
    (void)hipStreamSynchronize((hipStream_t)stream);
    dev_free(c, tmp);
    return st;
}

gesmc_status gesmc_run(gesmc_ctx *ctx, void *stream, const uint64_t *d_in, uint64_t *d_out, uint64_t m, uint32_t n,
                       uint64_t seed, uint32_t t0, uint32_t r, uint32_t pl, uint32_t flags, gesmc_stats *stats,
                       gesmc_step_stats *steps) {
    if (flags != 0) {
        set_error("flags must be 0");
        return GESMC_E_INVAL;
    }
    return run_impl(ctx, stream, d_in, d_out, m, n, seed, t0, r, pl, stats, steps, nullptr);
}

gesmc_status gesmc_run_class(gesmc_ctx *ctx, void *stream, const uint64_t *d_in, uint64_t *d_out, uint64_t m,
                             uint32_t n, uint64_t seed, uint32_t t0, uint32_t r, uint32_t pl, uint32_t cls,
                             gesmc_stats *stats, gesmc_step_stats *steps, uint8_t *d_outcome) {
    return run_impl(ctx, stream, d_in, d_out, m, n, seed, t0, r, pl, stats, steps, d_outcome, cls);
}

gesmc_status gesmc_run_host(gesmc_ctx *c, const uint32_t *uv, uint32_t *uv_out, uint64_t m, uint32_t n,
                            uint64_t seed, uint32_t t0, uint32_t r, uint32_t pl, uint32_t flags, gesmc_stats *stats) {
    if (!c || (m > 0 && (!uv || !uv_out))) {
        set_error("null argument");
        return GESMC_E_INVAL;
    }
    if (flags != 0) {
        set_error("flags must be 0");
        return GESMC_E_INVAL;
    }
    if (m >= kMaxEdges) {
        set_error("m = %llu exceeds the limit 2^30 - 1", (unsigned long long)m);
        return GESMC_E_RANGE;
    }
    GESMC_TRY(check_hip(hipSetDevice(c->device), "hipSetDevice"));
    const uint64_t words = std::max<uint64_t>(m, 1);
    if (words > c->hr_cap) {
        if (c->hr_dev) dev_free(c, c->hr_dev);
        c->hr_dev = nullptr;
        c->hr_cap = 0;
        GESMC_TRY(dev_alloc(c, (void **)&c->hr_dev, 2 * words * 8));
        c->hr_cap = words;
    }
    if (words > c->h_hr_cap) {
        if (c->h_hr) (void)hipHostFree(c->h_hr);
        c->h_hr = nullptr;
        c->h_hr_cap = 0;
        if (hipHostMalloc((void **)&c->h_hr, words * 8, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipHostMalloc of %llu bytes failed", (unsigned long long)(words * 8));
            return GESMC_E_NOMEM;
        }
        c->h_hr_cap = words;
    }
    uint64_t *d_in = c->hr_dev, *d_out = c->hr_dev + c->hr_cap;
    for (uint64_t i = 0; i < m; ++i) c->h_hr[i] = ((uint64_t)uv[2 * i] << 32) | uv[2 * i + 1];
    hipStream_t s = nullptr;
    gesmc_status st = check_hip(hipMemcpyAsync(d_in, c->h_hr, m * 8, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    if (st == GESMC_OK) st = run_impl(c, s, d_in, d_out, m, n, seed, t0, r, pl, stats, nullptr, nullptr);
    if (st == GESMC_OK)
        st = check_hip(hipMemcpyAsync(c->h_hr, d_out, m * 8, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    const gesmc_status sy = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");  // staging free again
    if (st != GESMC_OK) return st;
    if (sy != GESMC_OK) return sy;
    for (uint64_t i = 0; i < m; ++i) {
        uv_out[2 * i] = (uint32_t)(c->h_hr[i] >> 32);
        uv_out[2 * i + 1] = (uint32_t)c->h_hr[i];
    }
    return GESMC_OK;
}

gesmc_status gesmc_run_noalloc(gesmc_ctx *ctx, void *stream, const uint64_t *d_in, uint64_t *d_out, uint64_t m,
                               uint32_t n, uint64_t seed, uint32_t t0, uint32_t r, uint32_t pl, uint32_t flags,
                               gesmc_stats *stats) {
    if (flags != 0) {
        set_error("flags must be 0");
        return GESMC_E_INVAL;
    }
    return run_noalloc_impl(ctx, stream, d_in, d_out, m, n, seed, t0, r, pl, stats);
}

gesmc_status gesmc_superstep_outcomes(gesmc_ctx *ctx, void *stream, const uint64_t *d_in, uint64_t *d_out, uint64_t m,
                                      uint32_t n, uint64_t seed, uint32_t t, uint32_t pl, uint8_t *d_outcome,
                                      gesmc_step_stats *step) {
    if (m >= 2 && !d_outcome) {
        set_error("null outcome pointer");
        return GESMC_E_INVAL;
    }
    return run_impl(ctx, stream, d_in, d_out, m, n, seed, t, 1, pl, nullptr, step, d_outcome);
}

gesmc_status gesmc_perm_keys(gesmc_ctx *c, void *stream, uint64_t m, uint64_t seed, uint32_t t, uint64_t *d_keys) {
    if (!c || (m > 0 && !d_keys)) {
        set_error("null argument");
        return GESMC_E_INVAL;
    }
    if (m >= kMaxEdges) {
        set_error("m too large");
        return GESMC_E_RANGE;
    }
    GESMC_TRY(check_hip(hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    if (m > 0)
        GESMC_TRY(launch(c, s, KID_MISC, m, k_perm_keys, dim3(ceil_div(m, kBlock)), dim3(kBlock), 0, (uint32_t)m, t,
                         (uint32_t)seed, (uint32_t)(seed >> 32), (unsigned long long *)d_keys));
    GESMC_TRY(check_hip(hipStreamSynchronize(s), "hipStreamSynchronize"));
    if (c->profile) collect_profile(c);
    return GESMC_OK;
}

gesmc_status gesmc_permutation(gesmc_ctx *c, void *stream, uint64_t m64, uint64_t seed, uint32_t t, uint32_t *d_pi) {
    if (!c || (m64 > 0 && !d_pi)) {
        set_error("null argument");
        return GESMC_E_INVAL;
    }
    if (m64 >= kMaxEdges) {
        set_error("m too large");
        return GESMC_E_RANGE;
    }
    GESMC_TRY(check_hip(hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    const uint32_t m = (uint32_t)m64;
    if (m > 0) {
        GESMC_TRY(ensure_capacity(c, m));
        GESMC_TRY(ensure_counters(c, 1));
        c->ctr_step = c->ctr;
        GESMC_TRY(launch(c, s, KID_MISC, 0, k_zero_words, dim3(4), dim3(256), 0, c->err, (uint64_t)64));
        GESMC_TRY(launch(c, s, KID_MISC, 0, k_identity_records, dim3(ceil_div(m, kBlock)), dim3(kBlock), 0,
                         c->idx[0], c->key[0], m));
        Plan p = make_plan(c, m);
        p.dig_in_key = digit_in_key(p, 0);  // the records' keys are their indices (top byte zero)
        int sorted = 0;
        GESMC_TRY(permute(c, s, p, t, (uint32_t)seed, (uint32_t)(seed >> 32), 0, &sorted, false));
        GESMC_TRY(launch(c, s, KID_MISC, 0, k_extract_pi, dim3(ceil_div(m, kBlock)), dim3(kBlock), 0,
                         c->idx[sorted], m, d_pi));
        GESMC_TRY(check_hip(hipMemcpyAsync(c->h_err, c->err, 4, hipMemcpyDeviceToHost, s), "hipMemcpyAsync"));
    }
    GESMC_TRY(check_hip(hipStreamSynchronize(s), "hipStreamSynchronize"));
    if (c->profile) collect_profile(c);
    if (m > 0) return map_err(*c->h_err);
    return GESMC_OK;
}

gesmc_status gesmc_tune_cache_save(const char *path) {
    if (!path) {
        set_error("null path");
        return GESMC_E_INVAL;
    }
    FILE *f = fopen(path, "w");
    if (!f) {
        set_error("cannot write %s", path);
        return GESMC_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    fprintf(f, "[\n");
    size_t i = 0;
    for (const auto &kv : g_tune) {
        const gesmc_tuning &t = kv.second;
        fprintf(f,
                "{\"key\": \"%s\", \"bucket_avg\": %u, \"level1_bits\": %u, \"fuse_emit\": %u, \"candidates\": %u, "
                "\"best_ms\": %.6f, \"default_ms\": %.6f}%s\n",
                kv.first.c_str(), t.bucket_avg, t.level1_bits, t.fuse_emit, t.candidates, t.best_ms, t.default_ms,
                ++i < g_tune.size() ? "," : "");
    }
    fprintf(f, "]\n");
    const bool ok = fclose(f) == 0;
    if (!ok) {
        set_error("cannot write %s", path);
        return GESMC_E_INVAL;
    }
    return GESMC_OK;
}

gesmc_status gesmc_tune_cache_load(const char *path) {
    if (!path) {
        set_error("null path");
        return GESMC_E_INVAL;
    }
    FILE *f = fopen(path, "r");
    if (!f) {
        set_error("cannot read %s", path);
        return GESMC_E_INVAL;
    }
    std::map<std::string, gesmc_tuning> got;
    char line[1024];
    bool bad = false;
    while (fgets(line, sizeof(line), f)) {
        if (line[0] != '{') continue;  // "[" and "]"
        char key[256];
        gesmc_tuning t{};
        if (sscanf(line,
                   "{\"key\": \"%255[^\"]\", \"bucket_avg\": %u, \"level1_bits\": %u, \"fuse_emit\": %u, "
                   "\"candidates\": %u, \"best_ms\": %lf, \"default_ms\": %lf}",
                   key, &t.bucket_avg, &t.level1_bits, &t.fuse_emit, &t.candidates, &t.best_ms, &t.default_ms) != 7 ||
            t.bucket_avg < 64 || t.bucket_avg > kLdsCap || t.level1_bits > kMaxCoarseBits || t.fuse_emit > 1) {
            bad = true;
            break;
        }
        got[key] = t;
    }
    fclose(f);
    if (bad) {
        set_error("%s is not a tuning cache written by gesmc_tune_cache_save", path);
        return GESMC_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto &kv : got) g_tune[kv.first] = kv.second;
    return GESMC_OK;
}

void gesmc_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
}

uint32_t gesmc_tune_cache_size(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return (uint32_t)g_tune.size();
}

gesmc_status gesmc_set_allocator(gesmc_ctx *c, gesmc_alloc_fn alloc, gesmc_free_fn free_fn, void *user) {
    if (!c || (alloc == nullptr) != (free_fn == nullptr)) {
        set_error("null context, or only one of the allocate and free functions given");
        return GESMC_E_INVAL;
    }
    if (c->serving) {
        set_error("the context serves a gesmc_server; destroy the server first");
        return GESMC_E_INVAL;
    }
    c->alloc_fn = alloc;
    c->free_fn = free_fn;
    c->alloc_user = user;
    return GESMC_OK;
}

gesmc_status gesmc_set_option(gesmc_ctx *c, int option, int64_t v) {
    if (!c) {
        set_error("null context");
        return GESMC_E_INVAL;
    }
    switch (option) {
        case GESMC_OPT_BUCKET_AVG:
            if (v < 64 || v > (int64_t)(3 * kLdsCap / 4)) break;
            c->bucket_avg = (uint32_t)v;
            return GESMC_OK;
        case GESMC_OPT_SORT_CAP:
            if (v < 64 || v > (int64_t)kLdsCap) break;
            c->sort_cap = (uint32_t)v;
            return GESMC_OK;
        case GESMC_OPT_FAST_ROUNDS:
            if (v < 0 || v > 64) break;
            c->fast_rounds = (int)v;
            c->fast_rounds_auto = false;
            return GESMC_OK;
        case GESMC_OPT_PROFILE:
            c->profile = v != 0;
            return GESMC_OK;
        case GESMC_OPT_ROUND_LIMIT:
            if (v < 0 || v > 0xFFFFFFFFll) break;
            c->round_limit = (uint32_t)v;
            return GESMC_OK;
        case GESMC_OPT_SMALL_GRAPHS:
            if (v < 0 || v > 1) break;
            c->small_graphs = v != 0;
            return GESMC_OK;
        case GESMC_OPT_UNPERMUTE_BUCKETS:
            if (v < 0 || v > 1) break;
            c->unpermute_buckets = v != 0;
            return GESMC_OK;
        case GESMC_OPT_TUNE_CACHE:
            if (v < 0 || v > 1) break;
            c->tune_cache = v != 0;
            return GESMC_OK;
        case GESMC_OPT_PACK_TUPLES:
            if (v < 0 || v > 2) break;
            c->pack_tuples = (int)v;
            return GESMC_OK;
        case GESMC_OPT_GRAPH:
            if (v < 0 || v > 1) break;
            c->use_graph = v != 0;
            if (!c->use_graph && c->graph_exec) {
                (void)hipGraphExecDestroy(c->graph_exec);
                c->graph_exec = nullptr;
            }
            c->graph_key = c->graph_last_key = 0;
            return GESMC_OK;
        case GESMC_OPT_FUSE_EMIT:
            if (v < 0 || v > 1) break;
            c->fuse_emit = v != 0;
            return GESMC_OK;
        case GESMC_OPT_LEVEL1_BITS:
            if (v < 0 || v > (int64_t)kMaxCoarseBits) break;
            c->level1_cap = (uint32_t)v;
            return GESMC_OK;
        case GESMC_OPT_PROFILE_ONLY:
            if (v < -1 || v >= KID_COUNT) break;
            c->profile_only = (int)v;
            return GESMC_OK;
        case GESMC_OPT_PERSIST:
            if (v < 0 || v > 64) break;
            c->persist_mult = (int)v;
            return GESMC_OK;
        case GESMC_OPT_STRATEGY:
            if (v < 0 || v > 1) break;
            if (c->strategy != (int)v) {
                (void)hipDeviceSynchronize();
                free_buffers(c);  // buffers differ per strategy; reallocated on the next call
            }
            c->strategy = (int)v;
            return GESMC_OK;
        default:
            set_error("unknown option %d", option);
            return GESMC_E_INVAL;
    }
    set_error("value %lld out of range for option %d", (long long)v, option);
    return GESMC_E_INVAL;
}

int gesmc_kernel_count(void) { return KID_COUNT; }

const char *gesmc_kernel_name(int id) { return (id >= 0 && id < KID_COUNT) ? kKernelNames[id] : ""; }

gesmc_status gesmc_profile_get(gesmc_ctx *c, int id, double *ms, uint64_t *launches, uint64_t *items) {
    if (!c || id < 0 || id >= KID_COUNT) {
        set_error("bad context or kernel id");
        return GESMC_E_INVAL;
    }
    if (ms) *ms = c->prof_ms[id];
    if (launches) *launches = c->prof_launch[id];
    if (items) *items = c->prof_items[id];
    return GESMC_OK;
}

gesmc_status gesmc_profile_reset(gesmc_ctx *c) {
    if (!c) {
        set_error("null context");
        return GESMC_E_INVAL;
    }
    for (int q = 0; q < KID_COUNT; ++q) {
        c->prof_ms[q] = 0;
        c->prof_launch[q] = 0;
        c->prof_items[q] = 0;
    }
    return GESMC_OK;
}

}  // extern "C"

#include "server_runtime.h"
#include "es_runtime.h"
#include "mixing_runtime.h"
#include "gen_runtime.h"

// ORACLE -- test infrastructure only.
//
// A plain, sequential CPU implementation of the Global Edge Switching Markov
// Chain (G-ES-MC) of Allendorf, Meyer, Penschuck and Tran, "Parallel Global
// Edge Switching for the Uniform Sampling of Simple Graphs with Prescribed
// Degrees" (arXiv 2111.03005).  It exists to check the HIP path: only the
// tests, the smoke check and the benchmark's CPU-baseline leg may load it.
// It shares no code with the HIP library.
//
// What it computes, step by step, in the paper's order:
//   * Def. 2.1 (edge switch): sigma = (i, j, g); e1 = E[i], e2 = E[j];
//     (e3, e4) = tau(e1, e2, g) with tau((u,v),(x,y),0) = ((u,x),(v,y)) and
//     tau((u,v),(x,y),1) = ((u,y),(v,x)); reject if e3 or e4 is a loop or is
//     already an edge, else E[i] <- e3, E[j] <- e4.  Edges are read in their
//     canonical orientation (min, max) (Sec. 2.1 notation).
//   * Def. 3.2 (global switch): a permutation pi of the m edge indices; the
//     k-th switch (0-based) is (pi[2k], pi[2k+1], g_k) with
//     g_k = [pi[2k] < pi[2k+1]]; the switches run one after another.
//   * Sec. 3 (P_L): each switch is independently skipped with probability
//     P_L = pl / 2^32 (pl = 0: every one of the floor(m/2) switches runs).
//   * Alg. 3 (ParGlobalES driver): r global switches in a row.
//
// Random choices (the paper uses MT19937-64 + Lemire, Sec. 5.3; that is not
// reproducible across implementations).  Here they are fixed by the
// counter-based Philox4x32-10 generator of Salmon, Moraes, Dror and Shaw
// ("Parallel random numbers: as easy as 1, 2, 3", SC'11):
//   K_i   = (x0 << 32) | x1 of Philox(ctr = (i, 0, t, 0), key = (seed_lo, seed_hi))
//   pi    = the edge indices sorted ascending by (K_i, i)
//   P_L   : switch k of superstep t is skipped iff
//           x0 of Philox(ctr = (k, 0, t, 1), key) < pl.
// A uniform random key per element, sorted, is a uniform random permutation
// (up to key ties, broken by index) -- the random-keys permutation the
// paper's parallel shuffling builds on (Sec. 5.3).
//
// ES-MC (Def. 2.1, the chain that Alg. 2, ParES, parallelises): r edge
// switches in sequence, switch k (a 64-bit counter, k0 .. k0+r-1) drawn as
//   (x0, x1, x2, x3) = Philox(ctr = (k_lo, k_hi, 0, 2), key = (seed_lo, seed_hi))
//   i = floor(((x0 << 32) | x1) * m / 2^64)            uniform on [0, m)
//   j' = floor(((x2 << 32) | x3) * (m - 1) / 2^64),  j = j' + [j' >= i]
//                                                       uniform on [0, m) \ {i}
//   g = x1 & 1
// (i != j as Alg. 2 samples them; the biases of the 64-bit products are
// below m / 2^64).  Tags 0 and 1 of the Philox counter are the permutation
// and P_L draws of G-ES-MC, so the streams never meet.
#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <unordered_map>
#include <unordered_set>
#include <utility>
#include <vector>

namespace {

// ---- Philox4x32-10 (SC'11): Weyl key schedule, 10 rounds ------------------
const uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
const uint32_t kWeyl0 = 0x9E3779B9u, kWeyl1 = 0xBB67AE85u;

void philox10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += kWeyl0;
            k1 += kWeyl1;
        }
        uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
        uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

uint64_t perm_key(uint64_t seed, uint32_t t, uint64_t i) {
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), t, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    philox10(ctr, key, x);
    return ((uint64_t)x[0] << 32) | x[1];
}

bool pl_skip(uint64_t seed, uint32_t t, uint64_t k, uint32_t pl) {
    if (pl == 0) return false;
    uint32_t ctr[4] = {(uint32_t)k, (uint32_t)(k >> 32), t, 1u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    philox10(ctr, key, x);
    return x[0] < pl;
}

// ---- edge keys: (min << 32) | max (Sec. 5.1 packing, smaller node first) ---
inline uint32_t key_u(uint64_t e) { return (uint32_t)(e >> 32); }
inline uint32_t key_v(uint64_t e) { return (uint32_t)e; }
inline uint64_t make_key(uint32_t a, uint32_t b) {
    return a < b ? (((uint64_t)a << 32) | b) : (((uint64_t)b << 32) | a);
}

// ---- the edge set: plain linear-probing hash set with tombstones ----------
// Sentinels are non-canonical words (a loop at vertex 0xFFFFFFFF), which no
// valid edge key can equal.
class EdgeSet {
   public:
    static constexpr uint64_t kEmpty = ~0ull;
    static constexpr uint64_t kTomb = ~0ull - 1;

    explicit EdgeSet(size_t expected) { reset(expected); }

    void reset(size_t expected) {
        size_t cap = 16;
        while (cap < 2 * expected + 16) cap <<= 1;
        slots_.assign(cap, kEmpty);
        used_ = 0;
        live_ = 0;
    }
    bool contains(uint64_t k) const {
        size_t mask = slots_.size() - 1;
        for (size_t s = mix(k) & mask;; s = (s + 1) & mask) {
            if (slots_[s] == k) return true;
            if (slots_[s] == kEmpty) return false;
        }
    }
    // returns false if k was already present
    bool insert(uint64_t k) {
        if (contains(k)) return false;
        if (2 * (used_ + 1) > slots_.size()) {
            // too many used slots (live + tombstones): rebuild with live load <= 1/4
            size_t cap = slots_.size();
            while (4 * (live_ + 1) > cap) cap <<= 1;
            rehash(cap);
        }
        size_t mask = slots_.size() - 1;
        for (size_t s = mix(k) & mask;; s = (s + 1) & mask) {
            if (slots_[s] == kEmpty || slots_[s] == kTomb) {
                if (slots_[s] == kEmpty) ++used_;
                slots_[s] = k;
                ++live_;
                return true;
            }
        }
    }
    bool erase(uint64_t k) {
        size_t mask = slots_.size() - 1;
        for (size_t s = mix(k) & mask;; s = (s + 1) & mask) {
            if (slots_[s] == k) {
                slots_[s] = kTomb;
                --live_;
                return true;
            }
            if (slots_[s] == kEmpty) return false;
        }
    }
    size_t size() const { return live_; }

   private:
    static size_t mix(uint64_t x) {
        x ^= x >> 33;
        x *= 0xff51afd7ed558ccdull;
        x ^= x >> 33;
        x *= 0xc4ceb9fe1a85ec53ull;
        x ^= x >> 33;
        return (size_t)x;
    }
    void rehash(size_t cap) {
        std::vector<uint64_t> old;
        old.swap(slots_);
        slots_.assign(cap, kEmpty);
        used_ = 0;
        live_ = 0;
        for (uint64_t k : old)
            if (k != kEmpty && k != kTomb) insert(k);
    }
    std::vector<uint64_t> slots_;
    size_t used_, live_;
};

}  // namespace

extern "C" {

// Outcome codes of one edge switch.
enum { OR_LEGAL = 1, OR_LOOP = 2, OR_EXISTS = 3, OR_PL = 4 };

// Planted mistakes, for tests that show a pin catches them.  0 = the method.
enum {
    MUT_FLIP_G = 1,         // g_k = [pi[2k] > pi[2k+1]]
    MUT_NO_LOOP = 2,        // loops not rejected
    MUT_NO_EXISTS = 4,      // existing targets not rejected
    MUT_TAU_SWAP = 8,       // tau cases for g = 0 and g = 1 exchanged
    MUT_WRITE_SWAP = 16,    // E[i] <- e4, E[j] <- e3
    MUT_NO_ERASE = 32,      // sources not removed from the edge set
    MUT_PAIR_SHIFT = 64,    // switch k uses (pi[2k+1], pi[2k+2 mod m])
    MUT_KEY_SWAP = 128,     // K_i built as (x1 << 32) | x0
};

struct oracle_counts {
    uint64_t attempts, legal, rej_loop, rej_exists, rej_pl;
};

void oracle_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out) { philox10(ctr, key, out); }

uint64_t oracle_perm_key(uint64_t seed, uint32_t t, uint64_t i) { return perm_key(seed, t, i); }

void oracle_perm_keys(uint64_t seed, uint32_t t, uint64_t m, uint64_t *out) {
    for (uint64_t i = 0; i < m; ++i) out[i] = perm_key(seed, t, i);
}

int oracle_pl_skip(uint64_t seed, uint32_t t, uint64_t k, uint32_t pl) { return pl_skip(seed, t, k, pl) ? 1 : 0; }

// pi of superstep t (Def. 3.2): indices sorted ascending by (K_i, i).
void oracle_permutation_mut(uint64_t m, uint64_t seed, uint32_t t, uint32_t *pi, uint32_t mutate) {
    std::vector<std::pair<uint64_t, uint32_t>> v(m);
    for (uint64_t i = 0; i < m; ++i) {
        uint64_t k = perm_key(seed, t, i);
        if (mutate & MUT_KEY_SWAP) k = (k << 32) | (k >> 32);
        v[i] = {k, (uint32_t)i};
    }
    std::sort(v.begin(), v.end());
    for (uint64_t r = 0; r < m; ++r) pi[r] = v[r].second;
}

void oracle_permutation(uint64_t m, uint64_t seed, uint32_t t, uint32_t *pi) { oracle_permutation_mut(m, seed, t, pi, 0); }

// One edge switch of Def. 2.1 on edge list E and its edge set S.
static int edge_switch(uint64_t *E, EdgeSet &S, uint64_t i, uint64_t j, int g, uint32_t mutate) {
    uint64_t e1 = E[i], e2 = E[j];
    uint32_t u = key_u(e1), v = key_v(e1), x = key_u(e2), y = key_v(e2);
    int tau_case = (mutate & MUT_TAU_SWAP) ? !g : g;
    uint32_t a0, a1, b0, b1;
    if (tau_case == 0) {
        a0 = u; a1 = x; b0 = v; b1 = y;
    } else {
        a0 = u; a1 = y; b0 = v; b1 = x;
    }
    if (!(mutate & MUT_NO_LOOP) && (a0 == a1 || b0 == b1)) return OR_LOOP;
    uint64_t e3 = make_key(a0, a1), e4 = make_key(b0, b1);
    if (!(mutate & MUT_NO_EXISTS) && (S.contains(e3) || S.contains(e4))) return OR_EXISTS;
    if (!(mutate & MUT_NO_ERASE)) {
        S.erase(e1);
        S.erase(e2);
    }
    S.insert(e3);
    S.insert(e4);
    if (mutate & MUT_WRITE_SWAP) {
        E[i] = e4;
        E[j] = e3;
    } else {
        E[i] = e3;
        E[j] = e4;
    }
    return OR_LEGAL;
}

// One global switch (Def. 3.2) with an explicit pi and an explicit P_L skip
// mask (skip[k] != 0: switch k is skipped).  outcome[k] (nullable) receives
// the outcome code of switch k.  E is updated in place.
static void global_switch(uint64_t *E, uint64_t m, EdgeSet &S, const uint32_t *pi, const uint8_t *skip,
                          uint8_t *outcome, oracle_counts *c, uint32_t mutate) {
    uint64_t ell = m / 2;
    for (uint64_t k = 0; k < ell; ++k) {
        uint64_t i = pi[2 * k], j = pi[2 * k + 1];
        if (mutate & MUT_PAIR_SHIFT) {
            i = pi[2 * k + 1];
            j = pi[(2 * k + 2) % m];
        }
        int oc;
        if (skip && skip[k]) {
            oc = OR_PL;
        } else {
            int g = (mutate & MUT_FLIP_G) ? (i > j) : (i < j);
            oc = edge_switch(E, S, i, j, g, mutate);
        }
        if (outcome) outcome[k] = (uint8_t)oc;
        if (c) {
            c->attempts++;
            if (oc == OR_LEGAL) c->legal++;
            if (oc == OR_LOOP) c->rej_loop++;
            if (oc == OR_EXISTS) c->rej_exists++;
            if (oc == OR_PL) c->rej_pl++;
        }
    }
}

// ---- ES-MC (Def. 2.1; the sequential chain of Alg. 2) -------------------
static uint64_t mulhi64(uint64_t a, uint64_t b) { return (uint64_t)(((unsigned __int128)a * b) >> 64); }

// Planted mistakes of the ES-MC draws (for the pin tests).
enum {
    MUT_ES_J_ANY = 1u << 16,    // j drawn from all of [0, m) (may equal i)
    MUT_ES_G_HIGH = 1u << 17,   // g taken from bit 0 of x0 instead of x1
    MUT_ES_NO_SKIP = 1u << 18,  // j = j' (no skip of i): j never reaches m - 1
};

static void es_draw(uint64_t seed, uint64_t k, uint64_t m, uint32_t mutate, uint64_t *i, uint64_t *j, int *g) {
    uint32_t ctr[4] = {(uint32_t)k, (uint32_t)(k >> 32), 0u, 2u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    philox10(ctr, key, x);
    const uint64_t w0 = ((uint64_t)x[0] << 32) | x[1], w1 = ((uint64_t)x[2] << 32) | x[3];
    *i = mulhi64(w0, m);
    if (mutate & MUT_ES_J_ANY) {
        *j = mulhi64(w1, m);
    } else {
        const uint64_t jp = mulhi64(w1, m - 1);
        *j = (mutate & MUT_ES_NO_SKIP) ? jp : jp + (jp >= *i ? 1 : 0);
    }
    *g = (mutate & MUT_ES_G_HIGH) ? (int)(x[0] & 1u) : (int)(x[1] & 1u);
}

// Checks that E is a simple graph on [0, n): every key has min < max < n.
// Returns 0 if simple, -2 for a loop or duplicate, -3 for an id out of range.
int oracle_validate(const uint64_t *E, uint64_t m, uint32_t n) {
    EdgeSet S(m);
    for (uint64_t e = 0; e < m; ++e) {
        uint32_t a = key_u(E[e]), b = key_v(E[e]);
        if (a == b) return -2;
        if (a >= n || b >= n || a == 0xFFFFFFFFu || b == 0xFFFFFFFFu) return -3;
        if (!S.insert(make_key(a, b))) return -2;
    }
    return 0;
}

// Global switch with explicit pi / skip mask (for exhaustive tests).
int oracle_global_switch(uint64_t *E, uint64_t m, const uint32_t *pi, const uint8_t *skip, uint8_t *outcome,
                         oracle_counts *c, uint32_t mutate) {
    EdgeSet S(m);
    for (uint64_t e = 0; e < m; ++e) S.insert(E[e]);
    global_switch(E, m, S, pi, skip, outcome, c, mutate);
    return 0;
}

// Alg. 3 sequentially: r global switches t = t0 .. t0+r-1 on E (canonical
// keys, validated first; a non-canonical key (max, min) is rewritten as
// (min, max)).  per_step (nullable) receives r count records; last_outcome
// (nullable, floor(m/2) bytes) the outcome codes of the last superstep.
// Returns 0, or the validation error code (E untouched).
int oracle_run(uint64_t *E, uint64_t m, uint32_t n, uint64_t seed, uint32_t t0, uint32_t r, uint32_t pl,
               oracle_counts *per_step, uint8_t *last_outcome, uint32_t mutate) {
    int rc = oracle_validate(E, m, n);
    if (rc) return rc;
    for (uint64_t e = 0; e < m; ++e) E[e] = make_key(key_u(E[e]), key_v(E[e]));
    if (per_step) memset(per_step, 0, sizeof(oracle_counts) * r);
    if (m < 2) return 0;
    EdgeSet S(m);
    for (uint64_t e = 0; e < m; ++e) S.insert(E[e]);
    std::vector<uint32_t> pi(m);
    std::vector<uint8_t> skip(m / 2);
    for (uint32_t s = 0; s < r; ++s) {
        uint32_t t = t0 + s;
        oracle_permutation_mut(m, seed, t, pi.data(), mutate);
        for (uint64_t k = 0; k < m / 2; ++k) skip[k] = pl_skip(seed, t, k, pl) ? 1 : 0;
        global_switch(E, m, S, pi.data(), skip.data(), (s + 1 == r) ? last_outcome : nullptr,
                      per_step ? &per_step[s] : nullptr, mutate);
    }
    return 0;
}

// The draws (i, j, g) of ES-MC switches k0 .. k0+count-1 on m edges.
void oracle_es_draws(uint64_t seed, uint64_t k0, uint64_t count, uint64_t m, uint64_t *i, uint64_t *j, uint8_t *g,
                     uint32_t mutate) {
    for (uint64_t q = 0; q < count; ++q) {
        int gg = 0;
        es_draw(seed, k0 + q, m, mutate, &i[q], &j[q], &gg);
        g[q] = (uint8_t)gg;
    }
}

// One edge switch (i, j, g) of Def. 2.1 on E and its edge set (built here):
// for exhaustive tests.  Returns the outcome code.
int oracle_edge_switch(uint64_t *E, uint64_t m, uint64_t i, uint64_t j, int g) {
    EdgeSet S(m);
    for (uint64_t e = 0; e < m; ++e) S.insert(E[e]);
    return edge_switch(E, S, i, j, g, 0);
}

// ES-MC: switches k = k0 .. k0+r-1 with the draws above, applied one after
// another by Def. 2.1 (validated and canonicalised first, as oracle_run).
// counts (nullable): totals; outcome (nullable, r bytes): per switch.
// m < 2 leaves E as it is (no pair of distinct indices exists).
int oracle_es_run(uint64_t *E, uint64_t m, uint32_t n, uint64_t seed, uint64_t k0, uint64_t r, oracle_counts *counts,
                  uint8_t *outcome, uint32_t mutate) {
    int rc = oracle_validate(E, m, n);
    if (rc) return rc;
    for (uint64_t e = 0; e < m; ++e) E[e] = make_key(key_u(E[e]), key_v(E[e]));
    if (counts) memset(counts, 0, sizeof(*counts));
    if (m < 2) return 0;
    EdgeSet S(m);
    for (uint64_t e = 0; e < m; ++e) S.insert(E[e]);
    for (uint64_t q = 0; q < r; ++q) {
        uint64_t i, j;
        int g;
        es_draw(seed, k0 + q, m, mutate, &i, &j, &g);
        const int oc = edge_switch(E, S, i, j, g, mutate & 0xFFFFu);
        if (outcome) outcome[q] = (uint8_t)oc;
        if (counts) {
            counts->attempts++;
            if (oc == OR_LEGAL) counts->legal++;
            if (oc == OR_LOOP) counts->rej_loop++;
            if (oc == OR_EXISTS) counts->rej_exists++;
        }
    }
    return 0;
}

// ---- graph classes (Sec. 1: directed graphs, graphs with loops, with
// multi-edges) -----------------------------------------------------------
// cls bits: 1 = loops allowed, 2 = multi-edges allowed, 4 = directed.
//   undirected: edges stored (min, max); tau of Def. 2.1 with g;
//   directed:   edges stored (tail, head) as given; the switch exchanges the
//               heads, (u->v), (x->y) -> (u->y), (x->v), whatever g is (out-
//               and in-degrees are kept);
//   a loop target is rejected unless loops are allowed; a present target is
//   rejected unless multi-edges are allowed, and so is a switch whose two
//   targets coincide (it would double an edge);
//   undirected with loops and no multi-edges: a switch with a loop among its
//   sources gives the same targets for g = 0 and g = 1, while its reverse
//   move has one g, so it runs for g = 0 only and is rejected (as a loop) for
//   g = 1 -- this keeps the chain symmetric (Thm. 3.3's argument), hence
//   uniform over the class.  With multi-edges the plain switch is kept: the
//   chain then balances the configuration model's weight 1 / (prod over
//   edges of multiplicity! * 2^loops) (directed: 1 / prod multiplicity!).
// The edge multiset is a count per key.
enum { CLS_LOOPS = 1, CLS_MULTI = 2, CLS_DIRECTED = 4 };

static uint64_t cls_key(uint32_t a, uint32_t b, uint32_t cls) {
    return (cls & CLS_DIRECTED) ? (((uint64_t)a << 32) | b) : make_key(a, b);
}

// Planted mistakes of the class switch (for the pin tests).
enum { CMUT_DIR_TAILS = 1, CMUT_NO_SAME = 2, CMUT_LOOPS_ALWAYS = 4, CMUT_LOOP_BOTH_G = 8 };

static int edge_switch_cls(uint64_t *E, std::unordered_map<uint64_t, uint32_t> &S, uint64_t i, uint64_t j, int g,
                           uint32_t cls, uint32_t mutate) {
    const uint64_t e1 = E[i], e2 = E[j];
    const uint32_t u = key_u(e1), v = key_v(e1), x = key_u(e2), y = key_v(e2);
    uint32_t a0, a1, b0, b1;
    if ((cls & CLS_DIRECTED) && (mutate & CMUT_DIR_TAILS)) {
        a0 = u; a1 = x; b0 = v; b1 = y;
    } else if (cls & CLS_DIRECTED) {
        a0 = u; a1 = y; b0 = x; b1 = v;
    } else if (g == 0) {
        a0 = u; a1 = x; b0 = v; b1 = y;
    } else {
        a0 = u; a1 = y; b0 = v; b1 = x;
    }
    if (!(cls & CLS_LOOPS) && !(mutate & CMUT_LOOPS_ALWAYS) && (a0 == a1 || b0 == b1)) return OR_LOOP;
    if ((cls & (CLS_LOOPS | CLS_MULTI | CLS_DIRECTED)) == CLS_LOOPS && g == 1 && (u == v || x == y) &&
        !(mutate & CMUT_LOOP_BOTH_G))
        return OR_LOOP;
    const uint64_t e3 = cls_key(a0, a1, cls), e4 = cls_key(b0, b1, cls);
    if (!(cls & CLS_MULTI)) {
        if ((e3 == e4 && !(mutate & CMUT_NO_SAME)) || S.count(e3) || S.count(e4)) return OR_EXISTS;
    }
    for (uint64_t e : {e1, e2}) {
        auto it = S.find(e);
        if (--it->second == 0) S.erase(it);
    }
    ++S[e3];
    ++S[e4];
    E[i] = e3;
    E[j] = e4;
    return OR_LEGAL;
}

// Input check of a graph of class cls on [0, n): ids in range, loops only if
// allowed, duplicates only if multi-edges are allowed.  Returns 0, -2 or -3.
int oracle_validate_class(const uint64_t *E, uint64_t m, uint32_t n, uint32_t cls) {
    std::unordered_map<uint64_t, uint32_t> S;
    for (uint64_t e = 0; e < m; ++e) {
        const uint32_t a = key_u(E[e]), b = key_v(E[e]);
        if (a >= n || b >= n || a == 0xFFFFFFFFu || b == 0xFFFFFFFFu) return -3;
        if (a == b && !(cls & CLS_LOOPS)) return -2;
        if (S[cls_key(a, b, cls)]++ && !(cls & CLS_MULTI)) return -2;
    }
    return 0;
}

// Alg. 3 for a graph class: r global switches from superstep t0 (pi and the
// P_L skips as in oracle_run) with the class's switch.  Undirected inputs
// given as (max, min) are canonicalised; directed ones are kept as given.
int oracle_run_class(uint64_t *E, uint64_t m, uint32_t n, uint64_t seed, uint32_t t0, uint32_t r, uint32_t pl,
                     uint32_t cls, oracle_counts *per_step, uint8_t *last_outcome, uint32_t mutate) {
    int rc = oracle_validate_class(E, m, n, cls);
    if (rc) return rc;
    for (uint64_t e = 0; e < m; ++e) E[e] = cls_key(key_u(E[e]), key_v(E[e]), cls);
    if (per_step) memset(per_step, 0, sizeof(oracle_counts) * r);
    if (m < 2) return 0;
    std::unordered_map<uint64_t, uint32_t> S;
    for (uint64_t e = 0; e < m; ++e) ++S[E[e]];
    std::vector<uint32_t> pi(m);
    for (uint32_t s = 0; s < r; ++s) {
        const uint32_t t = t0 + s;
        oracle_permutation_mut(m, seed, t, pi.data(), 0);
        for (uint64_t k = 0; k < m / 2; ++k) {
            const uint64_t i = pi[2 * k], j = pi[2 * k + 1];
            const int oc = pl_skip(seed, t, k, pl) ? OR_PL : edge_switch_cls(E, S, i, j, i < j, cls, mutate);
            if (s + 1 == r && last_outcome) last_outcome[k] = (uint8_t)oc;
            if (per_step) {
                oracle_counts &c = per_step[s];
                c.attempts++;
                c.legal += oc == OR_LEGAL;
                c.rej_loop += oc == OR_LOOP;
                c.rej_exists += oc == OR_EXISTS;
                c.rej_pl += oc == OR_PL;
            }
        }
    }
    return 0;
}

// One switch of class cls with explicit (i, j, g) on E (for exhaustive tests).
int oracle_edge_switch_class(uint64_t *E, uint64_t m, uint64_t i, uint64_t j, int g, uint32_t cls, uint32_t mutate) {
    std::unordered_map<uint64_t, uint32_t> S;
    for (uint64_t e = 0; e < m; ++e) ++S[E[e]];
    return edge_switch_cls(E, S, i, j, g, cls, mutate);
}

// Self-check of the edge set against std::unordered_set on a seeded random
// mix of insert / erase / lookup.  Returns the number of disagreements.
uint64_t oracle_selftest_edgeset(uint64_t ops, uint64_t seed) {
    EdgeSet a(16);
    std::unordered_set<uint64_t> b;
    uint64_t s = seed, bad = 0;
    for (uint64_t q = 0; q < ops; ++q) {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        uint32_t op = (uint32_t)(s >> 62);
        uint64_t k = make_key((uint32_t)(s >> 40) & 1023u, ((uint32_t)(s >> 20) & 1023u) + 1024u);
        if (op == 0 || op == 1) {
            bool x = a.insert(k), y = b.insert(k).second;
            bad += (x != y);
        } else if (op == 2) {
            bool x = a.erase(k), y = b.erase(k) > 0;
            bad += (x != y);
        } else {
            bad += (a.contains(k) != (b.count(k) > 0));
        }
        bad += (a.size() != b.size());
    }
    return bad;
}

}  // extern "C"

// ORACLE -- test infrastructure only.
//
// Plain sequential CPU definitions of the input realisation steps (the
// steps before the chain: Sec. 6 builds its synthetic inputs as G(n,p)
// graphs, SynGnp, and as Havel-Hakimi realisations of i.i.d. power-law
// degree sequences Pld([a..b], gamma), SynPld).  Only the tests, the smoke
// check and the benchmark's CPU-baseline leg may load this; the HIP library
// never does, and the two share no code.
//
// Random draws come from Philox4x32-10 (the oracle's, pinned to rocRAND) with
// key (seed_lo, seed_hi) and counter tags 3 (G(n,p)) and 4 (degrees); tags
// 0 .. 2 belong to the chain.  Where floating point decides an integer, it
// is done by the portable ln_p / exp_p below, built only from correctly
// rounded IEEE double operations (+, -, *, /, exact bit manipulation and
// floor) in a fixed order, never contracted into fused multiply-adds, so an
// implementation following the same steps gets the same bits.
//
//   ln_p(x), x > 0 normal: x = 2^e * m with m in [1, 2); if m > sqrt(2)
//     (the double nearest it) then m /= 2, e += 1.  f = m - 1,
//     s = f / (2 + f), z = s * s, P = Horner over z of c_1 .. c_11 with
//     c_j = 1 / (2j + 1) (P = c_11; for j = 10 .. 1: P = P * z + c_j),
//     t = 2 * s, ln m = t + t * (z * P), and
//     ln_p(x) = e * LN2_HI + (e * LN2_LO + ln m)  (fdlibm's split of ln 2).
//     This is ln m = 2 atanh(s) by its power series (Abramowitz & Stegun
//     4.1.27), |s| <= 0.1716, eleven terms.
//   exp_p(x), -700 <= x <= 0: k = floor(x * INV_LN2 + 0.5),
//     r = (x - k * LN2_HI) - k * LN2_LO, p = Horner over r of 1/j!,
//     j = 13 .. 0 (p = 1/13!; for j = 12 .. 0: p = p * r + 1/j!), times 2^k.
//
// G(n,p) (each of the N = n(n-1)/2 vertex pairs an edge independently with
// probability p): pairs w < v are indexed q = v(v-1)/2 + w.  [0, N) is cut
// into chunks of L pairs, L the smallest power of two >= 64 with L p >= 64
// (at most 2^40).  In chunk j = [jL, min(jL + L, N)) a cursor c starts at
// jL; draw t = 0, 1, ... takes (x0, x1) of Philox(ctr = (j_lo, j_hi, t, 3)),
// U = ((x0 << 32 | x1) >> 11) + 1) / 2^53 in (0, 1], G = ln_p(U) /
// ln_p(1 - p); if G >= end - c the chunk ends, else pair q = c + floor(G) is
// an edge and c = q + 1 (the chunk ends when c reaches its end).  floor(G)
// is geometric: the number of failures before a success (Batagelj and
// Brandes, Phys. Rev. E 71, 2005); restarting at a chunk start is exact,
// the trials being independent.  p >= 1: every pair; p <= 0 or n < 2: none.
// Edges come out in q order as (w << 32) | v.
//
// Degrees: weight W_i = floor(exp_p(-(gamma * (ln_p(a + i) - ln_p(a)))) *
// 2^43) for i = 0 .. b - a (an integer proportional to (a+i)^-gamma), CDF
// C_i = W_0 + ... + W_i, total T.  Vertex v's draw r: R = x0 << 32 | x1 of
// Philox(ctr = (v, r, 0, 4)), u = floor(R T / 2^64), degree a + min{i :
// C_i > u}.  Every vertex takes draw 0; while the sum is odd vertex 0 takes
// draws 1, 2, ... (at most 65535; a = b with an odd sum fails at once).
//
// Havel-Hakimi: the vertices are placed in positions 0 .. n-1 by (degree
// descending, id ascending); the residual degree of a position starts at its
// degree.  While some residual is positive: v = the position of largest
// residual (smallest position among ties), d its residual; its partners are
// the d other positions of positive residual with the largest (residual,
// position) pairs (fewer than d: not graphical); v's residual becomes 0 and
// each partner's drops by one; edges (v, partner) are emitted by ascending
// partner position.  Any choice of the d largest residuals realises a
// graphical sequence (Havel 1955, Hakimi 1962), so this fails exactly on
// non-graphical input.  Edge keys are (min id << 32) | max id.
//
// Relabel: pi = the permutation of Def. 3.2 over n elements (the oracle's
// oracle_permutation) with seed ^ 0x9E3779B97F4A7C15 and superstep 0; vertex
// pi[r] gets id r; every edge key is rewritten and made canonical.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <set>
#include <utility>
#include <vector>

extern "C" void oracle_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out);
extern "C" void oracle_permutation(uint64_t m, uint64_t seed, uint32_t t, uint32_t *pi);

namespace {

// Planted mistakes, for tests that show a pin catches them (0: the definitions).
enum : uint32_t {
    GMUT_LN_TERMS = 1,        // ln_p series cut to five terms
    GMUT_GNP_NO_ADVANCE = 2,  // the cursor stays on the chosen pair
    GMUT_GNP_CEIL = 4,        // ceil instead of floor of G
    GMUT_GNP_CHUNK_SKIP = 8,  // each chunk's cursor starts one pair late
    GMUT_PLD_SIGN = 16,       // weights (a+i)^+gamma
    GMUT_PLD_OFF1 = 32,       // degree a + i + 1
    GMUT_HH_TIE = 64,         // boundary partners of smallest position
    GMUT_HH_PICK = 128,       // v of largest position among ties
    GMUT_RELABEL_INV = 256,   // vertex r gets id pi[r]
    GMUT_EXP_TERMS = 512,     // exp_p series cut to seven terms
};
uint32_t g_mut = 0;

uint64_t bits_of(double x) {
    uint64_t b;
    memcpy(&b, &x, 8);
    return b;
}
double of_bits(uint64_t b) {
    double x;
    memcpy(&x, &b, 8);
    return x;
}

const double kLn2Hi = 6.93147180369123816490e-01;
const double kLn2Lo = 1.90821492927058770002e-10;
const double kSqrt2 = 1.4142135623730951;
const double kInvLn2 = 1.4426950408889634;

double ln_p(double x) {
    const uint64_t b = bits_of(x);
    int e = (int)((b >> 52) & 0x7FF) - 1023;
    double m = of_bits((b & 0xFFFFFFFFFFFFFull) | 0x3FF0000000000000ull);
    if (m > kSqrt2) {
        m = m * 0.5;
        e += 1;
    }
    const double f = m - 1.0;
    const double s = f / (2.0 + f);
    const double z = s * s;
    double P = 1.0 / 23.0;
    for (int j = 10; j >= 1; --j) P = P * z + 1.0 / (double)(2 * j + 1);
    if (g_mut & GMUT_LN_TERMS) {
        P = 1.0 / 11.0;
        for (int j = 4; j >= 1; --j) P = P * z + 1.0 / (double)(2 * j + 1);
    }
    const double t = 2.0 * s;
    const double lnm = t + t * (z * P);
    return (double)e * kLn2Hi + ((double)e * kLn2Lo + lnm);
}

double exp_p(double x) {
    const double kd = std::floor(x * kInvLn2 + 0.5);
    const int k = (int)kd;
    const double r = (x - kd * kLn2Hi) - kd * kLn2Lo;
    double fact[14];
    fact[0] = 1.0;
    for (int j = 1; j < 14; ++j) fact[j] = fact[j - 1] * (double)j;  // exact below 2^53
    const int top = (g_mut & GMUT_EXP_TERMS) ? 7 : 13;
    double p = 1.0 / fact[top];
    for (int j = top - 1; j >= 0; --j) p = p * r + 1.0 / fact[j];
    return p * of_bits((uint64_t)(k + 1023) << 52);
}

void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed, uint32_t out[4]) {
    const uint32_t ctr[4] = {c0, c1, c2, c3};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, out);
}

uint64_t canon(uint32_t a, uint32_t b) { return a < b ? ((uint64_t)a << 32) | b : ((uint64_t)b << 32) | a; }

// q -> (w, v) with q = v(v-1)/2 + w, 0 <= w < v: an estimate, then exact
// integer correction.
void pair_of(uint64_t q, uint32_t *w, uint32_t *v) {
    uint64_t vv = (uint64_t)((1.0 + std::sqrt(1.0 + 8.0 * (double)q)) / 2.0);
    while (vv > 0 && vv * (vv - 1) / 2 > q) --vv;
    while ((vv + 1) * vv / 2 <= q) ++vv;
    *v = (uint32_t)vv;
    *w = (uint32_t)(q - vv * (vv - 1) / 2);
}

}  // namespace

extern "C" {

void oracle_gen_set_mutate(uint32_t mutate) { g_mut = mutate; }

double oracle_ln_p(double x) { return ln_p(x); }
double oracle_exp_p(double x) { return exp_p(x); }

void oracle_pair_of(uint64_t q, uint32_t *w, uint32_t *v) { pair_of(q, w, v); }

// Chunk length of G(n,p) for probability p (0 < p < 1).
uint64_t oracle_gnp_chunk(double p) {
    uint64_t L = 64;
    while ((double)L * p < 64.0 && L < (1ull << 40)) L <<= 1;
    return L;
}

// G(n,p) as defined above.  Writes at most cap keys; returns the edge count
// (the number written is min(count, cap)).
int64_t oracle_gen_gnp(uint32_t n, double p, uint64_t seed, uint64_t *out, int64_t cap) {
    int64_t m = 0;
    auto emit = [&](uint64_t q) {
        if (m < cap) {
            uint32_t w, v;
            pair_of(q, &w, &v);
            out[m] = ((uint64_t)w << 32) | v;
        }
        ++m;
    };
    if (n < 2 || !(p > 0.0)) return 0;
    const uint64_t N = (uint64_t)n * (n - 1) / 2;
    if (p >= 1.0) {
        for (uint64_t q = 0; q < N; ++q) emit(q);
        return m;
    }
    const uint64_t L = oracle_gnp_chunk(p);
    const double lq = ln_p(1.0 - p);
    for (uint64_t j = 0; j * L < N; ++j) {
        const uint64_t end = std::min(j * L + L, N);
        uint64_t c = j * L + ((g_mut & GMUT_GNP_CHUNK_SKIP) ? 1 : 0);
        for (uint32_t t = 0;; ++t) {
            uint32_t x[4];
            philox((uint32_t)j, (uint32_t)(j >> 32), t, 3u, seed, x);
            const uint64_t R = ((uint64_t)x[0] << 32) | x[1];
            const double U = (double)((R >> 11) + 1) * 0x1.0p-53;
            const double G = ln_p(U) / lq;
            if (!(G < (double)(end - c))) break;
            const uint64_t q = c + ((g_mut & GMUT_GNP_CEIL) ? (uint64_t)std::ceil(G) : (uint64_t)G);
            if (q >= end) break;
            emit(q);
            c = (g_mut & GMUT_GNP_NO_ADVANCE) ? q : q + 1;
            if (c >= end) break;
        }
    }
    return m;
}

// Degree sequence as defined above.  Returns the (even) degree sum, or -1 for
// bad parameters or when no even sum was reached; *redraws (nullable) gets
// the number of redraws of vertex 0.
int64_t oracle_gen_pld(uint32_t n, double gamma, uint32_t dmin, uint32_t dmax, uint64_t seed, uint32_t *deg,
                       uint32_t *redraws) {
    if (n == 0 || dmin < 1 || dmax < dmin || dmax - dmin >= (1u << 20) || !(gamma >= 0.0)) return -1;
    const uint32_t nv = dmax - dmin + 1;
    const double l0 = ln_p((double)dmin);
    std::vector<uint64_t> C(nv);
    uint64_t acc = 0;
    for (uint32_t i = 0; i < nv; ++i) {
        const double a = ln_p((double)(dmin + i)) - l0;
        // the planted sign mistake keeps the weight in range by flipping about ln(b/a)
        const double x = (g_mut & GMUT_PLD_SIGN) ? gamma * a - gamma * (ln_p((double)dmax) - l0) : -(gamma * a);
        if (x < -700.0) return -1;
        acc += (uint64_t)(exp_p(x) * 0x1.0p43);
        C[i] = acc;
    }
    const uint64_t T = acc;
    auto draw = [&](uint32_t v, uint32_t r) {
        uint32_t x[4];
        philox(v, r, 0u, 4u, seed, x);
        const uint64_t R = ((uint64_t)x[0] << 32) | x[1];
        const uint64_t u = (uint64_t)(((unsigned __int128)R * T) >> 64);
        const uint32_t i = (uint32_t)(std::upper_bound(C.begin(), C.end(), u) - C.begin());
        return dmin + i + ((g_mut & GMUT_PLD_OFF1) ? 1u : 0u);
    };
    int64_t sum = 0;
    for (uint32_t v = 0; v < n; ++v) {
        deg[v] = draw(v, 0);
        sum += deg[v];
    }
    uint32_t r = 0;
    while (sum & 1) {
        if (dmin == dmax || r == 65535) return -1;
        ++r;
        sum -= deg[0];
        deg[0] = draw(0, r);
        sum += deg[0];
    }
    if (redraws) *redraws = r;
    return sum;
}

// Havel-Hakimi as defined above.  Returns the edge count (writes at most cap
// keys), or -1 if the sequence is not graphical.
int64_t oracle_gen_havel_hakimi(uint32_t n, const uint32_t *deg, uint64_t *out, int64_t cap) {
    std::vector<uint32_t> O(n);
    for (uint32_t v = 0; v < n; ++v) O[v] = v;
    std::sort(O.begin(), O.end(), [&](uint32_t a, uint32_t b) {
        return deg[a] != deg[b] ? deg[a] > deg[b] : a < b;
    });
    std::vector<uint32_t> res(n);
    std::set<std::pair<uint32_t, uint32_t>> S;  // (residual, position), residual > 0
    for (uint32_t p = 0; p < n; ++p) {
        res[p] = deg[O[p]];
        if (res[p] > 0) S.insert({res[p], p});
    }
    int64_t m = 0;
    std::vector<uint32_t> part;
    while (!S.empty()) {
        const uint32_t top = S.rbegin()->first;
        const auto it = (g_mut & GMUT_HH_PICK) ? std::prev(S.end()) : S.lower_bound({top, 0u});
        const uint32_t s = it->second, d = top;
        S.erase(it);
        res[s] = 0;
        if (S.size() < d) return -1;
        part.clear();
        auto rit = S.rbegin();
        for (uint32_t q = 0; q < d; ++q, ++rit) part.push_back(rit->second);
        if (g_mut & GMUT_HH_TIE) {  // among the boundary residual, the smallest positions
            const uint32_t x = res[part.back()];
            uint32_t k = 0;
            for (uint32_t p : part) k += res[p] == x;
            part.erase(std::remove_if(part.begin(), part.end(), [&](uint32_t p) { return res[p] == x; }),
                       part.end());
            for (auto fit = S.lower_bound({x, 0u}); k > 0; ++fit, --k) part.push_back(fit->second);
        }
        std::sort(part.begin(), part.end());
        for (uint32_t p : part) {
            S.erase({res[p], p});
            if (--res[p] > 0) S.insert({res[p], p});
            if (m < cap) out[m] = canon(O[s], O[p]);
            ++m;
        }
    }
    return m;
}

// Relabel as defined above (in place).
void oracle_gen_relabel(uint64_t *E, uint64_t m, uint32_t n, uint64_t seed) {
    std::vector<uint32_t> pi(std::max<uint32_t>(n, 1)), sigma(std::max<uint32_t>(n, 1));
    if (n > 0) oracle_permutation(n, seed ^ 0x9E3779B97F4A7C15ull, 0u, pi.data());
    for (uint32_t r = 0; r < n; ++r) {
        if (g_mut & GMUT_RELABEL_INV)
            sigma[r] = pi[r];
        else
            sigma[pi[r]] = r;
    }
    for (uint64_t e = 0; e < m; ++e) E[e] = canon(sigma[(uint32_t)(E[e] >> 32)], sigma[(uint32_t)E[e]]);
}

}  // extern "C"

/*
 * Seeded synthetic graph generators: the inputs that both the HIP path and the
 * oracle consume.  Nothing here performs an edge switch; these routines only
 * produce a simple undirected starting graph with a prescribed structure.
 *
 * Workloads (stand-ins for the paper's SynGnp and SynPld families, Sec. 6):
 *   - G(n,p) by geometric skipping (Batagelj & Brandes, Phys. Rev. E 71, 2005).
 *   - Pld([a..b], gamma) degree sequences (Sec. 2.1 notation), realised with
 *     the Havel-Hakimi construction, then vertex ids relabelled at random.
 *
 * Random source: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014), seeded per call.
 * Edge keys are packed as (min << 32) | max.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t s;
} gg_rng;

static uint64_t gg_next(gg_rng *r) {
    uint64_t z = (r->s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* uniform double in [0, 1) with 53 random bits */
static double gg_unif(gg_rng *r) { return (double)(gg_next(r) >> 11) * (1.0 / 9007199254740992.0); }

/* uniform integer in [0, bound) by rejection (bound > 0) */
static uint64_t gg_below(gg_rng *r, uint64_t bound) {
    uint64_t lim = UINT64_MAX - (UINT64_MAX % bound);
    uint64_t x;
    do {
        x = gg_next(r);
    } while (x >= lim);
    return x % bound;
}

static uint64_t pack(uint32_t a, uint32_t b) {
    uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
    return ((uint64_t)lo << 32) | hi;
}

/*
 * G(n,p): each of the n(n-1)/2 vertex pairs is an edge independently with
 * probability p.  Edges come out ordered by (larger id, smaller id).
 * Returns the edge count, or -(needed) if cap is too small (nothing valid
 * is written in that case beyond cap).
 */
int64_t gg_gnp(uint32_t n, double p, uint64_t seed, uint64_t *out, int64_t cap) {
    gg_rng r = {seed};
    int64_t m = 0;
    if (n < 2 || p <= 0.0) return 0;
    if (p >= 1.0) {
        for (uint32_t v = 1; v < n; ++v)
            for (uint32_t w = 0; w < v; ++w) {
                if (m < cap) out[m] = pack(w, v);
                ++m;
            }
        return m <= cap ? m : -m;
    }
    double lq = log(1.0 - p);
    int64_t v = 1, w = -1;
    while (v < (int64_t)n) {
        double u = gg_unif(&r);
        w += 1 + (int64_t)floor(log(1.0 - u) / lq);
        while (w >= v && v < (int64_t)n) {
            w -= v;
            ++v;
        }
        if (v < (int64_t)n) {
            if (m < cap) out[m] = pack((uint32_t)w, (uint32_t)v);
            ++m;
        }
    }
    return m <= cap ? m : -m;
}

/*
 * Degree sequence with i.i.d. entries from Pld([dmin..dmax], gamma):
 * P(X = k) proportional to k^-gamma for dmin <= k <= dmax.  If the sum is odd,
 * entry 0 is redrawn until it is even.  Returns the degree sum.
 */
int64_t gg_powerlaw_degrees(uint32_t n, uint32_t dmin, uint32_t dmax, double gamma, uint64_t seed,
                            uint32_t *deg) {
    if (dmin < 1 || dmax < dmin || n == 0) return -1;
    uint32_t nv = dmax - dmin + 1;
    double *cdf = (double *)malloc(sizeof(double) * nv);
    if (!cdf) return -1;
    double acc = 0.0;
    for (uint32_t i = 0; i < nv; ++i) {
        acc += pow((double)(dmin + i), -gamma);
        cdf[i] = acc;
    }
    for (uint32_t i = 0; i < nv; ++i) cdf[i] /= acc;
    cdf[nv - 1] = 1.0;
    gg_rng r = {seed};
    int64_t sum = 0;
    for (uint32_t v = 0; v < n; ++v) {
        double u = gg_unif(&r);
        uint32_t lo = 0, hi = nv - 1;
        while (lo < hi) {
            uint32_t mid = (lo + hi) / 2;
            if (cdf[mid] > u)
                hi = mid;
            else
                lo = mid + 1;
        }
        deg[v] = dmin + lo;
        sum += deg[v];
    }
    while (sum & 1) {
        sum -= deg[0];
        double u = gg_unif(&r);
        uint32_t lo = 0, hi = nv - 1;
        while (lo < hi) {
            uint32_t mid = (lo + hi) / 2;
            if (cdf[mid] > u)
                hi = mid;
            else
                lo = mid + 1;
        }
        deg[0] = dmin + lo;
        sum += deg[0];
    }
    free(cdf);
    return sum;
}

/*
 * Havel-Hakimi realisation of a degree sequence.  Repeatedly takes a vertex
 * of largest residual degree d and joins it to d other vertices of largest
 * residual degree.  Vertices of equal residual degree sit in a LIFO bucket;
 * buckets are filled initially in ascending id order, so ties favour the
 * most recently (re)inserted vertex.  The construction is deterministic.
 * Returns the edge count, or -1 if the sequence is not graphical.
 */
int64_t gg_havel_hakimi(uint32_t n, const uint32_t *deg_in, uint64_t *out) {
    uint32_t maxd = 0;
    int64_t sum = 0;
    for (uint32_t v = 0; v < n; ++v) {
        if (deg_in[v] > maxd) maxd = deg_in[v];
        sum += deg_in[v];
    }
    if (sum & 1) return -1;
    if (maxd >= n && sum > 0) return -1;
    uint32_t *d = (uint32_t *)malloc(sizeof(uint32_t) * n);
    int64_t *head = (int64_t *)malloc(sizeof(int64_t) * ((size_t)maxd + 1));
    int64_t *nxt = (int64_t *)malloc(sizeof(int64_t) * n);
    int64_t *prv = (int64_t *)malloc(sizeof(int64_t) * n);
    uint32_t *pick = (uint32_t *)malloc(sizeof(uint32_t) * ((size_t)maxd + 1));
    if (!d || !head || !nxt || !prv || !pick) {
        free(d); free(head); free(nxt); free(prv); free(pick);
        return -1;
    }
    for (uint32_t b = 0; b <= maxd; ++b) head[b] = -1;
#define GG_PUSH(v)                                   \
    do {                                             \
        uint32_t b_ = d[(v)];                        \
        prv[(v)] = -1;                               \
        nxt[(v)] = head[b_];                         \
        if (head[b_] >= 0) prv[head[b_]] = (v);      \
        head[b_] = (v);                              \
    } while (0)
#define GG_UNLINK(v)                                 \
    do {                                             \
        uint32_t b_ = d[(v)];                        \
        if (prv[(v)] >= 0)                           \
            nxt[prv[(v)]] = nxt[(v)];                \
        else                                         \
            head[b_] = nxt[(v)];                     \
        if (nxt[(v)] >= 0) prv[nxt[(v)]] = prv[(v)]; \
    } while (0)
    for (uint32_t v = 0; v < n; ++v) {
        d[v] = deg_in[v];
        if (d[v] > 0) GG_PUSH(v);
    }
    int64_t m = 0, bad = 0;
    uint32_t top = maxd;
    while (!bad) {
        while (top > 0 && head[top] < 0) --top;
        if (top == 0) break;
        uint32_t v = (uint32_t)head[top];
        GG_UNLINK(v);
        uint32_t need = d[v];
        d[v] = 0;
        uint32_t got = 0;
        for (uint32_t b = top; b >= 1 && got < need; --b)
            for (int64_t u = head[b]; u >= 0 && got < need; u = nxt[u]) pick[got++] = (uint32_t)u;
        if (got < need) {
            bad = 1;
            break;
        }
        for (uint32_t q = 0; q < got; ++q) {
            uint32_t u = pick[q];
            GG_UNLINK(u);
            d[u] -= 1;
            if (d[u] > 0) GG_PUSH(u);
            out[m++] = pack(v, u);
        }
    }
#undef GG_PUSH
#undef GG_UNLINK
    free(d); free(head); free(nxt); free(prv); free(pick);
    return bad ? -1 : m;
}

/* Relabel vertex ids by a uniform random permutation of [0, n) (Fisher-Yates)
 * and re-pack every edge as (min << 32) | max.  Edge order is unchanged. */
int gg_shuffle_ids(uint32_t n, uint64_t seed, uint64_t *edges, int64_t m) {
    uint32_t *perm = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    if (!perm) return -1;
    for (uint32_t v = 0; v < n; ++v) perm[v] = v;
    gg_rng r = {seed};
    for (uint32_t v = n; v > 1; --v) {
        uint32_t j = (uint32_t)gg_below(&r, v);
        uint32_t tmp = perm[v - 1];
        perm[v - 1] = perm[j];
        perm[j] = tmp;
    }
    for (int64_t e = 0; e < m; ++e) {
        uint32_t a = (uint32_t)(edges[e] >> 32), b = (uint32_t)edges[e];
        edges[e] = pack(perm[a], perm[b]);
    }
    free(perm);
    return 0;
}

/* Uniform draws for harness-level sampling (graph sizes, exponents, arrival
 * times): n values in [0,1). */
void gg_uniforms(uint64_t seed, double *out, int64_t n) {
    gg_rng r = {seed};
    for (int64_t i = 0; i < n; ++i) out[i] = gg_unif(&r);
}

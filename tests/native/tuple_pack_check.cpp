// Host checks of the packed tuple word (paper_2111_03005_amd/csrc/tuple_pack.h),
// the functions the kernels use, run on the CPU:
//   1. mix_w is a bijection on w-bit words (exhaustive for w <= 20) with
//      inverse unmix_w, and the (u, v - u) coding of edge keys returns u;
//   2. tag codes round-trip and keep the order of the 32-bit tags;
//   3. the packed word (H' << (64 - w + b1)) | code orders as (H', tag);
//   4. the top hash bits spread structured key sets (banded, star and
//      batched graphs) evenly over partitions and cells.
// Prints "ok" or the first failure.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <vector>

#include "tuple_pack.h"

using namespace gesmc;

static uint64_t sm_state = 0x1234567ull;
static uint64_t splitmix() {
    uint64_t z = (sm_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

#define CHECK(cond, ...)                  \
    do {                                  \
        if (!(cond)) {                    \
            printf("FAIL: " __VA_ARGS__); \
            printf("\n");                 \
            return 1;                     \
        }                                 \
    } while (0)

static uint64_t key_of(uint64_t u, uint64_t v) { return (u << 32) | v; }

// Largest bucket of the top `bits` bits of H over a key set, and the mean.
static int spread(const std::vector<uint64_t> &keys, int vb, int db, int bits, double *ratio) {
    const int w = vb + db;
    std::vector<uint32_t> cnt((size_t)1 << bits, 0);
    for (uint64_t k : keys) ++cnt[key_hash_w(k, db, w) >> (w - bits)];
    const double mean = (double)keys.size() / cnt.size();
    const uint32_t mx = *std::max_element(cnt.begin(), cnt.end());
    *ratio = mx / mean;
    return (int)mx;
}

int main() {
    // 1. mix_w is a bijection with inverse unmix_w: exhaustive for w <= 20,
    //    2^18 random words for every wider w up to 62
    for (int w = 1; w <= 20; ++w) {
        std::vector<uint8_t> seen((size_t)1 << w, 0);
        for (uint64_t x = 0; x < (1ull << w); ++x) {
            const uint64_t h = mix_w(x, w);
            CHECK(h < (1ull << w), "mix out of range w=%d", w);
            CHECK(!seen[h], "mix collision w=%d x=%llu", w, (unsigned long long)x);
            seen[h] = 1;
            CHECK(unmix_w(h, w) == x, "inverse w=%d x=%llu", w, (unsigned long long)x);
        }
    }
    for (int w = 21; w <= 62; ++w) {
        for (int i = 0; i < (1 << 18); ++i) {
            const uint64_t x = splitmix() & low_mask(w);
            const uint64_t h = mix_w(x, w);
            CHECK(h <= low_mask(w), "mix out of range w=%d", w);
            CHECK(unmix_w(h, w) == x, "inverse w=%d", w);
        }
    }
    //    edge keys (u, v), u < v, coded as (u, v - u) on vb + db bits: the
    //    coding comes back through unmix_w (so distinct keys get distinct
    //    hashes) and so does the vertex
    const int widths[][2] = {{20, 20}, {22, 22}, {26, 17}, {31, 31}, {26, 1}, {5, 3}};
    for (const auto &vd : widths) {
        const int vb = vd[0], db = vd[1], w = vb + db;
        for (int i = 0; i < 200000; ++i) {
            const uint64_t d = 1 + splitmix() % ((1ull << db) - 1 + (db == 0));
            const uint64_t u = splitmix() % ((1ull << vb) - d > 0 ? (1ull << vb) - d : 1);
            if (u + d >= (1ull << vb) || d >= (1ull << db)) continue;
            const uint64_t k = key_of(u, u + d);
            const uint64_t h = key_hash_w(k, db, w);
            CHECK(h <= low_mask(w), "key hash out of range vb=%d db=%d", vb, db);
            CHECK(key_hash_w_vertex(h, db, w) == u, "vertex vb=%d db=%d", vb, db);
            CHECK(unmix_w(h, w) == ((u << db) | d), "coding vb=%d db=%d", vb, db);
        }
    }
    // 2. tag codes
    for (int kb = 1; kb <= 30; ++kb) {
        std::vector<uint32_t> tags;
        const uint32_t ell_max = (1u << (kb - 1)) - (kb == 1 ? 0u : 1u);  // 2 ell < 2^kb
        tags.push_back(kTagStays);
        for (int i = 0; i < 2000; ++i) {
            if (ell_max == 0) break;
            const uint32_t k = (uint32_t)(splitmix() % ell_max);
            tags.push_back(k);                                          // ERASE
            tags.push_back(kTagInsert | (k << 1) | (uint32_t)(i & 1));  // INSERT
        }
        if (ell_max > 0) {
            tags.push_back(ell_max - 1);
            tags.push_back(kTagInsert | ((ell_max - 1) << 1) | 1u);
            tags.push_back(0);
            tags.push_back(kTagInsert);
        }
        for (uint32_t t : tags) {
            const uint32_t c = tag_code(t, kb);
            CHECK(c < (2u << kb), "code out of range kb=%d", kb);
            CHECK(tag_of_code(c, kb) == t, "round trip kb=%d tag=%08x", kb, t);
        }
        for (size_t i = 0; i + 1 < tags.size(); ++i)
            for (size_t j = i + 1; j < std::min(tags.size(), i + 8); ++j)
                CHECK((tags[i] < tags[j]) == (tag_code(tags[i], kb) < tag_code(tags[j], kb)),
                      "order kb=%d %08x %08x", kb, tags[i], tags[j]);
    }
    // 3. packed word order = (remaining hash bits, tag) order
    {
        const int vb = 22, w = 44, b1 = 9, kb = 26;
        for (int i = 0; i < 200000; ++i) {
            uint64_t h[2];
            uint32_t t[2];
            for (int a = 0; a < 2; ++a) {
                h[a] = splitmix() & low_mask(w - b1);
                if (i & 1) h[a] &= 0xFF;  // many equal keys
                const uint32_t k = (uint32_t)(splitmix() % ((1u << (kb - 1)) - 1));
                const uint32_t sel = (uint32_t)(splitmix() % 3);
                t[a] = sel == 0 ? k : sel == 1 ? kTagStays : (kTagInsert | (k << 1) | (uint32_t)(splitmix() & 1));
            }
            uint64_t word[2];
            for (int a = 0; a < 2; ++a) {
                const uint64_t full = (splitmix() & low_mask(b1)) << (w - b1) | h[a];  // dropped digit: any
                word[a] = ((full << (64 - w)) << b1) | tag_code(t[a], kb);
            }
            const bool lt_pair = h[0] < h[1] || (h[0] == h[1] && t[0] < t[1]);
            CHECK((word[0] < word[1]) == lt_pair, "word order");
            const uint64_t cm = low_mask(kb + 1);
            CHECK(((word[0] & ~cm) == (word[1] & ~cm)) == (h[0] == h[1]), "key equality");
            CHECK(tag_of_code((uint32_t)(word[0] & cm), kb) == t[0], "tag field");
        }
        (void)vb;
    }
    // 4. spread of structured key sets over partitions (top 11 bits) and cells
    //    (the next 10): a banded and a star graph on 2^18 vertices, and a batch
    //    of 4096 disjoint small graphs (ids up to 2^22, offsets below 2^10)
    {
        std::vector<uint64_t> band, star, batch;
        for (uint64_t u = 0; u < (1u << 17); ++u)
            for (uint64_t d = 1; d <= 16; ++d) band.push_back(key_of(u, u + d));
        for (uint64_t hub = 0; hub < 64; ++hub)
            for (uint64_t v = 64; v < 64 + 32768; ++v) star.push_back(key_of(hub, v));
        for (uint64_t g = 0; g < 4096; ++g)
            for (uint64_t a = 0; a < 32; ++a)
                for (uint64_t b = a + 1; b < a + 17; ++b) batch.push_back(key_of(g * 1024 + a, g * 1024 + b));
        const struct {
            const std::vector<uint64_t> *keys;
            int vb, db;
            const char *name;
        } sets[] = {{&band, 18, 18, "band"}, {&star, 18, 18, "star"}, {&batch, 22, 10, "batch"}};
        for (const auto &st : sets) {
            double r, rc;
            const int mx = spread(*st.keys, st.vb, st.db, 11, &r);
            spread(*st.keys, st.vb, st.db, 21, &rc);
            CHECK(r < 1.25, "partition spread %s: largest %d (%.3f x mean)", st.name, mx, r);
            CHECK(rc < 16, "cell spread %s: %.2f x mean", st.name, rc);
        }
    }
    printf("ok\n");
    return 0;
}

// Drives every entry point of the oracle (oracle/gesmc_oracle.cpp,
// oracle/gen_oracle.cpp) on small inputs, for builds under AddressSanitizer
// and UndefinedBehaviorSanitizer; also checks a few cross-consistencies.
// Prints "ok" and exits 0 on success.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

struct Counts {
    uint64_t attempts, legal, rej_loop, rej_exists, rej_pl;
};

extern "C" {
void oracle_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out);
void oracle_perm_keys(uint64_t seed, uint32_t t, uint64_t m, uint64_t *out);
void oracle_permutation(uint64_t m, uint64_t seed, uint32_t t, uint32_t *pi);
int oracle_validate(const uint64_t *E, uint64_t m, uint32_t n);
int oracle_run(uint64_t *E, uint64_t m, uint32_t n, uint64_t seed, uint32_t t0, uint32_t r, uint32_t pl,
               Counts *per_step, uint8_t *last_outcome, uint32_t mutate);
int oracle_es_run(uint64_t *E, uint64_t m, uint32_t n, uint64_t seed, uint64_t k0, uint64_t r, Counts *counts,
                  uint8_t *outcome, uint32_t mutate);
int oracle_run_class(uint64_t *E, uint64_t m, uint32_t n, uint64_t seed, uint32_t t0, uint32_t r, uint32_t pl,
                     uint32_t cls, Counts *per_step, uint8_t *last_outcome, uint32_t mutate);
int64_t oracle_gen_gnp(uint32_t n, double p, uint64_t seed, uint64_t *out, int64_t cap);
int64_t oracle_gen_pld(uint32_t n, double gamma, uint32_t dmin, uint32_t dmax, uint64_t seed, uint32_t *deg,
                       uint32_t *redraws);
int64_t oracle_gen_havel_hakimi(uint32_t n, const uint32_t *deg, uint64_t *out, int64_t cap);
void oracle_gen_relabel(uint64_t *E, uint64_t m, uint32_t n, uint64_t seed);
uint64_t oracle_selftest_edgeset(uint64_t ops, uint64_t seed);
}

static int fails = 0;
#define CHECK(c)                                                    \
    do {                                                            \
        if (!(c)) {                                                 \
            std::printf("check failed: %s (line %d)\n", #c, __LINE__); \
            ++fails;                                                \
        }                                                           \
    } while (0)

int main() {
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    oracle_philox4x32_10(ctr, key, out);
    std::vector<uint64_t> keys(1000);
    oracle_perm_keys(42, 3, keys.size(), keys.data());
    std::vector<uint32_t> pi(1000);
    oracle_permutation(pi.size(), 42, 3, pi.data());
    std::vector<char> seen(1000, 0);
    for (uint32_t i : pi) seen[i] = 1;
    for (char s : seen) CHECK(s == 1);

    // inputs from the oracle's own G(n,p) and Havel-Hakimi
    const uint32_t n = 400;
    int64_t m = oracle_gen_gnp(n, 0.03, 9, nullptr, 0);
    std::vector<uint64_t> E(m);
    CHECK(oracle_gen_gnp(n, 0.03, 9, E.data(), m) == m);
    CHECK(oracle_validate(E.data(), m, n) == 0);
    std::vector<uint32_t> deg(n);
    const int64_t sum = oracle_gen_pld(n, 2.3, 2, 19, 4, deg.data(), nullptr);
    CHECK(sum > 0 && sum % 2 == 0);
    std::vector<uint64_t> H(sum / 2 + 1);
    CHECK(oracle_gen_havel_hakimi(n, deg.data(), H.data(), sum / 2) == sum / 2);
    oracle_gen_relabel(H.data(), sum / 2, n, 11);

    for (std::vector<uint64_t> *G : {&E, &H}) {
        const uint64_t mm = G == &E ? (uint64_t)m : (uint64_t)(sum / 2);
        std::vector<uint64_t> a(G->begin(), G->begin() + mm), b = a, c = a;
        std::vector<Counts> pa(5), pb(5);
        std::vector<uint8_t> oa(mm / 2 + 1), ob(mm / 2 + 1);
        CHECK(oracle_run(a.data(), mm, n, 7, 0, 5, 1u << 30, pa.data(), oa.data(), 0) == 0);
        CHECK(oracle_run_class(b.data(), mm, n, 7, 0, 5, 1u << 30, 0, pb.data(), ob.data(), 0) == 0);
        CHECK(std::memcmp(a.data(), b.data(), mm * 8) == 0);
        for (uint32_t cls = 1; cls < 8; ++cls) {
            std::vector<uint64_t> d(G->begin(), G->begin() + mm);
            std::vector<Counts> pd(3);
            CHECK(oracle_run_class(d.data(), mm, n, 7 + cls, 2, 3, 0, cls, pd.data(), nullptr, 0) == 0);
        }
        Counts ce;
        std::vector<uint8_t> oe(20000);
        CHECK(oracle_es_run(c.data(), mm, n, 3, 1ull << 40, 20000, &ce, oe.data(), 0) == 0);
        CHECK(ce.attempts == 20000);
    }
    uint64_t bad[2] = {(2ull << 32) | 2, 1};
    CHECK(oracle_validate(bad, 2, 3) != 0);
    CHECK(oracle_selftest_edgeset(50000, 3) == 0);
    if (fails) return 1;
    std::printf("ok\n");
    return 0;
}

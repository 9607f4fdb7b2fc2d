// Test helper: evaluates rocRAND's Philox4x32-10 engine on the host.
// stdin lines:  "R c0 c1 c2 c3 k0 k1"   -> prints the 4 output words
//               "K seed t m"            -> prints m permutation keys
//                                           (x0 << 32 | x1 at counter (i, 0, t, 0))
// The engine is seeded with key = (seed_lo, seed_hi); subsequence s sets
// counter words (2, 3) and an offset of 4*i numbers advances counter words (0, 1) by i.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdint>
#include <cstdio>

int main() {
    char op;
    while (std::scanf(" %c", &op) == 1) {
        if (op == 'R') {
            unsigned c0, c1, c2, c3, k0, k1;
            if (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) != 6) return 1;
            unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
            unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
            // counter word 0 via the offset; word 1 by whole 2^32-block skips,
            // split so that no single offset overflows 64 bits
            rocrand_device::philox4x32_10_engine e(seed, sub, 4ull * c0);
            unsigned long long quarter = (unsigned long long)(c1 / 4u) << 34;
            for (int q = 0; q < 4; ++q)
                if (quarter) e.discard(quarter);
            if (c1 % 4u) e.discard((unsigned long long)(c1 % 4u) << 34);
            uint4 r = e.next4();
            std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
        } else if (op == 'K') {
            unsigned long long seed, m;
            unsigned t;
            if (std::scanf("%llu %u %llu", &seed, &t, &m) != 3) return 1;
            for (unsigned long long i = 0; i < m; ++i) {
                rocrand_device::philox4x32_10_engine e(seed, (unsigned long long)t, 4ull * i);
                uint4 r = e.next4();
                std::printf("%llu\n", ((unsigned long long)r.x << 32) | r.y);
            }
        } else {
            return 1;
        }
    }
    return 0;
}

// Checks gesmc::CopyPool: every job's bytes arrive exactly, for jobs of many
// shapes issued back to back (the serving loop issues one per iteration).
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "copy_pool.h"

int main(int argc, char **argv) {
    const unsigned threads = argc > 1 ? (unsigned)atoi(argv[1]) : 7u;
    const int jobs = argc > 2 ? atoi(argv[2]) : 200;
    const size_t max_bytes = (size_t)(argc > 3 ? atoi(argv[3]) : 9) << 20;
    gesmc::CopyPool pool(threads);
    std::mt19937_64 rng(12345);
    for (int job = 0; job < jobs; ++job) {
        const int nseg = (int)(rng() % 6);  // includes empty jobs
        std::vector<std::vector<unsigned char>> src(nseg), dst(nseg);
        std::vector<gesmc::CopyPool::Seg> segs;
        for (int g = 0; g < nseg; ++g) {
            const size_t bytes = (rng() % 4 == 0) ? (size_t)(rng() % 64) : (size_t)(rng() % max_bytes);
            src[g].resize(bytes);
            for (size_t i = 0; i < bytes; ++i) src[g][i] = (unsigned char)(i * 131 + g * 7 + job);
            dst[g].assign(bytes, 0xEE);
            segs.push_back({dst[g].data(), src[g].data(), bytes});
        }
        pool.copy(segs);
        for (int g = 0; g < nseg; ++g)
            if (src[g] != dst[g]) {
                std::printf("job %d segment %d (%zu bytes) differs\n", job, g, src[g].size());
                return 1;
            }
    }
    std::printf("ok\n");
    return 0;
}

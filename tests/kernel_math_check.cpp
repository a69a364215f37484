// Host-side check of the pure integer helpers that the tabu-search kernel
// uses (compiled for the CPU by tests/test_kernel_math.py): magic-number
// division, the squeezed move scale and its aspiration bound, and the
// crossover kernel's threshold division.
#include <cstdint>
#include <cstdio>
#include <random>

#include "../paper_2103_10453_amd/csrc/device_common.h"

using namespace plse;

static int fails = 0;
#define CHECK(c, ...)                       \
    do {                                    \
        if (!(c)) {                         \
            if (fails++ < 20) {             \
                std::printf(__VA_ARGS__);   \
                std::printf("\n");          \
            }                               \
        }                                   \
    } while (0)

int main() {
    std::mt19937_64 rng(12345);
    // floor division by a run-time divisor through its magic multiplier
    const uint32_t divs[] = {1, 2, 3, 7, 10, 11, 13, 51, 71, 101, 128, 1000, 65535};
    for (uint32_t d : divs) {
        const uint32_t m = 0xFFFFFFFFu / d;
        const uint32_t edge[] = {0u, 1u, d - 1, d, d + 1, 2 * d - 1, 0x7FFFFFFFu, 0x40000000u};
        for (uint32_t x : edge) CHECK(udiv_by(x, d, m) == x / d, "udiv %u/%u", x, d);
        for (int i = 0; i < 200000; ++i) {
            const uint32_t x = (uint32_t)(rng() & 0x7FFFFFFFu);
            CHECK(udiv_by(x, d, m) == x / d, "udiv %u/%u", x, d);
        }
    }
    // e = 4 dc + df orders moves as |V| dc + df (|df| <= 1, |V| >= 3)
    for (int nv = 3; nv <= 260; ++nv)
        for (int dc1 = -40; dc1 <= 40; ++dc1)
            for (int df1 = -1; df1 <= 1; ++df1)
                for (int dc2 = dc1 - 2; dc2 <= dc1 + 2; ++dc2)
                    for (int df2 = -1; df2 <= 1; ++df2)
                        CHECK((nv * dc1 + df1 < nv * dc2 + df2) ==
                                  (4 * dc1 + df1 < 4 * dc2 + df2),
                              "order nv=%d", nv);
    // aspiration: delta < F* - F  <=>  e < squeezed_bound
    const int nvs[] = {3, 4, 5, 64, 65, 200, 1250, 3430, 16129};
    for (int nv : nvs) {
        for (int i = 0; i < 20000; ++i) {
            const int fbest = (int)(rng() % (uint64_t)(nv + 1)), f = (int)(rng() % (uint64_t)(nv + 1));
            const int cbest = (int)(rng() % 200), c = (int)(rng() % 200);
            const int dfg = fbest - f, dcg = cbest - c;
            const int64_t thr = (int64_t)dfg + (int64_t)nv * dcg;
            const int32_t b = squeezed_bound(dfg, dcg, nv);
            const int q0 = (int)((thr >= 0 ? thr : thr - (nv - 1)) / nv);
            for (int dc = q0 - 3; dc <= q0 + 3; ++dc)
                for (int df = -1; df <= 1; ++df)
                    CHECK(((int64_t)nv * dc + df < thr) == (4 * dc + df < b),
                          "bound nv=%d dfg=%d dcg=%d dc=%d df=%d", nv, dfg, dcg, dc, df);
        }
    }
    // AUX threshold floor(x 2^32 / y), x < y, against 128-bit division: the
    // whole range of beta_num D (beta_num <= 10^6, D <= 16129)
    for (int i = 0; i < 2000000; ++i) {
        const uint64_t y = 1 + rng() % 16129000000ull;
        const uint64_t x = rng() % y;
        const uint64_t ref = (uint64_t)((((unsigned __int128)x) << 32) / y);
        CHECK(frac_shift32(x, y) == ref, "frac %llu/%llu", (unsigned long long)x,
              (unsigned long long)y);
    }
    for (uint64_t y : {1ull, 2ull, 3ull, 1250ull, 25000ull, 4294967295ull, 4294967296ull,
                       16129000000ull}) {
        for (uint64_t x : {(uint64_t)0, (uint64_t)1, y / 2, y - 1}) {
            if (x >= y) continue;
            const uint64_t ref = (uint64_t)((((unsigned __int128)x) << 32) / y);
            CHECK(frac_shift32(x, y) == ref, "frac edge %llu/%llu", (unsigned long long)x,
                  (unsigned long long)y);
        }
    }
    if (fails) {
        std::printf("FAILED %d\n", fails);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}

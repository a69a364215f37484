// CPU check of the host-only bookkeeping of libplse (host_books.h): the
// serving arena's first-fit placement and merging against a granule-by-
// granule model, and the sizing of a finished run's results by the device's
// count of generations run.  Built with g++ (and sanitizers) by
// tests/test_server_host.py; no GPU involved.
#include <cstdio>
#include <memory>
#include <random>
#include <vector>

#include "../paper_2103_10453_amd/csrc/host_books.h"

using namespace plse;

static int fails = 0;
#define CHECK(c, ...)                     \
    do {                                  \
        if (!(c)) {                       \
            if (fails++ < 20) {           \
                std::printf(__VA_ARGS__); \
                std::printf("\n");        \
            }                             \
        }                                 \
    } while (0)

// Lowest granule index of a run of `need` free granules, or -1.
static long model_first_fit(const std::vector<char> &used, size_t need) {
    size_t run = 0;
    for (size_t g = 0; g < used.size(); ++g) {
        run = used[g] ? 0 : run + 1;
        if (run == need) return (long)(g + 1 - need);
    }
    return -1;
}

static void check_arena(uint64_t seed) {
    std::mt19937_64 rng(seed);
    const size_t A = 256, G = 500 + rng() % 1500;
    const size_t budget = G * A + rng() % A;  // a ragged tail is never used
    FirstFitArena arena(budget, A);
    std::vector<char> used(G, 0);
    struct Blk { size_t off, bytes; };
    std::vector<Blk> live;
    for (int step = 0; step < 4000; ++step) {
        const bool add = live.empty() || rng() % 3 != 0;
        if (add) {
            const size_t bytes = 1 + rng() % (A * (1 + rng() % 120));
            const size_t need = (bytes + A - 1) / A;
            size_t off = 0;
            const bool ok = arena.place(bytes, &off);
            const long want = model_first_fit(used, need);
            CHECK(ok == (want >= 0), "seed %llu step %d: placed %d, model %ld",
                  (unsigned long long)seed, step, (int)ok, want);
            if (ok && want >= 0) {
                CHECK(off == (size_t)want * A, "seed %llu step %d: offset %zu, model %ld",
                      (unsigned long long)seed, step, off, want * (long)A);
                for (size_t g = off / A; g < off / A + need && g < G; ++g) {
                    CHECK(!used[g], "overlap at granule %zu", g);
                    used[g] = 1;
                }
                live.push_back({off, bytes});
            }
        } else {
            const size_t i = rng() % live.size();
            arena.release(live[i].off, live[i].bytes);
            const size_t need = (live[i].bytes + A - 1) / A;
            for (size_t g = live[i].off / A; g < live[i].off / A + need; ++g) used[g] = 0;
            live.erase(live.begin() + (long)i);
        }
        // free blocks are maximal, disjoint, in range, and cover the free granules
        size_t free_g = 0, prev_end = (size_t)-1;
        for (const auto &kv : arena.free_blocks()) {
            CHECK(kv.first % A == 0 && kv.second % A == 0 && kv.second > 0, "granules");
            CHECK(kv.first != prev_end, "adjacent free blocks not merged at %zu", kv.first);
            CHECK(kv.first + kv.second <= G * A, "block past the arena");
            for (size_t g = kv.first / A; g < (kv.first + kv.second) / A && g < G; ++g)
                CHECK(!used[g], "free block over a used granule %zu", g);
            free_g += kv.second / A;
            prev_end = kv.first + kv.second;
        }
        size_t model_free = 0;
        for (char u : used) model_free += !u;
        CHECK(free_g == model_free, "free granules %zu vs model %zu", free_g, model_free);
    }
    for (const Blk &b : live) arena.release(b.off, b.bytes);
    CHECK(arena.free_blocks().size() == 1 && arena.free_blocks().begin()->first == 0 &&
              arena.free_blocks().begin()->second == G * A,
          "released arena is not one block");
    CHECK(arena.could_fit(G * A, budget) && !arena.could_fit(G * A + 1, budget), "capacity");
}

static void check_results() {
    std::mt19937_64 rng(7);
    for (int trial = 0; trial < 300; ++trial) {
        // the device ran `gens` generations; the caller saw `seen` of them end
        const int gens = (int)(rng() % 40), seen = gens ? (int)(rng() % (gens + 1)) : 0;
        std::unique_ptr<GenStat[]> gs(new GenStat[(size_t)std::max(gens, 1)]);
        uint64_t tot[kCounters] = {};
        for (int g = 0; g < gens; ++g) {
            gs[g].best_f = 1000 - g;
            for (int q = 0; q < kCounters; ++q) {
                gs[g].cnt[q] = rng() % 1000;
                tot[q] += gs[g].cnt[q];
            }
        }
        Ctl c{};
        c.gens_run = gens;
        c.fstar = gens ? 1000 - gens + 1 : INT32_MAX;
        c.best_gen = gens ? 1 + (int)(rng() % gens) : 0;
        const RunResult r = summarize(c, gs.get(), gens);
        CHECK((int)r.gen_best.size() == gens && r.gen_cnt.size() == (size_t)gens * kCounters,
              "result sizes");
        CHECK(r.stats.generations_run == gens && r.stats.best_generation == c.best_gen, "stats");
        for (int q = 0; q < kCounters; ++q) CHECK(r.stats.totals[q] == tot[q], "totals");
        // generation end times: seen ones kept, drained ones completed
        std::vector<double> t;
        for (int g = 0; g < seen; ++g) t.push_back(0.5 + g);
        const double done = 100.0;
        const double tb = time_to_best(t, gens, c.best_gen, done);
        CHECK((int)t.size() == gens, "end times %zu for %d generations", t.size(), gens);
        if (c.best_gen >= 1)
            CHECK(tb == (c.best_gen <= seen ? 0.5 + (c.best_gen - 1) : done), "time to best");
        else
            CHECK(tb == done, "time to best without generations");
    }
    // the best grid of an n x n instance fills exactly n * n cells
    const int n = 5;
    std::vector<int> cell_v((size_t)n * n, -1);
    std::vector<int8_t> grid((size_t)n * n, 1);
    std::vector<uint8_t> star(3, 4);
    cell_v[3] = 0;
    cell_v[7] = 1;
    cell_v[11] = -2;
    cell_v[20] = 2;
    grid[3] = grid[7] = grid[11] = grid[20] = 0;
    std::unique_ptr<int8_t[]> out(new int8_t[(size_t)n * n]);
    CHECK(best_grid(n, cell_v, grid, star.data(), 1, out.get()) == n * n - 1, "filled");
    CHECK(best_grid(n, cell_v, grid, star.data(), 0, out.get()) == n * n - 4, "no generation");
}

int main() {
    for (uint64_t seed = 1; seed <= 12; ++seed) check_arena(seed);
    check_results();
    if (fails) {
        std::printf("FAILED %d\n", fails);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}

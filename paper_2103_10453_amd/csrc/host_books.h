// host_books.h -- host-only bookkeeping of libplse: the server's first-fit
// device arena, and the results of a finished run sized from the device's
// own count of generations run.  Plain C++ (no HIP calls), so the same code
// is exercised on the CPU, under sanitizers, by the test suite.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <iterator>
#include <map>
#include <vector>

#include "../../include/plse.h"
#include "plse_internal.h"

namespace plse {

// First-fit placement of workspaces in an arena of `budget` bytes (offsets and
// sizes in whole granules of `align` bytes); released blocks merge with free
// neighbours, so a fully released arena is one free block again.
class FirstFitArena {
public:
    FirstFitArena(size_t budget, size_t align) : align_(align) {
        const size_t usable = budget / align * align;
        if (usable) free_[0] = usable;
    }

    // Lowest offset of a free block that holds `bytes` (rounded up to the
    // granule); false when none does.
    bool place(size_t bytes, size_t *off) {
        bytes = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at2 = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at2] = rest;
            return true;
        }
        return false;
    }

    void release(size_t off, size_t bytes) {
        bytes = round(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

    // Whether a workspace of `bytes` could ever be placed (empty arena).
    bool could_fit(size_t bytes, size_t budget) const { return round(bytes) <= budget / align_ * align_; }

    const std::map<size_t, size_t> &free_blocks() const { return free_; }

private:
    size_t round(size_t b) const { return (b + align_ - 1) / align_ * align_; }
    size_t align_;
    std::map<size_t, size_t> free_;  // offset -> bytes
};

// Statistics of a run from the device's per-generation records: exactly
// `gens` records are read (the control block's count of generations run,
// which may exceed the generations a caller saw end).
struct RunResult {
    plse_stats stats{};
    std::vector<int32_t> gen_best;   // [gens]
    std::vector<uint64_t> gen_cnt;   // [gens][kCounters]
};

inline RunResult summarize(const Ctl &c, const GenStat *gs, int gens) {
    RunResult r;
    gens = std::max(gens, 0);
    r.gen_best.assign((size_t)gens, 0);
    r.gen_cnt.assign((size_t)gens * kCounters, 0);
    for (int g = 0; g < gens; ++g) {
        r.gen_best[g] = gs[g].best_f;
        for (int q = 0; q < kCounters; ++q) {
            r.gen_cnt[(size_t)g * kCounters + q] = gs[g].cnt[q];
            r.stats.totals[q] += gs[g].cnt[q];
        }
    }
    r.stats.generations_run = gens;
    r.stats.best_f = c.fstar;
    r.stats.best_generation = c.best_gen;
    r.stats.stop_reason = c.stop_reason;
    return r;
}

// The best grid: prefilled cells, then S* on the vertices (nothing when no
// generation has run); returns the number of non-zero cells.
inline int best_grid(int n, const std::vector<int> &cell_v, const std::vector<int8_t> &grid,
                     const uint8_t *star, int gens, int8_t *out) {
    int cnt = 0;
    for (int q = 0; q < n * n; ++q) {
        const int v = cell_v[q];
        const int8_t val = (v == -1) ? grid[q] : ((v >= 0 && gens > 0) ? (int8_t)star[v] : (int8_t)0);
        out[q] = val;
        cnt += (val != 0);
    }
    return cnt;
}

// End times of a served request's generations: those the worker saw end
// (t_gen), completed to `gens` with the time the request finished for the
// generations that ran after it last looked (queued generations drained at a
// cancel or a stop).  The time to the best is the end of its generation.
inline double time_to_best(std::vector<double> &t_gen, int gens, int best_gen, double t_done) {
    if ((int)t_gen.size() > gens) t_gen.resize((size_t)std::max(gens, 0));
    while ((int)t_gen.size() < gens) t_gen.push_back(t_done);
    return (best_gen >= 1 && best_gen <= (int)t_gen.size()) ? t_gen[(size_t)best_gen - 1] : t_done;
}

}  // namespace plse

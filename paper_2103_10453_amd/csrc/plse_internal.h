// plse_internal.h -- structures shared by the host orchestrator and the HIP
// kernels of libplse (gfx950).  Plain data only.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace plse {

constexpr int kHist = 64;        // partner-history slots per individual
constexpr int kCounters = 9;     // iters, moves, idle, cands, elig, nupd, snaps, repairs, cupd
constexpr int kAdj = 32;         // close-neighbour list capacity per candidate (select)
constexpr uint8_t kNoSlot = 0xFF;

// nupd: conflict-table entries a move changes (Section 3.3: every neighbour of
// the moved vertex, once per coloured end); cupd: the row/column counts that
// hold the same table in factored form (two per coloured end).
enum Counter { C_ITERS = 0, C_MOVES, C_IDLE, C_CANDS, C_ELIG, C_NUPD, C_SNAPS, C_REPAIRS, C_CUPD };

// Random-stream tags: which decision a Philox draw belongs to.
enum Tag : uint32_t {
    TAG_INIT_ORDER = 0x01,
    TAG_INIT_PICK = 0x02,
    TAG_PLITS1 = 0x11,
    TAG_PLITS2 = 0x12,
    TAG_PARTIAL = 0x13,
    TAG_SELECT = 0x21,
    TAG_XOVER = 0x31,
    TAG_MATCH = 0x41,
};

// Reduced graph of one instance, as device pointers into the workspace.
struct DevInstance {
    int32_t n, nv, nd, stride;       // order, |V|, sum |D*(v)|, row stride (bytes)
    int32_t l, ub;
    int32_t ts;                      // candidate row length: |D*(v)| + 1 <= ts, ts % 8 == 0
    int32_t pad;
    const uint16_t *vrc;             // [nv] row | column << 8
    const void *vrec;                // [nv] 32-byte records: D*(v) as a 128-bit colour
                                     //   mask, first slot offset, row | column << 8 |
                                     //   |D*(v)| << 16
    const uint32_t *vinfo;           // [nv] row | column << 8 | |D*(v)| << 16 | degree << 24
    const uint8_t *cand;             // [nv][ts] moves of v: 0 (uncolour), then D*(v)
                                     //   ascending; the last colour repeats to ts
    int32_t nl, pad2;                // neighbour list length per vertex, 2(n-1)
    const uint32_t *nbr;             // [nv][nl] the other vertices of v's row, then of
                                     //   its column: vertex | its other coordinate << 16 |
                                     //   column flag << 31 (degree entries used)
    const uint32_t *rcl;             // vertices of each row (vertex | column << 16), then
                                     //   of each column (vertex | row << 16), in order
    const uint32_t *rclo;            // [2n+1] offsets of those lists
};

struct Params {
    int64_t depth1, depth2;
    int64_t alpha_num, alpha_den;
    int64_t beta_num, beta_den;
    int64_t spacing;
    int64_t max_iters;  // > 0: iteration budget of a run (Section 4.3), checked per generation
    int32_t stop_at_ub;
    int32_t hist_len;
    int32_t crossover;  // 0 AUX (Alg. 5), 1 UX (p_ij = 1/2), 2 none (Section 5.2)
    int32_t matching;   // 0 nearest neighbour (Section 3.5.1), 1 random (Section 5.3)
    int32_t variant;    // 0 MPMA, 1 Partial-MPMA (Section 3.7)
};

// Device control block of a solve (one per handle).
struct Ctl {
    int32_t gen;          // current generation (1-based once started)
    int32_t stop;         // set when the bound is reached with stop_at_ub, or the budget
    int32_t fstar;        // best f so far (INT32_MAX before generation 1)
    int32_t best_gen;
    int32_t gens_run;
    int32_t stop_reason;  // 0 none, 1 bound reached, 2 iteration budget spent
    uint64_t iters;       // tabu iterations of the whole population so far
};

// Per-generation record.
struct GenStat {
    int32_t best_f;
    int32_t pad;
    uint64_t cnt[kCounters];
};

}  // namespace plse

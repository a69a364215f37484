// kernels.h -- argument blocks and launch entry points of the libplse HIP
// kernels (gfx950), shared by the kernels and the host orchestrator.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "plse_internal.h"

namespace plse {

// One launch serves up to kMaxLaunch instances: blockIdx.y selects the
// instance, whose argument block lives in its own workspace.
constexpr int kMaxLaunch = 128;
struct ArgList {
    const void *p[kMaxLaunch];
};

template <typename T>
__device__ __forceinline__ T arg_of(const ArgList &L) {
    return *static_cast<const T *>(L.p[blockIdx.y]);
}

struct FillArgs {
    uint32_t *p;
    size_t n;
};

struct PopSetupArgs {
    int32_t p, stride;
    uint64_t *uid;
    int32_t *hc;
    const uint8_t *S;
    uint8_t *S_off;
};

struct PlitsArgs {
    DevInstance I;
    Params P;
    const uint8_t *S_in;   // [p][stride]
    uint8_t *S_out;        // [p][stride]
    int32_t *f_out;        // [p]
    uint64_t *cnt_out;     // [p][kCounters]
    uint32_t *tabu;        // [p][nv][ts], all zero between phases
    const Ctl *ctl;        // generation and stop flag when gen_fixed == 0
    int32_t gen_fixed;
    int32_t p;
    uint32_t seed_lo, seed_hi;
    int32_t lds_per_wave;
    int32_t off_h, off_bm, off_tm, off_el, off_ring, off_hk, off_planes;
    int32_t nplanes;       // bit planes of floor(|D*(v)| / CH), at most 7
    // LDS-resident kernel: tabu marks, dirty set, per-word chunk offsets (the
    // stage is at off_el, 8 bytes per entry); npos = tabu mark positions
    int32_t off_mk, off_dirty, off_wpre, npos;
};

// Eligible vertices a PLITS bitmap scan stages for dealing (u16 each, LDS).
constexpr int kPlitsStage = 256;
// LDS-resident PLITS kernel: eligible vertices staged at a time, and the
// layout of its staging area: staged vertex ids (u16), 64 chunk-start flags,
// vertices joining the eligible list (u16), the row/column list offsets
// (2n + 1 u32, n <= 127).
constexpr int kLeanStage = 256;
constexpr int kLeanFlags = 2 * kLeanStage;
constexpr int kLeanIns = kLeanFlags + 64;
constexpr int kLeanRclo = kLeanIns + 2 * kLeanStage;
constexpr int kLeanAreaBytes = kLeanRclo + 4 * 256;

struct InitArgs {
    DevInstance I;
    uint8_t *S;            // [p][stride] out
    int32_t *f;            // [p] out
    int32_t p;
    int32_t pow2;          // power of two >= nv (sort size)
    uint32_t seed_lo, seed_hi;
};

struct BestArgs {
    Ctl *ctl;
    GenStat *stats;          // [max generations]
    const int32_t *f_new;    // [p]
    const uint8_t *S_new;    // [p][stride]
    const uint64_t *cnt;     // [p][kCounters]
    uint8_t *Sstar;          // [stride]
    int32_t p, stride, nsq_minus_l, ub, stop_at_ub;
    int64_t max_iters;       // > 0: stop once ctl->iters reaches it
};

struct PackArgs {
    const Ctl *ctl;
    const uint8_t *S;        // [rows][stride]
    uint32_t *planes;        // [rows][W][B]
    int32_t m, nv, stride, W, B;  // m: rows packed, from row row0
    int32_t row0;
};

struct DistArgs {
    const Ctl *ctl;
    const uint32_t *planes;  // [m][W][B]
    int16_t *D;              // [m][ld]
    int32_t m, W, ld, ntiles;  // ntiles: per side (ceil(m / kDistTile))
    int32_t tile0;             // first triangular tile index of the launch
};

constexpr int kDistTile = 64;  // rows and columns per distance tile

struct CloseArgs {
    const Ctl *ctl;
    const int16_t *D;
    int32_t *deg;
    uint16_t *adj;           // [m][kAdj]
    int32_t m, ld, nv;
    int64_t spacing;
};

struct SelectArgs {
    const Ctl *ctl;
    const int32_t *f_all;    // [m]
    const int16_t *D;        // [m][ld]
    const int32_t *deg;
    const uint16_t *adj;
    uint64_t *keys_g;        // [pow2] global scratch (when not in LDS)
    int32_t *rej;            // [m] scratch
    int32_t *acc;            // [p] out
    int32_t *pos;            // [m] out: -1 (the fill; gather sets accepted ones)
    int32_t p, m, ld, nv, pow2, keys_in_lds, gen_fixed;
    int64_t spacing;
    uint32_t seed_lo, seed_hi;
};

struct GatherArgs {
    const Ctl *ctl;
    const int32_t *acc;
    const uint8_t *S_all;    // [2p][stride]
    const int32_t *f_all;    // [2p]
    const uint64_t *uid;     // [p]
    const uint64_t *hist;    // [p][kHist]
    const int32_t *hc;       // [p]
    uint8_t *S_tmp;
    int32_t *f_tmp;
    uint64_t *uid_tmp, *hist_tmp;
    int32_t *hc_tmp;
    int32_t *pos;            // [m] new index of each accepted candidate
    int32_t p, stride;
};

struct HashArgs {
    const Ctl *ctl;
    const uint64_t *uid;     // [p]
    uint64_t *hkeys;         // [hsize]
    int32_t *hvals;
    int32_t p, hsize;
};

struct MatchArgs {
    const Ctl *ctl;
    const int16_t *D;        // distances, row/col through idx (identity if null)
    const int32_t *idx;      // [p] row of D of each individual
    const int32_t *pos;      // [m] individual of each row of D, -1 if none (with idx)
    const uint64_t *uid;
    uint64_t *hist;          // [p][kHist]
    int32_t *hc;
    const uint64_t *hkeys;
    const int32_t *hvals;
    int32_t *partner, *dpart;
    int32_t p, m, ld, hsize, hist_len;  // m: rows of D scanned through pos
    int32_t mode, gen_fixed;            // matching variant; generation (0: from ctl)
    uint32_t seed_lo, seed_hi;
};

struct AuxArgs {
    const Ctl *ctl;
    const uint8_t *S;        // [p][stride]
    const int32_t *partner, *dpart;
    uint8_t *S_off;          // [p][stride]
    int32_t p, nv, stride, gen_fixed;
    int32_t mode;            // crossover variant: 0 AUX, 1 UX, 2 none
    int64_t beta_num, beta_den;
    uint32_t seed_lo, seed_hi;
};

// Launch entry points: `L` lists the argument blocks (device addresses) of
// `count` instances; grid.y = count.
// partial: Partial-MPMA's search (repair, then PartialCol) instead of PLITS.
hipError_t launch_plits(const ArgList &L, int count, int p, int lds_per_wave,
                        int slots_per_lane, int waves_per_block, bool partial, bool lean,
                        hipStream_t stream);
const void *plits_fn(int slots_per_lane, bool partial);
// The LDS-resident PLITS kernel (MPMA only) of a chunk size; null for others.
const void *plits_lean_fn(int slots_per_lane);
hipError_t launch_fill_zero(const ArgList &L, int count, hipStream_t stream);
hipError_t plits_set_lds_limit(int bytes);
int plits_waves_per_cu(int slots_per_lane, int waves_per_block, int lds_per_wave, bool partial,
                       bool lean, bool persistent = false);
// Persistent PLITS over `count` instances of population p: `blocks` blocks
// take (instance, individual) items from *queue (zeroed first, by a kernel)
// until all count * p are done.
hipError_t launch_plits_persistent(const ArgList &L, int count, int p, int lds_per_wave,
                                   int slots_per_lane, int waves_per_block, bool partial,
                                   int blocks, uint32_t *queue, hipStream_t stream);
hipError_t launch_init(const ArgList &L, int count, int p, size_t lds, hipStream_t stream);
size_t init_lds_bytes(const DevInstance &I, int pow2);
hipError_t init_set_lds_limit(int bytes);
hipError_t launch_best(const ArgList &L, int count, hipStream_t stream);
hipError_t launch_pack(const ArgList &L, int count, size_t max_threads, hipStream_t stream);
// tiles: triangular tiles (I <= J) of the launch, from the arg block's tile0
hipError_t launch_dist(const ArgList &L, int count, long tiles, int B, hipStream_t stream);
hipError_t launch_close(const ArgList &L, int count, int m, hipStream_t stream);
hipError_t launch_select(const ArgList &L, int count, size_t lds, int pow2, bool keys_in_lds,
                         hipStream_t stream);
size_t select_lds_bytes(int m, int pow2, bool keys_in_lds);
hipError_t launch_gather(const ArgList &L, int count, int p, hipStream_t stream);
hipError_t launch_hash(const ArgList &L, int count, int p, int hsize, hipStream_t stream);
hipError_t launch_match(const ArgList &L, int count, int p, hipStream_t stream);
hipError_t launch_aux(const ArgList &L, int count, int p, hipStream_t stream);
hipError_t launch_ctl_reset(const ArgList &L, int count, hipStream_t stream);
hipError_t launch_gen_begin(const ArgList &L, int count, hipStream_t stream);
hipError_t launch_pop_setup(const ArgList &L, int count, hipStream_t stream);
hipError_t evo_set_lds_limit(int bytes);
// LDS read bandwidth measurement: *bytes receives the bytes one launch reads.
hipError_t launch_lds_read(int blocks, uint32_t iters, uint32_t *sink, hipStream_t stream,
                           double *bytes);

}  // namespace plse

// host.cpp -- libplse host side: instance preprocessing (Section 2.2, Alg. 1),
// workspace planning, sessions of one or many instances driving the
// per-generation HIP graphs (Alg. 2), and the C ABI of include/plse.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <cstddef>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/plse.h"
#include "host_books.h"
#include "kernels.h"

using namespace plse;

namespace {

constexpr size_t kAlign = 256;

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int next_pow2(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Bits needed for colours 0..n.
// Distance tiles (64 x 64, I <= J) that lie within P_t (rows 0..p-1).
long old_tiles(int p) {
    const long j0 = p / kDistTile;
    return j0 * (j0 + 1) / 2;
}

int colour_bits(int n) {
    int b = 0;
    while ((1 << b) <= n) ++b;
    return b;
}

// Offsets of every device array of one handle, for a population p.
struct Layout {
    size_t vrc, vrec, cand, vinfo, nbr, rcl, rclo;
    size_t args, ctl, stats, Sstar;
    size_t S_all, S_off, S_tmp, f_all, f_tmp, uid, uid_tmp, hist, hist_tmp, hc, hc_tmp, cnt;
    size_t tabu, planes, D, deg, adj, keys, rej, acc, pos, hkeys, hvals, partner, dpart;
    size_t queue;  // work queue of a persistent batched search launch led by this instance
    size_t total;
    int pow2_sel, hsize;
};

// Argument blocks of every kernel of one instance; a device copy lives in
// the instance's workspace and launches pass its address.
struct ArgBlock {
    PlitsArgs plits;
    InitArgs init;
    BestArgs best;
    PackArgs pack, pack_t;  // rows of P' (after the search), of P_t (beside it)
    DistArgs dist, dist_t;  // tiles involving P', tiles within P_t
    CloseArgs close;
    SelectArgs select;
    GatherArgs gather;
    HashArgs hash;
    MatchArgs match;
    AuxArgs aux;
    PopSetupArgs pop;
    FillArgs fill;
};

struct Session;

}  // namespace

struct plse_instance {
    int n = 0, nv = 0, l = 0, ub = 0, nd = 0, stride = 16;
    int dmax = 0, ts = 8;  // largest |D*(v)|; candidate row length (dmax + 1 rounded to 8)
    std::vector<int8_t> grid;
    std::vector<int> cell_v;  // -1 prefilled, -2 impossible, else vertex id
    // vertices of each row (vertex | column << 16), then of each column (vertex
    // | row << 16), in order; offsets of the 2n lists
    std::vector<uint32_t> rcl, rclo;
    // host images of the device instance tables
    std::vector<uint16_t> vrc;
    std::vector<uint32_t> vrec;  // 8 words per vertex
    std::vector<uint8_t> cand;   // [nv][ts] candidate rows: 0, D*(v) ascending, 0 padding
    std::vector<uint32_t> vinfo; // [nv] row | column << 8 | |D*(v)| << 16
    int nl = 0;                   // neighbour list length per vertex: 2(n-1)
    std::vector<uint32_t> nbr;    // [nv][nl] row then column vertices of v (not v):
                                  //   u | other coordinate << 16 | column flag << 31

    Params P{};
    int spl = 0;  // candidate positions per lane and round in PLITS; 0: automatic
    int wpb = 0;  // waves per block in PLITS; 0: automatic
    int kernel = 0;  // PLITS kernel: 0 automatic, 1 global tabu table, 2 LDS-resident
    int persistent = 1;  // batched searches: one persistent launch per group (0: a grid per instance)
    int fail_at = 0;  // serving test hook: end the request after this generation
    int max_gens = PLSE_MAX_GENERATIONS;  // generations a session may run (sizes its records)
    int sel_global = 0;  // test hook: sort selection keys in global memory when possible

    uint8_t *ws = nullptr;
    size_t ws_bytes = 0;
    Layout L{};
    ArgBlock args{};

    Session *own = nullptr;  // session of plse_begin / plse_step / plse_end
    bool in_session = false;

    plse_stats last{};
    std::vector<int32_t> gen_best;
    std::vector<uint64_t> gen_cnt;
    std::vector<float> ms_plits, ms_rest;
    int stage_timing = 0;           // time every stage of a generation (no graphs)
    std::vector<float> ms_stages;   // [generations][kStages] of the last session
    std::atomic<int> busy{0};
};

namespace {

thread_local std::string g_hip_error;

int hip_fail(hipError_t e, const char *what = nullptr) {
    g_hip_error = hipGetErrorString(e);
    if (what) g_hip_error += std::string(" in ") + what;
    return PLSE_E_HIP;
}

#define HIP_TRY(x)                                      \
    do {                                                \
        hipError_t e_ = (x);                            \
        if (e_ != hipSuccess) return hip_fail(e_, #x);  \
    } while (0)

#define RC_TRY(x)            \
    do {                     \
        const int rc_ = (x); \
        if (rc_) return rc_; \
    } while (0)

std::once_flag g_attr_once;
int g_lds_limit = 65536 - 1024;  // dynamic LDS per block every kernel may use

// Raise the dynamic-LDS limit of the kernels to the device's per-block LDS.
// If the runtime refuses, kernels keep the default 64 KiB and launch shapes
// are chosen within it.
void set_attributes_once() {
    std::call_once(g_attr_once, [] {
        int dev = 0, lds = 65536;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                hipSuccess)
            lds = 65536;
        if (lds > 65536 && plits_set_lds_limit(lds) == hipSuccess &&
            init_set_lds_limit(lds) == hipSuccess && evo_set_lds_limit(lds) == hipSuccess)
            g_lds_limit = lds - 1024;  // headroom for the kernels' static LDS
        else
            g_lds_limit = 65536 - 1024;
        (void)hipGetLastError();
    });
}

int max_lds_per_block() { return g_lds_limit; }

// Candidate positions per lane and round in PLITS: the chunk size CH that
// minimises the modelled evaluation work of one pass over every candidate
// row, sum_v ceil((d_v + 1) / CH) (CH + 3), the 3 standing for a chunk's
// fixed work (descriptor, vertex state, loads) in units of one move (fitted
// to measured runs: with 1.5 the model picked 4 for the 70x70 grid 70 %
// prefilled, which runs 7 % faster with 8).
int choose_spl(const plse_instance *h) {
    if (h->spl) return h->spl;
    int pick = 4;
    double best = 0.0;
    for (int ch : {2, 4, 8}) {
        double cost = 0.0;
        for (int v = 0; v < h->nv; ++v) cost += (double)((((h->vinfo[v] >> 16) & 0xFFu) + ch) / ch) * (ch + 3.0);
        if (ch == 2 || cost < best) {
            best = cost;
            pick = ch;
        }
    }
    return pick;
}

// PLITS per-wave LDS: S, row/column colour counts, eligibility bitmap,
// per-vertex relative tabu expiry marks (u8), kPlitsStage staged eligible
// vertices, ring of chunk descriptors (one group of 64 vertices dealt while
// under 64 are pending), colour halves of the tie values (u16 per colour),
// bit planes of the chunk counts.
struct PlitsLds {
    int per_wave, off_h, off_bm, off_tm, off_el, off_ring, off_hk, off_planes;
    int nplanes;
    bool lean = false;  // the LDS-resident kernel
    int off_mk = 0, off_dirty = 0, off_wpre = 0, npos = 0;
};

// Per-wave LDS the automatic choice allows the LDS-resident kernel (at least
// four resident waves per CU).
constexpr int kLeanMaxPerWave = 40 * 1024;

// LDS-resident PLITS per wave: S, row/column colour counts, eligibility
// bitmap, one tabu mark per candidate move (rows padded to CH), the dirty
// set, chunk-count planes, per-word chunk offsets, the staging area (staged
// eligible vertices, chunk-start flags, joining vertices, row/column list
// offsets) and the colour halves of the tie values.
PlitsLds plits_lean_layout(const plse_instance *h, int ch) {
    PlitsLds L{};
    const int W = (h->nv + 31) / 32;
    long npos = 0;
    for (int v = 0; v < h->nv; ++v) npos += (long)(((h->vinfo[v] >> 16) & 0xFFu) / ch + 1) * ch;
    L.lean = true;
    L.npos = (int)std::min<long>(npos, 1L << 30);
    L.nplanes = 0;
    while ((h->dmax / ch) >> L.nplanes) ++L.nplanes;
    L.off_h = h->stride;
    L.off_bm = L.off_h + (int)round_up((size_t)2 * h->n * (h->n + 1), 16);
    L.off_mk = L.off_bm + (int)round_up((size_t)W * 4, 16);
    L.off_dirty = L.off_mk + (int)round_up((size_t)L.npos, 16);
    L.off_planes = L.off_dirty + (int)round_up((size_t)W * 4, 16);
    L.off_wpre = L.off_planes + (int)round_up((size_t)L.nplanes * W * 4, 16);
    L.off_el = L.off_wpre + (int)round_up((size_t)W * 4, 16);
    L.off_hk = L.off_el + kLeanAreaBytes;
    L.per_wave = L.off_hk + (int)round_up((size_t)2 * (h->n + 1), 16);
    L.off_tm = L.off_ring = 0;
    return L;
}

PlitsLds plits_lds(const plse_instance *h) {
    PlitsLds L;
    const int W = (h->nv + 31) / 32;
    const int ch = choose_spl(h);
    if (h->P.variant == 0 && h->kernel == 2 && h->nv < 65536) {
        const PlitsLds Ln = plits_lean_layout(h, ch);
        if (Ln.per_wave <= max_lds_per_block()) return Ln;
    }
    const int qcap = 64 * ((h->dmax + ch) / ch);  // 64 vertices' chunks
    L.off_h = h->stride;
    L.off_bm = L.off_h + (int)round_up((size_t)2 * h->n * (h->n + 1), 16);
    L.off_tm = L.off_bm + (int)round_up((size_t)W * 4, 16);
    L.off_el = L.off_tm + (int)round_up((size_t)h->nv, 16);
    L.off_ring = L.off_el + 2 * kPlitsStage;
    L.off_hk = L.off_ring + qcap * 4;
    L.off_planes = L.off_hk + (int)round_up((size_t)2 * (h->n + 1), 16);
    L.nplanes = 0;
    while ((h->dmax / ch) >> L.nplanes) ++L.nplanes;
    L.per_wave = L.off_planes + (int)round_up((size_t)L.nplanes * W * 4, 16);
    return L;
}

// Waves per block: the most resident waves per CU for every chunk size in
// use; among equals the fewest waves per block, since a block keeps its LDS
// until its slowest wave ends and searches end at very different times.
int auto_wpb(int per_wave, const std::vector<int> &spls, bool partial, bool lean) {
    const int lim = max_lds_per_block();
    int best = 1, best_waves = -1;
    for (int w : {1, 2, 4}) {
        if (w * per_wave > lim) continue;
        int waves = 1 << 30;
        for (int spl : spls)
            waves = std::min(waves, plits_waves_per_cu(spl, w, per_wave, partial, lean));
        if (waves > best_waves) {
            best = w;
            best_waves = waves;
        }
    }
    return best;
}

int choose_wpb(const plse_instance *h) {
    const PlitsLds pl = plits_lds(h);
    return h->wpb ? h->wpb : auto_wpb(pl.per_wave, {choose_spl(h)}, h->P.variant != 0, pl.lean);
}

Layout plan(const plse_instance *h, int p) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = round_up(o + std::max<size_t>(bytes, 1), kAlign);
        return at;
    };
    const size_t nv = h->nv, n = h->n, nd = h->nd, st = h->stride;
    const size_t m = 2 * (size_t)p;
    const int W = (h->nv + 31) / 32, B = colour_bits(h->n);
    L.vrc = take(2 * nv);
    L.vrec = take(32 * nv);
    L.cand = take(nv * (size_t)h->ts);
    L.vinfo = take(4 * nv);
    L.nbr = take(4 * nv * (size_t)std::max(h->nl, 1));
    L.rcl = take(4 * h->rcl.size());
    L.rclo = take(4 * h->rclo.size());
    L.args = take(sizeof(ArgBlock));
    L.ctl = take(sizeof(Ctl));
    L.stats = take(sizeof(GenStat) * (size_t)h->max_gens);
    L.Sstar = take(st);
    L.S_all = take(m * st);
    L.S_off = take((size_t)p * st);
    L.S_tmp = take((size_t)p * st);
    L.f_all = take(4 * m);
    L.f_tmp = take(4 * (size_t)p);
    L.uid = take(8 * (size_t)p);
    L.uid_tmp = take(8 * (size_t)p);
    L.hist = take(8 * (size_t)p * kHist);
    L.hist_tmp = take(8 * (size_t)p * kHist);
    L.hc = take(4 * (size_t)p);
    L.hc_tmp = take(4 * (size_t)p);
    L.cnt = take(8 * (size_t)p * kCounters);
    L.tabu = take((size_t)p * nv * h->ts * 4);
    L.planes = take(m * W * B * 4);
    L.D = take(m * m * 2);
    L.deg = take(4 * m);
    L.adj = take(2 * m * kAdj);
    L.pow2_sel = next_pow2(std::max<int>(4, (int)m));
    L.keys = take(8 * (size_t)L.pow2_sel);
    L.rej = take(4 * m);
    L.acc = take(4 * (size_t)p);
    L.pos = take(4 * m);
    L.hsize = next_pow2(std::max<int>(4, (int)m));
    L.hkeys = take(8 * (size_t)L.hsize);
    L.hvals = take(4 * (size_t)L.hsize);
    L.partner = take(4 * (size_t)p);
    L.dpart = take(4 * (size_t)p);
    L.queue = take(64);
    L.total = o;
    return L;
}

template <typename T>
T *at(plse_instance *h, size_t off) {
    return reinterpret_cast<T *>(h->ws + off);
}

DevInstance dev_instance(plse_instance *h) {
    const Layout &L = h->L;
    DevInstance I;
    I.n = h->n;
    I.nv = h->nv;
    I.nd = h->nd;
    I.ts = h->ts;
    I.stride = h->stride;
    I.l = h->l;
    I.ub = h->ub;
    I.vrc = at<uint16_t>(h, L.vrc);
    I.vrec = at<void>(h, L.vrec);
    I.cand = at<uint8_t>(h, L.cand);
    I.vinfo = at<uint32_t>(h, L.vinfo);
    I.nl = h->nl;
    I.nbr = at<uint32_t>(h, L.nbr);
    I.rcl = at<uint32_t>(h, L.rcl);
    I.rclo = at<uint32_t>(h, L.rclo);
    return I;
}

int upload_instance(plse_instance *h, hipStream_t s) {
    const Layout &L = h->L;
    auto put = [&](size_t off, const void *src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync(h->ws + off, src, bytes, hipMemcpyHostToDevice, s);
    };
    HIP_TRY(put(L.vrc, h->vrc.data(), 2 * h->vrc.size()));
    HIP_TRY(put(L.vrec, h->vrec.data(), 4 * h->vrec.size()));
    HIP_TRY(put(L.cand, h->cand.data(), h->cand.size()));
    HIP_TRY(put(L.vinfo, h->vinfo.data(), 4 * h->vinfo.size()));
    HIP_TRY(put(L.nbr, h->nbr.data(), 4 * h->nbr.size()));
    HIP_TRY(put(L.rcl, h->rcl.data(), 4 * h->rcl.size()));
    HIP_TRY(put(L.rclo, h->rclo.data(), 4 * h->rclo.size()));
    return PLSE_OK;
}

int upload_args(plse_instance *h, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(h->ws + h->L.args, &h->args, sizeof(ArgBlock), hipMemcpyHostToDevice,
                           s));
    return PLSE_OK;
}

// Device address of one argument block of h.
template <typename M>
const void *dev_arg(plse_instance *h, M ArgBlock::*member) {
    const size_t off = (size_t)(reinterpret_cast<const char *>(&(h->args.*member)) -
                                reinterpret_cast<const char *>(&h->args));
    return h->ws + h->L.args + off;
}

PlitsArgs make_plits(plse_instance *h, int p, int gen_fixed, uint64_t seed,
                     const uint8_t *S_in, uint8_t *S_out, int32_t *f_out, uint64_t *cnt,
                     const Ctl *ctl) {
    PlitsArgs a{};
    a.I = dev_instance(h);
    a.P = h->P;
    a.S_in = S_in;
    a.S_out = S_out;
    a.f_out = f_out;
    a.cnt_out = cnt;
    a.tabu = at<uint32_t>(h, h->L.tabu);
    a.ctl = ctl;
    a.gen_fixed = gen_fixed;
    a.p = p;
    a.seed_lo = (uint32_t)seed;
    a.seed_hi = (uint32_t)(seed >> 32);
    const PlitsLds pl = plits_lds(h);
    a.lds_per_wave = pl.per_wave;
    a.off_h = pl.off_h;
    a.off_bm = pl.off_bm;
    a.off_tm = pl.off_tm;
    a.off_el = pl.off_el;
    a.off_ring = pl.off_ring;
    a.off_hk = pl.off_hk;
    a.off_planes = pl.off_planes;
    a.nplanes = pl.nplanes;
    a.off_mk = pl.off_mk;
    a.off_dirty = pl.off_dirty;
    a.off_wpre = pl.off_wpre;
    a.npos = pl.npos;
    return a;
}

SelectArgs make_select(plse_instance *h, int p, int gen_fixed, uint64_t seed, const Ctl *ctl,
                       const int32_t *f_all, const int16_t *D, int ld, int32_t *acc) {
    const Layout &L = h->L;
    SelectArgs a{};
    a.ctl = ctl;
    a.f_all = f_all;
    a.D = D;
    a.deg = at<int32_t>(h, L.deg);
    a.adj = at<uint16_t>(h, L.adj);
    a.keys_g = at<uint64_t>(h, L.keys);
    a.rej = at<int32_t>(h, L.rej);
    a.acc = acc;
    a.pos = at<int32_t>(h, L.pos);
    a.p = p;
    a.m = 2 * p;
    a.ld = ld;
    a.nv = h->nv;
    a.pow2 = L.pow2_sel;
    // keys in LDS when they fit; the global-memory sort needs at least two
    // 4096-key tiles
    const bool fits = select_lds_bytes(2 * p, L.pow2_sel, true) <= (size_t)max_lds_per_block();
    a.keys_in_lds = (fits && !(h->sel_global && L.pow2_sel >= 8192)) || L.pow2_sel < 8192 ? 1 : 0;
    a.gen_fixed = gen_fixed;
    a.spacing = h->P.spacing;
    a.seed_lo = (uint32_t)seed;
    a.seed_hi = (uint32_t)(seed >> 32);
    return a;
}

size_t select_lds(plse_instance *h, int p) {
    return select_lds_bytes(2 * p, h->L.pow2_sel, h->args.select.keys_in_lds != 0);
}

// Argument blocks of the whole pipeline of a solve with population p.
void build_pipeline_args(plse_instance *h, int p, uint64_t seed) {
    const Layout &L = h->L;
    ArgBlock &A = h->args;
    const int st = h->stride, m = 2 * p;
    Ctl *ctl = at<Ctl>(h, L.ctl);
    uint8_t *S_all = at<uint8_t>(h, L.S_all);
    uint8_t *S_new = S_all + (size_t)p * st;
    int32_t *f_all = at<int32_t>(h, L.f_all);
    const uint32_t slo = (uint32_t)seed, shi = (uint32_t)(seed >> 32);
    A.init = InitArgs{dev_instance(h), S_all, f_all, p, next_pow2(std::max(4, h->nv)), slo, shi};
    A.pop = PopSetupArgs{p, st, at<uint64_t>(h, L.uid), at<int32_t>(h, L.hc), S_all,
                         at<uint8_t>(h, L.S_off)};
    A.fill = FillArgs{at<uint32_t>(h, L.tabu), (size_t)p * h->nv * h->ts};
    A.plits = make_plits(h, p, 0, seed, at<uint8_t>(h, L.S_off), S_new, f_all + p,
                         at<uint64_t>(h, L.cnt), ctl);
    A.best = BestArgs{ctl, at<GenStat>(h, L.stats), f_all + p, S_new, at<uint64_t>(h, L.cnt),
                      at<uint8_t>(h, L.Sstar), p, st, h->n * h->n - h->l, h->ub,
                      h->P.stop_at_ub, h->P.max_iters};
    const int W = (h->nv + 31) / 32;
    // distances among P_t (rows 0..p-1) need nothing from this generation's
    // searches, so they are packed and computed beside them; the rest after
    const int B = colour_bits(h->n);
    // (with no tile within P_t, p < 64, the rest packs all 2p rows)
    const bool split = old_tiles(p) > 0;
    A.pack_t = PackArgs{ctl, S_all, at<uint32_t>(h, L.planes), p, h->nv, st, W, B, 0};
    A.pack = split ? PackArgs{ctl, S_all, at<uint32_t>(h, L.planes), p, h->nv, st, W, B, p}
                   : PackArgs{ctl, S_all, at<uint32_t>(h, L.planes), m, h->nv, st, W, B, 0};
    const int nt1 = (m + kDistTile - 1) / kDistTile;
    A.dist_t = DistArgs{ctl, at<uint32_t>(h, L.planes), at<int16_t>(h, L.D), m, W, m, nt1, 0};
    A.dist = DistArgs{ctl, at<uint32_t>(h, L.planes), at<int16_t>(h, L.D), m, W, m, nt1,
                      (int32_t)old_tiles(p)};
    A.close = CloseArgs{ctl, at<int16_t>(h, L.D), at<int32_t>(h, L.deg), at<uint16_t>(h, L.adj),
                        m, m, h->nv, h->P.spacing};
    A.select = make_select(h, p, 0, seed, ctl, f_all, at<int16_t>(h, L.D), m,
                           at<int32_t>(h, L.acc));
    A.gather = GatherArgs{ctl, at<int32_t>(h, L.acc), S_all, f_all, at<uint64_t>(h, L.uid),
                          at<uint64_t>(h, L.hist), at<int32_t>(h, L.hc), at<uint8_t>(h, L.S_tmp),
                          at<int32_t>(h, L.f_tmp), at<uint64_t>(h, L.uid_tmp),
                          at<uint64_t>(h, L.hist_tmp), at<int32_t>(h, L.hc_tmp),
                          at<int32_t>(h, L.pos), p, st};
    A.hash = HashArgs{ctl, at<uint64_t>(h, L.uid), at<uint64_t>(h, L.hkeys),
                      at<int32_t>(h, L.hvals), p, L.hsize};
    A.match = MatchArgs{ctl, at<int16_t>(h, L.D), at<int32_t>(h, L.acc), at<int32_t>(h, L.pos),
                        at<uint64_t>(h, L.uid), at<uint64_t>(h, L.hist), at<int32_t>(h, L.hc),
                        at<uint64_t>(h, L.hkeys), at<int32_t>(h, L.hvals),
                        at<int32_t>(h, L.partner), at<int32_t>(h, L.dpart), p, m, m, L.hsize,
                        h->P.hist_len, h->P.matching, 0, slo, shi};
    A.aux = AuxArgs{ctl, S_all, at<int32_t>(h, L.partner), at<int32_t>(h, L.dpart),
                    at<uint8_t>(h, L.S_off), p, h->nv, st, 0, h->P.crossover, h->P.beta_num,
                    h->P.beta_den, slo, shi};
}

// Launch `fn` over the instances `hs`, kMaxLaunch at a time.
template <typename M, typename F>
int launch_over(const std::vector<plse_instance *> &hs, M ArgBlock::*member, F &&fn) {
    for (size_t b = 0; b < hs.size(); b += kMaxLaunch) {
        ArgList L{};
        const int count = (int)std::min<size_t>(kMaxLaunch, hs.size() - b);
        for (int i = 0; i < count; ++i) L.p[i] = dev_arg(hs[b + i], member);
        HIP_TRY(fn(L, count));
    }
    return PLSE_OK;
}

int launch_ctl(const std::vector<plse_instance *> &hs, bool reset, hipStream_t s) {
    for (size_t b = 0; b < hs.size(); b += kMaxLaunch) {
        ArgList L{};
        const int count = (int)std::min<size_t>(kMaxLaunch, hs.size() - b);
        for (int i = 0; i < count; ++i) L.p[i] = at<Ctl>(hs[b + i], hs[b + i]->L.ctl);
        if (reset)
            HIP_TRY(launch_ctl_reset(L, count, s));
        else
            HIP_TRY(launch_gen_begin(L, count, s));
    }
    return PLSE_OK;
}

// Instances whose PLITS launches share a shape: chunk size and resident
// waves per CU at their own LDS footprint.  One launch per group (per
// kMaxLaunch instances) with the group's largest footprint, so a small
// instance never runs at the occupancy of a large one.
struct PlitsGroup {
    int spl = 8, occ = 0, lds = 0, wpb = 1;
    bool partial = false, lean = false;
    // several instances: one persistent launch (per kMaxLaunch instances)
    // whose waves take (instance, individual) items longest first
    bool persistent = false;
    int blocks = 0;
    std::vector<plse_instance *> hs;
};

// Stages of a generation timed by the stage-timing mode (plse_last_stage_timing).
constexpr int kStages = 7;

// A solve over one or many instances sharing the population size.
struct Session {
    std::vector<plse_instance *> hs;  // launch order: longest estimated work first
    int p = 0;
    int steps = 0;  // generations stepped in this session
    int base = 0;   // generations run before it (a session resumed from a checkpoint)
    uint64_t seed = 0;  // single-instance sessions
    std::vector<PlitsGroup> groups;  // largest estimated work first
    hipGraphExec_t ls = nullptr, rest = nullptr;  // a generation's searches; the rest
    std::vector<hipEvent_t> ev;                   // 3 per generation
    bool staged = false;                          // stage timing: kStages + 1 events per generation
    std::vector<hipEvent_t> sev;
    std::vector<hipStream_t> side;                // groups 1.. of a generation
    std::vector<hipEvent_t> fork;                 // 1 + one per side stream
    // distances among P_t, beside the searches: graph, stream, fork / join
    hipGraphExec_t dold = nullptr;
    hipStream_t dstream = nullptr;
    hipEvent_t dfork = nullptr, djoin = nullptr;
    // pinned host copies of the (single) instance's stop flag when set: the
    // flag after generation index gi (0-based) lands in stop_host[gi %
    // kStopRing] before that generation's end event (serving: retire stopped
    // runs early).  A reader of generation gi's slot must have fewer than
    // kStopRing generations enqueued beyond gi.
    static constexpr int kStopRing = 8;
    int32_t *stop_host = nullptr;

    ~Session() {
        if (stop_host) (void)hipHostFree(stop_host);
        if (dstream) {
            (void)hipStreamSynchronize(dstream);
            (void)hipStreamDestroy(dstream);
        }
        if (dold) (void)hipGraphExecDestroy(dold);
        if (dfork) (void)hipEventDestroy(dfork);
        if (djoin) (void)hipEventDestroy(djoin);
        if (ls) (void)hipGraphExecDestroy(ls);
        if (rest) (void)hipGraphExecDestroy(rest);
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        for (hipEvent_t e : sev) (void)hipEventDestroy(e);
        for (hipStream_t q : side) {
            (void)hipStreamSynchronize(q);
            (void)hipStreamDestroy(q);
        }
        for (hipEvent_t e : fork) (void)hipEventDestroy(e);
    }
};

int launch_group(const Session &S, const PlitsGroup &g, hipStream_t s) {
    if (g.persistent) {
        for (size_t b = 0; b < g.hs.size(); b += kMaxLaunch) {
            ArgList L{};
            const int count = (int)std::min<size_t>(kMaxLaunch, g.hs.size() - b);
            for (int i = 0; i < count; ++i) L.p[i] = dev_arg(g.hs[b + i], &ArgBlock::plits);
            plse_instance *lead = g.hs[b];
            HIP_TRY(launch_plits_persistent(L, count, S.p, g.lds, g.spl, g.wpb, g.partial,
                                            g.blocks, at<uint32_t>(lead, lead->L.queue), s));
        }
        return PLSE_OK;
    }
    return launch_over(g.hs, &ArgBlock::plits, [&](const ArgList &L, int c) {
        return launch_plits(L, c, S.p, g.lds, g.spl, g.wpb, g.partial, g.lean, s);
    });
}

int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0, c = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
            cus = c;
        (void)hipGetLastError();
    }
    return cus > 0 ? cus : 256;
}

// One generation's tabu searches.  Several groups run concurrently: group 0
// on `s`, the others on side streams forked from and joined back into `s`
// (captured, they become the parallel branches of the generation's graph).
int enqueue_local_search(Session &S, hipStream_t s) {
    RC_TRY(launch_ctl(S.hs, false, s));
    if (S.groups.size() == 1) return launch_group(S, S.groups[0], s);
    const size_t ns = S.groups.size() - 1;
    while (S.side.size() < ns) {
        hipStream_t q = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
        S.side.push_back(q);
    }
    while (S.fork.size() < ns + 1) {
        hipEvent_t e = nullptr;
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        S.fork.push_back(e);
    }
    HIP_TRY(hipEventRecord(S.fork[0], s));
    for (size_t i = 0; i < ns; ++i) {
        HIP_TRY(hipStreamWaitEvent(S.side[i], S.fork[0], 0));
        RC_TRY(launch_group(S, S.groups[i + 1], S.side[i]));
        HIP_TRY(hipEventRecord(S.fork[i + 1], S.side[i]));
    }
    RC_TRY(launch_group(S, S.groups[0], s));
    for (size_t i = 0; i < ns; ++i) HIP_TRY(hipStreamWaitEvent(s, S.fork[i + 1], 0));
    return PLSE_OK;
}

// Bit planes of one half of P^all and the distance tiles of one tile range.
int enqueue_pack_dist(Session &S, PackArgs ArgBlock::*pk, DistArgs ArgBlock::*dt, int rows,
                      long tiles, hipStream_t s) {
    size_t pack_threads = 0;
    for (plse_instance *h : S.hs)
        pack_threads = std::max(pack_threads, (size_t)rows * ((h->nv + 31) / 32));
    RC_TRY(launch_over(S.hs, pk, [&](const ArgList &L, int c) {
        return launch_pack(L, c, pack_threads, s);
    }));
    for (int B = 1; B <= 7; ++B) {
        std::vector<plse_instance *> g;
        for (plse_instance *h : S.hs)
            if (colour_bits(h->n) == B) g.push_back(h);
        if (g.empty()) continue;
        RC_TRY(launch_over(g, dt, [&](const ArgList &L, int c) {
            return launch_dist(L, c, tiles, B, s);
        }));
    }
    return PLSE_OK;
}

// Distances among P_t, beside the generation's searches.
int enqueue_old_dist(Session &S, hipStream_t s) {
    return enqueue_pack_dist(S, &ArgBlock::pack_t, &ArgBlock::dist_t, S.p, old_tiles(S.p), s);
}

// The generation's stages after the searches.  `mark` (may be null) records
// an event after each stage: best, distances with P', selection (close,
// select, gather), matching (hash, match); the crossover ends the sequence.
int enqueue_rest(Session &S, hipStream_t s, hipEvent_t *mark = nullptr) {
    const int p = S.p, m = 2 * p;
    RC_TRY(launch_over(S.hs, &ArgBlock::best,
                       [&](const ArgList &L, int c) { return launch_best(L, c, s); }));
    if (mark) HIP_TRY(hipEventRecord(mark[0], s));
    const long nt1 = (m + kDistTile - 1) / kDistTile;
    RC_TRY(enqueue_pack_dist(S, &ArgBlock::pack, &ArgBlock::dist, old_tiles(p) > 0 ? p : m,
                             nt1 * (nt1 + 1) / 2 - old_tiles(p), s));
    if (mark) HIP_TRY(hipEventRecord(mark[1], s));
    RC_TRY(launch_over(S.hs, &ArgBlock::close,
                       [&](const ArgList &L, int c) { return launch_close(L, c, m, s); }));
    const size_t sl = select_lds(S.hs[0], p);
    const int pow2 = S.hs[0]->L.pow2_sel;
    const bool keys_lds = S.hs[0]->args.select.keys_in_lds != 0;
    RC_TRY(launch_over(S.hs, &ArgBlock::select, [&](const ArgList &L, int c) {
        return launch_select(L, c, sl, pow2, keys_lds, s);
    }));
    RC_TRY(launch_over(S.hs, &ArgBlock::gather,
                       [&](const ArgList &L, int c) { return launch_gather(L, c, p, s); }));
    if (mark) HIP_TRY(hipEventRecord(mark[2], s));
    const int hsize = S.hs[0]->L.hsize;
    RC_TRY(launch_over(S.hs, &ArgBlock::hash,
                       [&](const ArgList &L, int c) { return launch_hash(L, c, p, hsize, s); }));
    RC_TRY(launch_over(S.hs, &ArgBlock::match,
                       [&](const ArgList &L, int c) { return launch_match(L, c, p, s); }));
    if (mark) HIP_TRY(hipEventRecord(mark[3], s));
    RC_TRY(launch_over(S.hs, &ArgBlock::aux,
                       [&](const ArgList &L, int c) { return launch_aux(L, c, p, s); }));
    return PLSE_OK;
}

template <typename F>
int capture(F &&enqueue, hipGraphExec_t *out) {
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    const int rc = enqueue(cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        *out = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    return PLSE_OK;
}

// Estimated work per generation of one individual: depth x mean domain size.
double work_estimate(const plse_instance *h) {
    return (double)(h->P.depth1 + h->P.depth2) * (1.0 + (h->nv ? (double)h->nd / h->nv : 0.0));
}

int check_ws(plse_instance *h, int p) {
    if (p < 2 || p > PLSE_MAX_POPULATION) return PLSE_E_ARG;
    h->L = plan(h, p);
    if (!h->ws || h->ws_bytes < h->L.total) return PLSE_E_WORKSPACE;
    set_attributes_once();
    return PLSE_OK;
}

// Upload tables and argument blocks of new instances (workspaces attached),
// then build their initial populations P_1: batched launches.
int admit(const std::vector<plse_instance *> &hs, int p, const uint64_t *seeds, hipStream_t s) {
    for (size_t i = 0; i < hs.size(); ++i) {
        plse_instance *h = hs[i];
        RC_TRY(check_ws(h, p));
        build_pipeline_args(h, p, seeds[i]);
        RC_TRY(upload_instance(h, s));
        RC_TRY(upload_args(h, s));
    }
    RC_TRY(launch_ctl(hs, true, s));
    size_t init_lds = 0;
    for (plse_instance *h : hs)
        init_lds = std::max(init_lds, init_lds_bytes(dev_instance(h), next_pow2(std::max(4, h->nv))));
    RC_TRY(launch_over(hs, &ArgBlock::init,
                       [&](const ArgList &L, int c) { return launch_init(L, c, p, init_lds, s); }));
    RC_TRY(launch_over(hs, &ArgBlock::pop,
                       [&](const ArgList &L, int c) { return launch_pop_setup(L, c, s); }));
    RC_TRY(launch_over(hs, &ArgBlock::fill,
                       [&](const ArgList &L, int c) { return launch_fill_zero(L, c, s); }));
    return PLSE_OK;
}

// Launch order (longest estimated work first) and the PLITS launch groups.
void shape_session(Session &S) {
    std::stable_sort(S.hs.begin(), S.hs.end(), [](const plse_instance *a, const plse_instance *b) {
        return work_estimate(a) > work_estimate(b);
    });
    S.groups.clear();
    for (plse_instance *h : S.hs) {
        const PlitsLds pl = plits_lds(h);
        const int spl = choose_spl(h), per = pl.per_wave;
        const bool partial = h->P.variant != 0, lean = pl.lean;
        const int occ = plits_waves_per_cu(spl, 1, per, partial, lean);
        auto it = std::find_if(S.groups.begin(), S.groups.end(), [&](const PlitsGroup &g) {
            return g.spl == spl && g.occ == occ && g.partial == partial && g.lean == lean;
        });
        if (it == S.groups.end()) {
            S.groups.push_back(PlitsGroup{});
            it = S.groups.end() - 1;
            it->spl = spl;
            it->occ = occ;
            it->partial = partial;
            it->lean = lean;
        }
        it->lds = std::max(it->lds, per);
        it->hs.push_back(h);
    }
    for (PlitsGroup &g : S.groups) {
        bool same_wpb = true;
        for (plse_instance *h : g.hs) same_wpb = same_wpb && h->wpb == g.hs[0]->wpb;
        g.wpb = (same_wpb && g.hs[0]->wpb) ? g.hs[0]->wpb
                                            : auto_wpb(g.lds, {g.spl}, g.partial, g.lean);
        if (g.wpb * g.lds > max_lds_per_block()) g.wpb = 1;
        bool all_persistent = true;
        for (plse_instance *h : g.hs) all_persistent = all_persistent && h->persistent != 0;
        g.persistent = g.hs.size() > 1 && !g.lean && all_persistent;
        if (g.persistent) {
            const int occ = plits_waves_per_cu(g.spl, g.wpb, g.lds, g.partial, false, true);
            g.blocks = std::max(1, occ * device_cus() / g.wpb);
        }
    }
}

// Upload, initial population P_1 and generation graphs of a session.
int session_begin(Session &S, const uint64_t *seeds, hipStream_t s) {
    RC_TRY(admit(S.hs, S.p, seeds, s));
    shape_session(S);
    // a generation's searches are one graph (several groups: forked branches
    // that run side by side), the rest another
    S.staged = S.hs.size() == 1 && S.hs[0]->stage_timing != 0;
    if (S.staged) {
        S.steps = 0;
        return PLSE_OK;  // stages enqueued one by one, each bracketed by events
    }
    RC_TRY(capture([&](hipStream_t cs) { return enqueue_local_search(S, cs); }, &S.ls));
    RC_TRY(capture([&](hipStream_t cs) { return enqueue_rest(S, cs); }, &S.rest));
    if (old_tiles(S.p) > 0) {
        RC_TRY(capture([&](hipStream_t cs) { return enqueue_old_dist(S, cs); }, &S.dold));
        HIP_TRY(hipStreamCreateWithFlags(&S.dstream, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&S.dfork, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&S.djoin, hipEventDisableTiming));
    }
    S.steps = 0;
    return PLSE_OK;
}

int session_step(Session &S, int generations, hipStream_t s) {
    for (const plse_instance *h : S.hs)
        if (S.base + S.steps + generations > h->max_gens) return PLSE_E_ARG;
    while (S.ev.size() < 3 * (size_t)(S.steps + generations)) {
        hipEvent_t e = nullptr;
        HIP_TRY(hipEventCreate(&e));
        S.ev.push_back(e);
    }
    if (S.staged) {
        // distances among P_t, search, best, distances with P', selection,
        // matching, crossover: one after another on `s`
        while (S.sev.size() < (kStages + 1) * (size_t)(S.steps + generations)) {
            hipEvent_t e = nullptr;
            HIP_TRY(hipEventCreate(&e));
            S.sev.push_back(e);
        }
        for (int g = 0; g < generations; ++g) {
            const size_t k = 3 * (size_t)(S.steps + g);
            hipEvent_t *m = &S.sev[(kStages + 1) * (size_t)(S.steps + g)];
            HIP_TRY(hipEventRecord(m[0], s));
            if (old_tiles(S.p) > 0) RC_TRY(enqueue_old_dist(S, s));
            HIP_TRY(hipEventRecord(m[1], s));
            HIP_TRY(hipEventRecord(S.ev[k], s));
            RC_TRY(enqueue_local_search(S, s));
            HIP_TRY(hipEventRecord(S.ev[k + 1], s));
            HIP_TRY(hipEventRecord(m[2], s));
            RC_TRY(enqueue_rest(S, s, &m[3]));
            HIP_TRY(hipEventRecord(m[7], s));
            if (S.stop_host) {
                plse_instance *h = S.hs[0];
                HIP_TRY(hipMemcpyAsync(S.stop_host + (S.steps + g) % Session::kStopRing,
                                       &at<Ctl>(h, h->L.ctl)->stop, sizeof(int32_t),
                                       hipMemcpyDeviceToHost, s));
            }
            HIP_TRY(hipEventRecord(S.ev[k + 2], s));
        }
        S.steps += generations;
        return PLSE_OK;
    }
    for (int g = 0; g < generations; ++g) {
        const size_t k = 3 * (size_t)(S.steps + g);
        if (S.dold) {
            // P_t is final (previous generation's update, or P_1): its
            // distances run beside the searches, joined before the rest
            HIP_TRY(hipEventRecord(S.dfork, s));
            HIP_TRY(hipStreamWaitEvent(S.dstream, S.dfork, 0));
            HIP_TRY(hipGraphLaunch(S.dold, S.dstream));
            HIP_TRY(hipEventRecord(S.djoin, S.dstream));
        }
        HIP_TRY(hipEventRecord(S.ev[k], s));
        if (S.ls)
            HIP_TRY(hipGraphLaunch(S.ls, s));
        else
            RC_TRY(enqueue_local_search(S, s));
        HIP_TRY(hipEventRecord(S.ev[k + 1], s));
        if (S.dold) HIP_TRY(hipStreamWaitEvent(s, S.djoin, 0));
        HIP_TRY(hipGraphLaunch(S.rest, s));
        if (S.stop_host) {
            plse_instance *h = S.hs[0];
            HIP_TRY(hipMemcpyAsync(S.stop_host + (S.steps + g) % Session::kStopRing,
                                   &at<Ctl>(h, h->L.ctl)->stop, sizeof(int32_t),
                                   hipMemcpyDeviceToHost, s));
        }
        HIP_TRY(hipEventRecord(S.ev[k + 2], s));
    }
    S.steps += generations;
    return PLSE_OK;
}

// Wait for the stream; per instance: statistics, timings and the best grid.
int session_end(Session &S, hipStream_t s, const std::vector<plse_instance *> &order,
                int8_t *const *grids, int32_t *filled) {
    const int G = std::max(S.base + S.steps, 1);
    std::vector<Ctl> ctl(S.hs.size());
    std::vector<std::vector<GenStat>> gs(S.hs.size(), std::vector<GenStat>((size_t)G));
    std::vector<std::vector<uint8_t>> star(S.hs.size());
    for (size_t i = 0; i < S.hs.size(); ++i) {
        plse_instance *h = S.hs[i];
        star[i].resize((size_t)h->stride);
        HIP_TRY(hipMemcpyAsync(&ctl[i], at<Ctl>(h, h->L.ctl), sizeof(Ctl), hipMemcpyDeviceToHost,
                               s));
        HIP_TRY(hipMemcpyAsync(gs[i].data(), at<GenStat>(h, h->L.stats), sizeof(GenStat) * G,
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(star[i].data(), at<uint8_t>(h, h->L.Sstar), h->stride,
                               hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    const int timed = S.ev.size() >= 3 * (size_t)S.steps ? S.steps : 0;
    std::vector<float> tp((size_t)timed), tr((size_t)timed);
    for (int g = 0; g < timed; ++g) {
        HIP_TRY(hipEventElapsedTime(&tp[g], S.ev[3 * g], S.ev[3 * g + 1]));
        HIP_TRY(hipEventElapsedTime(&tr[g], S.ev[3 * g + 1], S.ev[3 * g + 2]));
    }
    std::vector<float> tst;
    if (S.staged && S.sev.size() >= (kStages + 1) * (size_t)S.steps) {
        tst.resize((size_t)kStages * S.steps);
        for (int g = 0; g < S.steps; ++g)
            for (int q = 0; q < kStages; ++q)
                HIP_TRY(hipEventElapsedTime(&tst[(size_t)kStages * g + q],
                                            S.sev[(kStages + 1) * (size_t)g + q],
                                            S.sev[(kStages + 1) * (size_t)g + q + 1]));
    }
    for (size_t i = 0; i < S.hs.size(); ++i) {
        plse_instance *h = S.hs[i];
        const int gens = std::min(ctl[i].gens_run, G);  // every stepped generation has ended
        RunResult rr = summarize(ctl[i], gs[i].data(), gens);
        h->last = rr.stats;
        h->gen_best = std::move(rr.gen_best);
        h->gen_cnt = std::move(rr.gen_cnt);
        h->ms_plits = tp;
        h->ms_rest = tr;
        h->ms_stages = tst;
        const size_t slot = (size_t)(std::find(order.begin(), order.end(), h) - order.begin());
        filled[slot] = best_grid(h->n, h->cell_v, h->grid, star[i].data(), gens, grids[slot]);
    }
    return PLSE_OK;
}

struct BusyGuard {
    plse_instance *h;
    bool ok;
    explicit BusyGuard(plse_instance *hh) : h(hh) {
        int z = 0;
        ok = h->busy.compare_exchange_strong(z, 1);
    }
    ~BusyGuard() {
        if (ok) h->busy.store(0);
    }
};

void drop_session(plse_instance *h) {
    delete h->own;
    h->own = nullptr;
    h->in_session = false;
}

// Stage calls: one instance, argument block prepared on the host.
int stage_prepare(plse_instance *h, int p, hipStream_t s) {
    if (h->in_session) return PLSE_E_BUSY;
    RC_TRY(check_ws(h, p));
    RC_TRY(upload_instance(h, s));
    return PLSE_OK;
}

template <typename M>
ArgList single(plse_instance *h, M ArgBlock::*member) {
    ArgList L{};
    L.p[0] = dev_arg(h, member);
    return L;
}

// Workspace of plse_solve_noalloc: a fixed device array, one copy per GPU
// the library runs on, held until the process ends.  Host code never passes
// the array's name to a kernel or copy: it takes the array's device address
// from hipGetSymbolAddress once per device (scratch_address) and uses that.
constexpr size_t kScratchBytes = (size_t)PLSE_NOALLOC_BYTES;
__device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_at[kMaxDevices] = {};

// Device address of the current device's scratch array.
int scratch_address(void **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return PLSE_E_ARG;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_at[dev]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr || ((uintptr_t)ptr % kAlign)) return PLSE_E_HIP;
        g_scratch_at[dev] = ptr;
    }
    *out = g_scratch_at[dev];
    return PLSE_OK;
}

// A whole solve of one instance enqueued kernel by kernel on `s`: no graphs,
// side streams or events (so no runtime object is created), distances among
// P_t in line before the searches instead of beside them.  Same kernels and
// arguments as a session, so the same result.
int solve_direct(plse_instance *h, int p, int G, uint64_t seed, hipStream_t s,
                 int8_t *best_grid, int32_t *filled) {
    Session S;
    S.hs = {h};
    S.p = p;
    S.seed = seed;
    RC_TRY(admit(S.hs, p, &seed, s));
    shape_session(S);
    if (S.groups.size() != 1) return PLSE_E_ARG;
    for (int g = 0; g < G; ++g) {
        if (old_tiles(p) > 0) RC_TRY(enqueue_old_dist(S, s));
        RC_TRY(enqueue_local_search(S, s));
        RC_TRY(enqueue_rest(S, s));
    }
    S.steps = G;
    int8_t *grids[1] = {best_grid};
    return session_end(S, s, {h}, grids, filled);
}

}  // namespace

extern "C" {

int plse_create(int32_t n, const int8_t *grid, plse_handle *out) {
    if (!grid || !out || n < 1 || n > 127) return PLSE_E_ARG;
    *out = nullptr;
    // A partial Latin square: symbols in [0, n], none repeated in a row or column.
    std::vector<uint64_t> rowm(2 * n, 0), colm(2 * n, 0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const int k = grid[i * n + j];
            if (k < 0 || k > n) return PLSE_E_GRID;
            if (!k) continue;
            const uint64_t bit = 1ull << (k & 63);
            const int hw = k >> 6;
            if ((rowm[2 * i + hw] & bit) || (colm[2 * j + hw] & bit)) return PLSE_E_GRID;
            rowm[2 * i + hw] |= bit;
            colm[2 * j + hw] |= bit;
        }
    plse_instance *h = new plse_instance();
    h->n = n;
    h->grid.assign(grid, grid + (size_t)n * n);
    h->cell_v.assign((size_t)n * n, -1);
    // Alg. 1: D*(cell) = {1..n} minus the symbols of its row and column; an
    // empty cell with D* empty is impossible (l); the others are vertices,
    // numbered row-major.
    uint64_t full[2] = {0, 0};
    for (int k = 1; k <= n; ++k) full[k >> 6] |= 1ull << (k & 63);
    std::vector<int> rowc(n, 0), colc(n, 0);
    std::vector<uint32_t> rowl((size_t)n * n, 0), coll((size_t)n * n, 0);
    std::vector<uint64_t> dmask;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (grid[i * n + j]) continue;
            const uint64_t d0 = full[0] & ~(rowm[2 * i] | colm[2 * j]);
            const uint64_t d1 = full[1] & ~(rowm[2 * i + 1] | colm[2 * j + 1]);
            if (!d0 && !d1) {
                h->cell_v[i * n + j] = -2;
                h->l++;
                continue;
            }
            const int v = h->nv++;
            h->cell_v[i * n + j] = v;
            h->vrc.push_back((uint16_t)(i | (j << 8)));
            dmask.push_back(d0);
            dmask.push_back(d1);
            rowl[(size_t)i * n + rowc[i]++] = (uint32_t)v | ((uint32_t)j << 16);
            coll[(size_t)j * n + colc[j]++] = (uint32_t)v | ((uint32_t)i << 16);
        }
    h->ub = (h->l == 1) ? n * n - 2 : n * n - h->l;
    h->rclo.assign((size_t)2 * n + 1, 0);
    for (int i = 0; i < n; ++i) {
        for (int t = 0; t < rowc[i]; ++t) h->rcl.push_back(rowl[(size_t)i * n + t]);
        h->rclo[i + 1] = (uint32_t)h->rcl.size();
    }
    for (int j = 0; j < n; ++j) {
        for (int t = 0; t < colc[j]; ++t) h->rcl.push_back(coll[(size_t)j * n + t]);
        h->rclo[n + j + 1] = (uint32_t)h->rcl.size();
    }
    // vertex records: 128-bit domain mask, first slot (sum of earlier domain
    // sizes), coordinates and domain size; vertex info words; candidate rows
    // (the moves 0, D*(v) ascending, zero padded to ts positions)
    h->vrec.assign((size_t)h->nv * 8, 0);
    h->vinfo.assign(h->nv, 0);
    h->nl = std::max(2 * (n - 1), 1);
    h->nbr.assign((size_t)h->nv * h->nl, 0);
    uint32_t off = 0;
    for (int v = 0; v < h->nv; ++v) {
        uint32_t *r = &h->vrec[(size_t)v * 8];
        r[0] = (uint32_t)dmask[2 * v];
        r[1] = (uint32_t)(dmask[2 * v] >> 32);
        r[2] = (uint32_t)dmask[2 * v + 1];
        r[3] = (uint32_t)(dmask[2 * v + 1] >> 32);
        const uint32_t d = (uint32_t)(__builtin_popcountll(dmask[2 * v]) +
                                      __builtin_popcountll(dmask[2 * v + 1]));
        r[4] = off;
        r[5] = (uint32_t)h->vrc[v] | (d << 16);
        // neighbours: the other vertices of v's row, then of its column
        const int i = h->vrc[v] & 0xFF, j = h->vrc[v] >> 8;
        uint32_t deg = 0;
        for (int t = 0; t < rowc[i]; ++t)
            if ((int)(rowl[(size_t)i * n + t] & 0xFFFFu) != v)
                h->nbr[(size_t)v * h->nl + deg++] = rowl[(size_t)i * n + t];
        for (int t = 0; t < colc[j]; ++t)
            if ((int)(coll[(size_t)j * n + t] & 0xFFFFu) != v)
                h->nbr[(size_t)v * h->nl + deg++] = coll[(size_t)j * n + t] | 0x80000000u;
        h->vinfo[v] = (uint32_t)h->vrc[v] | (d << 16) | (deg << 24);
        h->dmax = std::max(h->dmax, (int)d);
        off += d;
    }
    h->nd = (int)off;
    h->ts = (int)round_up((size_t)h->dmax + 1, 8);
    h->cand.assign((size_t)h->nv * h->ts, 0);
    for (int v = 0; v < h->nv; ++v) {
        // the last domain colour repeats to the end of the row: a repeated
        // position evaluates exactly as that colour's own, so the search
        // needs no test for positions past the domain
        uint8_t *row = &h->cand[(size_t)v * h->ts];
        int t = 1;
        for (int k = 1; k <= n; ++k)
            if ((dmask[2 * v + (k >> 6)] >> (k & 63)) & 1ull) row[t++] = (uint8_t)k;
        for (int q = t; q < h->ts; ++q) row[q] = row[t - 1];
    }
    h->stride = (int)round_up((size_t)std::max(h->nv, 1), 16);
    // defaults: Table 1 and Section 3.3, total depth 10 n^2
    const int64_t depth = 10LL * n * n;
    h->P.depth2 = std::min<int64_t>(2LL * h->nv, depth);
    h->P.depth1 = depth - h->P.depth2;
    h->P.alpha_num = 6;
    h->P.alpha_den = 10;
    h->P.beta_num = 20;
    h->P.beta_den = 1;
    h->P.spacing = 10;
    h->P.stop_at_ub = 0;
    h->P.max_iters = 0;  // no iteration budget
    h->P.hist_len = kHist;
    h->P.crossover = 0;  // AUX
    h->P.matching = 0;   // nearest neighbour
    h->P.variant = 0;    // MPMA
    *out = h;
    return PLSE_OK;
}

int plse_info(plse_handle h, int32_t *nv, int32_t *l, int32_t *ub) {
    if (!h) return PLSE_E_ARG;
    if (nv) *nv = h->nv;
    if (l) *l = h->l;
    if (ub) *ub = h->ub;
    return PLSE_OK;
}

int plse_sizes(plse_handle h, int32_t *n, int32_t *nv, int32_t *nd, int32_t *stride) {
    if (!h) return PLSE_E_ARG;
    if (n) *n = h->n;
    if (nv) *nv = h->nv;
    if (nd) *nd = h->nd;
    if (stride) *stride = h->stride;
    return PLSE_OK;
}

int plse_row_stride(plse_handle h, int32_t *stride) {
    if (!h || !stride) return PLSE_E_ARG;
    *stride = h->stride;
    return PLSE_OK;
}

int plse_set_param(plse_handle h, const char *key, int64_t v) {
    if (!h || !key) return PLSE_E_ARG;
    BusyGuard g(h);
    if (!g.ok || h->in_session) return PLSE_E_BUSY;
    const std::string k(key);
    Params &P = h->P;
    if (k == "depth") {
        if (v < 0 || v > INT32_MAX) return PLSE_E_PARAM;
        P.depth2 = std::min<int64_t>(2LL * h->nv, v);
        P.depth1 = v - P.depth2;
    } else if (k == "depth1") {
        if (v < 0 || v > INT32_MAX) return PLSE_E_PARAM;
        P.depth1 = v;
    } else if (k == "depth2") {
        if (v < 0 || v > INT32_MAX) return PLSE_E_PARAM;
        P.depth2 = v;
    } else if (k == "alpha_num") {
        if (v < 0 || v > 1000) return PLSE_E_PARAM;
        P.alpha_num = v;
    } else if (k == "alpha_den") {
        if (v < 1 || v > 1000) return PLSE_E_PARAM;
        P.alpha_den = v;
    } else if (k == "beta_num") {
        if (v < 1 || v > 1000000) return PLSE_E_PARAM;
        P.beta_num = v;
    } else if (k == "beta_den") {
        if (v < 1 || v > 1000000) return PLSE_E_PARAM;
        P.beta_den = v;
    } else if (k == "spacing") {
        if (v < 1 || v > 1000000) return PLSE_E_PARAM;
        P.spacing = v;
    } else if (k == "stop_at_ub") {
        if (v != 0 && v != 1) return PLSE_E_PARAM;
        P.stop_at_ub = (int32_t)v;
    } else if (k == "max_iterations") {
        if (v < 0) return PLSE_E_PARAM;
        P.max_iters = v;
    } else if (k == "nn_history") {
        if (v < 0 || v > kHist) return PLSE_E_PARAM;
        P.hist_len = (int32_t)v;
    } else if (k == "crossover") {
        if (v < 0 || v > 2) return PLSE_E_PARAM;
        P.crossover = (int32_t)v;
    } else if (k == "matching") {
        if (v < 0 || v > 1) return PLSE_E_PARAM;
        P.matching = (int32_t)v;
    } else if (k == "variant") {
        if (v < 0 || v > 1) return PLSE_E_PARAM;
        P.variant = (int32_t)v;
    } else if (k == "slots_per_lane") {
        if (v != 0 && v != 2 && v != 4 && v != 8) return PLSE_E_PARAM;
        h->spl = (int)v;
    } else if (k == "waves_per_block") {
        if (v != 0 && v != 1 && v != 2 && v != 4) return PLSE_E_PARAM;
        h->wpb = (int)v;
    } else if (k == "plits_kernel") {
        if (v < 0 || v > 2) return PLSE_E_PARAM;
        h->kernel = (int)v;
    } else if (k == "stage_timing") {
        if (v != 0 && v != 1) return PLSE_E_PARAM;
        h->stage_timing = (int)v;
    } else if (k == "persistent") {
        if (v != 0 && v != 1) return PLSE_E_PARAM;
        h->persistent = (int)v;
    } else if (k == "select_global_sort") {
        if (v != 0 && v != 1) return PLSE_E_PARAM;
        h->sel_global = (int)v;
    } else if (k == "fail_at_generation") {
        if (v < 0 || v > PLSE_MAX_GENERATIONS) return PLSE_E_PARAM;
        h->fail_at = (int)v;
    } else if (k == "max_generations") {
        if (v < 1 || v > PLSE_MAX_GENERATIONS) return PLSE_E_PARAM;
        h->max_gens = (int)v;
    } else {
        return PLSE_E_PARAM;
    }
    return PLSE_OK;
}

int plse_get_param(plse_handle h, const char *key, int64_t *v) {
    if (!h || !key || !v) return PLSE_E_ARG;
    const std::string k(key);
    const Params &P = h->P;
    if (k == "depth") *v = P.depth1 + P.depth2;
    else if (k == "depth1") *v = P.depth1;
    else if (k == "depth2") *v = P.depth2;
    else if (k == "alpha_num") *v = P.alpha_num;
    else if (k == "alpha_den") *v = P.alpha_den;
    else if (k == "beta_num") *v = P.beta_num;
    else if (k == "beta_den") *v = P.beta_den;
    else if (k == "spacing") *v = P.spacing;
    else if (k == "stop_at_ub") *v = P.stop_at_ub;
    else if (k == "max_iterations") *v = P.max_iters;
    else if (k == "nn_history") *v = P.hist_len;
    else if (k == "crossover") *v = P.crossover;
    else if (k == "matching") *v = P.matching;
    else if (k == "variant") *v = P.variant;
    else if (k == "slots_per_lane") *v = choose_spl(h);
    else if (k == "waves_per_block") *v = choose_wpb(h);
    else if (k == "fail_at_generation") *v = h->fail_at;
    else if (k == "max_generations") *v = h->max_gens;
    else if (k == "select_global_sort") *v = h->sel_global;
    else if (k == "plits_kernel") *v = plits_lds(h).lean ? 2 : 1;
    else if (k == "stage_timing") *v = h->stage_timing;
    else if (k == "plits_waves_per_cu") {
        // resident tabu-search waves per CU of this handle's launch shape
        // (registers, LDS and workgroup limits of the runtime's calculation)
        set_attributes_once();
        const PlitsLds pl = plits_lds(h);
        *v = plits_waves_per_cu(choose_spl(h), choose_wpb(h), pl.per_wave, P.variant != 0, pl.lean);
    }
    else if (k == "persistent") *v = h->persistent;
    else return PLSE_E_PARAM;
    return PLSE_OK;
}

int plse_workspace_bytes(plse_handle h, int32_t p, size_t *bytes) {
    if (!h || !bytes || p < 2 || p > PLSE_MAX_POPULATION) return PLSE_E_ARG;
    *bytes = plan(h, p).total;
    return PLSE_OK;
}

int plse_attach_workspace(plse_handle h, void *ptr, size_t bytes) {
    if (!h) return PLSE_E_ARG;
    if (ptr && ((uintptr_t)ptr % kAlign)) return PLSE_E_ARG;
    BusyGuard g(h);
    if (!g.ok || h->in_session) return PLSE_E_BUSY;
    h->ws = reinterpret_cast<uint8_t *>(ptr);
    h->ws_bytes = ptr ? bytes : 0;
    return PLSE_OK;
}

int plse_begin(plse_handle h, int32_t p, uint64_t seed, void *stream) {
    if (!h) return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    drop_session(h);
    Session *S = new Session();
    S->hs = {h};
    S->p = p;
    S->seed = seed;
    const int rc = session_begin(*S, &seed, reinterpret_cast<hipStream_t>(stream));
    if (rc) {
        delete S;
        return rc;
    }
    h->own = S;
    h->in_session = true;
    return PLSE_OK;
}

int plse_step(plse_handle h, int32_t generations, void *stream) {
    if (!h || generations < 0) return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    if (!h->in_session || !h->own) return PLSE_E_ARG;
    return session_step(*h->own, generations, reinterpret_cast<hipStream_t>(stream));
}

int plse_end(plse_handle h, void *stream, int8_t *best_grid, int32_t *filled) {
    if (!h || !best_grid || !filled) return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    if (!h->in_session || !h->own) return PLSE_E_ARG;
    int8_t *grids[1] = {best_grid};
    const int rc = session_end(*h->own, reinterpret_cast<hipStream_t>(stream), {h}, grids, filled);
    drop_session(h);
    return rc;
}

int plse_peek(plse_handle h, void *stream, plse_progress *out) {
    if (!h || !out) return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    if (!h->in_session || !h->own) return PLSE_E_ARG;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Ctl c;
    HIP_TRY(hipMemcpyAsync(&c, at<Ctl>(h, h->L.ctl), sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    out->generations_run = c.gens_run;
    out->best_f = c.fstar;
    out->best_generation = c.best_gen;
    out->stop_reason = c.stop_reason;
    out->iterations = c.iters;
    return PLSE_OK;
}

}  // extern "C"

namespace {

// Checkpoint image: header, then the device state at a generation boundary.
struct CkptHeader {
    uint32_t magic, version;
    int32_t n, nv, stride, p;
    uint64_t seed, ident;
    int32_t gens_run, pad;
};
constexpr uint32_t kCkptMagic = 0x4B534C50u;  // "PLSK"
// 2: nine counters per generation record
constexpr uint32_t kCkptVersion = 2u;

// FNV-1a over the grid and every parameter that shapes a run.
uint64_t run_ident(const plse_instance *h) {
    uint64_t x = 1469598103934665603ull;
    auto mix = [&](const void *p, size_t n) {
        const uint8_t *b = static_cast<const uint8_t *>(p);
        for (size_t i = 0; i < n; ++i) x = (x ^ b[i]) * 1099511628211ull;
    };
    mix(h->grid.data(), h->grid.size());
    const Params &P = h->P;
    const int64_t v[13] = {P.depth1, P.depth2, P.alpha_num, P.alpha_den, P.beta_num,
                           P.beta_den, P.spacing, P.max_iters, P.stop_at_ub, P.hist_len,
                           P.crossover, P.matching, P.variant};
    mix(v, sizeof(v));
    return x;
}

// The regions a checkpoint holds, in order: Ctl, the statistics of the
// generations run, S*, P_t, f of P_t, uids, partner histories and their
// counts, and the offspring waiting for the next generation's search.
struct CkptPart {
    size_t off, bytes;
};
std::vector<CkptPart> ckpt_parts(const plse_instance *h, int p, int gens) {
    const Layout &L = h->L;
    const size_t st = (size_t)h->stride, pp = (size_t)p;
    return {{L.ctl, sizeof(Ctl)},          {L.stats, sizeof(GenStat) * (size_t)gens},
            {L.Sstar, st},                 {L.S_all, pp * st},
            {L.f_all, 4 * pp},             {L.uid, 8 * pp},
            {L.hist, 8 * pp * kHist},      {L.hc, 4 * pp},
            {L.S_off, pp * st}};
}

size_t ckpt_bytes(const std::vector<CkptPart> &parts) {
    size_t b = sizeof(CkptHeader);
    for (const CkptPart &c : parts) b += c.bytes;
    return b;
}

}  // namespace

extern "C" {

int plse_checkpoint(plse_handle h, void *stream, void *buf, size_t capacity, size_t *bytes) {
    if (!h || !bytes) return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    if (!h->in_session || !h->own || h->own->hs.size() != 1) return PLSE_E_ARG;
    const Session &S = *h->own;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Ctl c;
    HIP_TRY(hipMemcpyAsync(&c, at<Ctl>(h, h->L.ctl), sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const std::vector<CkptPart> parts = ckpt_parts(h, S.p, c.gens_run);
    *bytes = ckpt_bytes(parts);
    if (!buf) return PLSE_OK;
    if (capacity < *bytes) return PLSE_E_ARG;
    CkptHeader hd{kCkptMagic, kCkptVersion, h->n, h->nv, h->stride, S.p, S.seed, run_ident(h),
                  c.gens_run, 0};
    uint8_t *out = static_cast<uint8_t *>(buf);
    std::memcpy(out, &hd, sizeof(hd));
    size_t o = sizeof(hd);
    for (const CkptPart &q : parts) {
        if (q.bytes)
            HIP_TRY(hipMemcpyAsync(out + o, h->ws + q.off, q.bytes, hipMemcpyDeviceToHost, s));
        o += q.bytes;
    }
    HIP_TRY(hipStreamSynchronize(s));
    return PLSE_OK;
}

int plse_resume(plse_handle h, int32_t p, void *stream, const void *buf, size_t bytes) {
    if (!h || !buf || bytes < sizeof(CkptHeader)) return PLSE_E_ARG;
    CkptHeader hd;
    std::memcpy(&hd, buf, sizeof(hd));
    if (hd.magic != kCkptMagic || hd.version != kCkptVersion || hd.n != h->n || hd.nv != h->nv ||
        hd.stride != h->stride || hd.p != p || hd.ident != run_ident(h) || hd.gens_run < 0 ||
        hd.gens_run > h->max_gens)
        return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    RC_TRY(check_ws(h, p));
    const std::vector<CkptPart> parts = ckpt_parts(h, p, hd.gens_run);
    if (bytes != ckpt_bytes(parts)) return PLSE_E_ARG;
    drop_session(h);
    Session *S = new Session();
    S->hs = {h};
    S->p = p;
    S->seed = hd.seed;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // a fresh session of the same seed, then its state replaced by the image
    int rc = session_begin(*S, &hd.seed, s);
    const uint8_t *in = static_cast<const uint8_t *>(buf);
    size_t o = sizeof(hd);
    for (const CkptPart &q : parts) {
        if (!rc && q.bytes) {
            const hipError_t e =
                hipMemcpyAsync(h->ws + q.off, in + o, q.bytes, hipMemcpyHostToDevice, s);
            if (e != hipSuccess) rc = hip_fail(e, "plse_resume");
        }
        o += q.bytes;
    }
    if (!rc) {
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = hip_fail(e, "plse_resume");
    }
    if (rc) {
        delete S;
        return rc;
    }
    S->base = hd.gens_run;
    h->own = S;
    h->in_session = true;
    return PLSE_OK;
}

int plse_solve(plse_handle h, int32_t p, int32_t G, uint64_t seed, void *stream,
               int8_t *best_grid, int32_t *filled) {
    if (!h || !best_grid || !filled || G < 1 || G > h->max_gens) return PLSE_E_ARG;
    int rc = plse_begin(h, p, seed, stream);
    if (rc) return rc;
    rc = plse_step(h, G, stream);
    if (rc) {
        std::vector<int8_t> tmp((size_t)h->n * h->n);
        int32_t f = 0;
        (void)plse_end(h, stream, tmp.data(), &f);
        return rc;
    }
    return plse_end(h, stream, best_grid, filled);
}

int plse_solve_noalloc(plse_handle h, int32_t p, int32_t G, uint64_t seed, void *stream,
                       int8_t *best_grid, int32_t *filled, size_t *bytes_needed) {
    if (!h || !best_grid || !filled || G < 1 || G > h->max_gens || p < 2 ||
        p > PLSE_MAX_POPULATION)
        return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok || h->in_session) return PLSE_E_BUSY;
    // per-generation records sized by this call's generations
    const int keep_gens = h->max_gens;
    h->max_gens = G;
    const size_t need = plan(h, p).total;
    if (bytes_needed) *bytes_needed = need;
    if (need > kScratchBytes) {
        h->max_gens = keep_gens;
        return PLSE_E_CAPACITY;
    }
    void *ptr = nullptr;
    int rc = scratch_address(&ptr);
    if (!rc) {
        uint8_t *keep_ws = h->ws;
        const size_t keep_bytes = h->ws_bytes;
        h->ws = reinterpret_cast<uint8_t *>(ptr);
        h->ws_bytes = kScratchBytes;
        rc = solve_direct(h, p, G, seed, reinterpret_cast<hipStream_t>(stream), best_grid, filled);
        h->ws = keep_ws;
        h->ws_bytes = keep_bytes;
    }
    h->max_gens = keep_gens;
    return rc;
}

int plse_measure_lds_bandwidth(void *stream, int32_t repeats, double *bytes_per_second) {
    if (!bytes_per_second || repeats < 1) return PLSE_E_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    void *sink = nullptr;
    RC_TRY(scratch_address(&sink));
    const int blocks = cus * 16;
    const uint32_t iters = 4096;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    double best = 0.0, bytes = 0.0;
    for (int r = 0; r <= repeats && e == hipSuccess; ++r) {
        e = hipEventRecord(e0, s);
        if (e == hipSuccess)
            e = launch_lds_read(blocks, iters, reinterpret_cast<uint32_t *>(sink), s, &bytes);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && r > 0 && ms > 0.0f) best = std::max(best, bytes / (ms * 1e-3));
    }
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "plse_measure_lds_bandwidth");
    *bytes_per_second = best;
    return PLSE_OK;
}

}  // extern "C"

// An open batched session (plse_batch_begin .. plse_batch_end): the session
// over the instances and the guards that keep each handle busy meanwhile.
struct plse_batch_t {
    Session S;
    std::vector<plse_instance *> order;  // caller's order
    std::vector<BusyGuard *> guards;
    ~plse_batch_t() {
        for (BusyGuard *g : guards) delete g;
    }
};

extern "C" {

int plse_batch_begin(const plse_handle *hs, int32_t count, int32_t p, const uint64_t *seeds,
                     void *stream, plse_batch *out) {
    if (!hs || count < 1 || !seeds || !out) return PLSE_E_ARG;
    *out = nullptr;
    for (int i = 0; i < count; ++i) {
        if (!hs[i]) return PLSE_E_ARG;
        for (int j = 0; j < i; ++j)
            if (hs[j] == hs[i]) return PLSE_E_ARG;
    }
    plse_batch_t *b = new plse_batch_t();
    int rc = PLSE_OK;
    for (int i = 0; i < count && !rc; ++i) {
        b->guards.push_back(new BusyGuard(hs[i]));
        if (!b->guards.back()->ok || hs[i]->in_session) rc = PLSE_E_BUSY;
    }
    if (!rc) {
        b->S.hs.assign(hs, hs + count);
        b->S.p = p;
        b->order.assign(hs, hs + count);
        std::vector<uint64_t> sd(seeds, seeds + count);
        rc = session_begin(b->S, sd.data(), reinterpret_cast<hipStream_t>(stream));
    }
    if (rc) {
        delete b;
        return rc;
    }
    *out = b;
    return PLSE_OK;
}

int plse_batch_step(plse_batch b, int32_t generations, void *stream) {
    if (!b || generations < 0) return PLSE_E_ARG;
    return session_step(b->S, generations, reinterpret_cast<hipStream_t>(stream));
}

int plse_batch_end(plse_batch b, void *stream, int8_t *const *best_grids, int32_t *filled) {
    if (!b) return PLSE_E_ARG;
    int rc = PLSE_E_ARG;
    if (best_grids && filled) {
        bool ok = true;
        for (size_t i = 0; i < b->order.size(); ++i) ok = ok && best_grids[i];
        if (ok)
            rc = session_end(b->S, reinterpret_cast<hipStream_t>(stream), b->order, best_grids,
                             filled);
    }
    if (rc) (void)hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
    delete b;
    return rc;
}

int plse_solve_batch(const plse_handle *hs, int32_t count, int32_t p, int32_t G,
                     const uint64_t *seeds, void *stream, int8_t *const *best_grids,
                     int32_t *filled) {
    if (!hs || count < 1 || !seeds || !best_grids || !filled || G < 1 ||
        G > PLSE_MAX_GENERATIONS)
        return PLSE_E_ARG;
    for (int i = 0; i < count; ++i) {
        if (!hs[i] || !best_grids[i] || G > hs[i]->max_gens) return PLSE_E_ARG;
        for (int j = 0; j < i; ++j)
            if (hs[j] == hs[i]) return PLSE_E_ARG;
    }
    std::vector<BusyGuard *> guards;
    int rc = PLSE_OK;
    for (int i = 0; i < count && !rc; ++i) {
        guards.push_back(new BusyGuard(hs[i]));
        if (!guards.back()->ok || hs[i]->in_session) rc = PLSE_E_BUSY;
    }
    if (!rc) {
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        Session S;
        S.hs.assign(hs, hs + count);
        S.p = p;
        std::vector<plse_instance *> order(hs, hs + count);
        std::vector<uint64_t> sd(seeds, seeds + count);
        rc = session_begin(S, sd.data(), s);
        if (!rc) rc = session_step(S, G, s);
        if (!rc) rc = session_end(S, s, order, best_grids, filled);
    }
    for (BusyGuard *g : guards) delete g;
    return rc;
}

int plse_last_timing(plse_handle h, int32_t *steps, float *plits_ms, float *rest_ms) {
    if (!h || !steps) return PLSE_E_ARG;
    *steps = (int32_t)h->ms_plits.size();
    if (plits_ms) std::copy(h->ms_plits.begin(), h->ms_plits.end(), plits_ms);
    if (rest_ms) std::copy(h->ms_rest.begin(), h->ms_rest.end(), rest_ms);
    return PLSE_OK;
}

int plse_last_stage_timing(plse_handle h, int32_t *steps, float *ms) {
    if (!h || !steps) return PLSE_E_ARG;
    *steps = (int32_t)(h->ms_stages.size() / kStages);
    if (ms) std::copy(h->ms_stages.begin(), h->ms_stages.end(), ms);
    return PLSE_OK;
}

int plse_last_stats(plse_handle h, plse_stats *out, int32_t *per_gen_best_f,
                    uint64_t *per_gen_counters) {
    if (!h || !out) return PLSE_E_ARG;
    *out = h->last;
    if (per_gen_best_f) std::copy(h->gen_best.begin(), h->gen_best.end(), per_gen_best_f);
    if (per_gen_counters) std::copy(h->gen_cnt.begin(), h->gen_cnt.end(), per_gen_counters);
    return PLSE_OK;
}

void plse_destroy(plse_handle h) {
    if (!h) return;
    drop_session(h);
    delete h;
}

const char *plse_strerror(int status) {
    switch (status) {
        case PLSE_OK: return "ok";
        case PLSE_E_ARG: return "invalid argument";
        case PLSE_E_GRID: return "grid is not a partial Latin square";
        case PLSE_E_WORKSPACE: return "workspace missing or too small";
        case PLSE_E_HIP: return g_hip_error.empty() ? "HIP error" : g_hip_error.c_str();
        case PLSE_E_BUSY: return "handle busy";
        case PLSE_PENDING: return "pending";
        case PLSE_E_PARAM: return "unknown parameter or value out of range";
        case PLSE_E_CAPACITY: return "request exceeds the server capacity";
        case PLSE_E_FAULT: return "request ended by the fault-injection hook";
        case PLSE_E_CANCELLED: return "request cancelled";
        default: return "unknown status";
    }
}

// ---------------------------------------------------------------------------
// stage calls
// ---------------------------------------------------------------------------
int plse_stage_init(plse_handle h, int32_t p, uint64_t seed, void *stream, uint8_t *S,
                    int32_t *f) {
    if (!h || !S || !f) return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    RC_TRY(stage_prepare(h, p, s));
    h->args.init = InitArgs{dev_instance(h), S, f, p, next_pow2(std::max(4, h->nv)),
                            (uint32_t)seed, (uint32_t)(seed >> 32)};
    RC_TRY(upload_args(h, s));
    HIP_TRY(launch_init(single(h, &ArgBlock::init), 1, p,
                        init_lds_bytes(h->args.init.I, h->args.init.pow2), s));
    return PLSE_OK;
}

int plse_stage_plits(plse_handle h, int32_t p, int32_t gen, uint64_t seed, void *stream,
                     const uint8_t *S_in, uint8_t *S_out, int32_t *f_out, uint64_t *counters) {
    if (!h || !S_in || !S_out || !f_out || !counters || S_in == S_out || gen < 1 ||
        gen >= (1 << 24))
        return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    RC_TRY(stage_prepare(h, p, s));
    h->args.plits = make_plits(h, p, gen, seed, S_in, S_out, f_out, counters, nullptr);
    h->args.fill = FillArgs{at<uint32_t>(h, h->L.tabu), (size_t)p * h->nv * h->ts};
    RC_TRY(upload_args(h, s));
    HIP_TRY(launch_fill_zero(single(h, &ArgBlock::fill), 1, s));
    const int wpb = choose_wpb(h);
    const PlitsLds pl = plits_lds(h);
    if (wpb * pl.per_wave > max_lds_per_block()) return PLSE_E_ARG;
    HIP_TRY(launch_plits(single(h, &ArgBlock::plits), 1, p, pl.per_wave, choose_spl(h), wpb,
                         h->P.variant != 0, pl.lean, s));
    return PLSE_OK;
}

}  // extern "C"

namespace {

// Times phase-1 searches of the initial population's first `sample`
// individuals under each launch shape (chunk sizes 2, 4, 8; with `waves`
// also 1, 2, 4 waves per block) and keeps the fastest on the handle.
int autotune(plse_instance *h, int32_t sample, int32_t depth, uint64_t seed, hipStream_t s,
             bool waves, float *out_ms) {
    RC_TRY(stage_prepare(h, sample, s));
    // the workspace's offspring, scratch and counter regions hold the sample
    uint8_t *S_in = at<uint8_t>(h, h->L.S_off), *S_out = at<uint8_t>(h, h->L.S_tmp);
    int32_t *f = at<int32_t>(h, h->L.f_tmp);
    uint64_t *cnt = at<uint64_t>(h, h->L.cnt);
    h->args.init = InitArgs{dev_instance(h), S_in, f, sample, next_pow2(std::max(4, h->nv)),
                            (uint32_t)seed, (uint32_t)(seed >> 32)};
    RC_TRY(upload_args(h, s));
    HIP_TRY(launch_init(single(h, &ArgBlock::init), 1, sample,
                        init_lds_bytes(h->args.init.I, h->args.init.pow2), s));
    // phase-1 searches of `depth` iterations per shape; without `waves` the
    // waves per block stay with the handle's setting (or the occupancy
    // rule, which also weighs the uneven search lengths of later generations)
    const Params saved = h->P;
    const int spl0 = h->spl, wpb0 = h->wpb;
    h->P.depth1 = depth;
    h->P.depth2 = 0;
    const int spls[3] = {2, 4, 8}, wpbs[3] = {1, 2, 4};
    const int nshape = waves ? 9 : 3;
    float ms[9] = {};
    bool fits[9] = {};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = PLSE_OK;
    auto chk = [&](hipError_t e, const char *what) {
        if (e != hipSuccess && !rc) rc = hip_fail(e, what);
    };
    chk(hipEventCreate(&e0), "hipEventCreate");
    chk(hipEventCreate(&e1), "hipEventCreate");
    // pass 0: one untimed launch (code loading, caches); pass 1: every shape
    for (int pass = 0; pass < 2 && !rc; ++pass) {
        for (int i = 0; i < nshape && !rc; ++i) {
            h->spl = spls[i % 3];
            if (waves) h->wpb = wpbs[i / 3];
            const PlitsLds pl = plits_lds(h);
            const int per = pl.per_wave, wpb = choose_wpb(h);
            fits[i] = plits_fn(h->spl, h->P.variant != 0) != nullptr &&
                      wpb * per <= max_lds_per_block();
            if (!fits[i] || (pass == 0 && i > 0)) continue;
            h->args.plits = make_plits(h, sample, 1, seed, S_in, S_out, f, cnt, nullptr);
            h->args.fill = FillArgs{at<uint32_t>(h, h->L.tabu), (size_t)sample * h->nv * h->ts};
            const int up = upload_args(h, s);
            if (up && !rc) rc = up;
            if (rc) break;
            chk(launch_fill_zero(single(h, &ArgBlock::fill), 1, s), "fill");
            if (pass == 1) chk(hipEventRecord(e0, s), "hipEventRecord");
            chk(launch_plits(single(h, &ArgBlock::plits), 1, sample, per, h->spl, wpb,
                             h->P.variant != 0, pl.lean, s),
                "plits");
            if (pass == 1) {
                chk(hipEventRecord(e1, s), "hipEventRecord");
                chk(hipEventSynchronize(e1), "hipEventSynchronize");
                chk(hipEventElapsedTime(&ms[i], e0, e1), "hipEventElapsedTime");
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    h->P = saved;
    h->spl = spl0;
    h->wpb = wpb0;
    if (rc) return rc;
    int best = -1;
    for (int i = 0; i < nshape; ++i) {
        if (out_ms) out_ms[i] = fits[i] ? ms[i] : -1.0f;
        if (fits[i] && (best < 0 || ms[i] < ms[best])) best = i;
    }
    if (best < 0) return PLSE_E_ARG;
    h->spl = spls[best % 3];
    if (waves) h->wpb = wpbs[best / 3];
    return PLSE_OK;
}

}  // namespace

extern "C" {

int plse_autotune(plse_handle h, int32_t sample, int32_t depth, uint64_t seed, void *stream,
                  float *out_ms) {
    if (!h || sample < 2 || depth < 1) return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    return autotune(h, sample, depth, seed, reinterpret_cast<hipStream_t>(stream), false, out_ms);
}

int plse_autotune_shape(plse_handle h, int32_t sample, int32_t depth, uint64_t seed,
                        void *stream, float *out_ms) {
    if (!h || sample < 2 || depth < 1) return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    return autotune(h, sample, depth, seed, reinterpret_cast<hipStream_t>(stream), true, out_ms);
}

int plse_stage_distances(plse_handle h, int32_t m, void *stream, const uint8_t *S, int16_t *D) {
    if (!h || !S || !D || m < 1) return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    RC_TRY(stage_prepare(h, std::max(2, (m + 1) / 2), s));
    const int W = (h->nv + 31) / 32, B = colour_bits(h->n);
    h->args.pack = PackArgs{nullptr, S, at<uint32_t>(h, h->L.planes), m, h->nv, h->stride, W, B, 0};
    const int nt1 = (m + kDistTile - 1) / kDistTile;
    h->args.dist = DistArgs{nullptr, at<uint32_t>(h, h->L.planes), D, m, W, m, nt1, 0};
    RC_TRY(upload_args(h, s));
    HIP_TRY(launch_pack(single(h, &ArgBlock::pack), 1, (size_t)m * W, s));
    HIP_TRY(launch_dist(single(h, &ArgBlock::dist), 1, (long)nt1 * (nt1 + 1) / 2, B, s));
    return PLSE_OK;
}

int plse_stage_select(plse_handle h, int32_t p, int32_t gen, uint64_t seed, void *stream,
                      const int32_t *f_all, const int16_t *D_all, int32_t *accepted) {
    if (!h || !f_all || !D_all || !accepted || gen < 1 || gen >= (1 << 24)) return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    RC_TRY(stage_prepare(h, p, s));
    const int m = 2 * p;
    h->args.close = CloseArgs{nullptr, D_all, at<int32_t>(h, h->L.deg), at<uint16_t>(h, h->L.adj),
                              m, m, h->nv, h->P.spacing};
    h->args.select = make_select(h, p, gen, seed, nullptr, f_all, D_all, m, accepted);
    RC_TRY(upload_args(h, s));
    HIP_TRY(launch_close(single(h, &ArgBlock::close), 1, m, s));
    HIP_TRY(launch_select(single(h, &ArgBlock::select), 1, select_lds(h, p), h->L.pow2_sel,
                          h->args.select.keys_in_lds != 0, s));
    return PLSE_OK;
}

int plse_stage_match(plse_handle h, int32_t p, void *stream, const int16_t *D,
                     const uint64_t *uid, uint64_t *hist, int32_t *hcount, int32_t *partner,
                     int32_t *dpart) {
    if (!h || !D || !uid || !hist || !hcount || !partner || !dpart) return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    RC_TRY(stage_prepare(h, p, s));
    const Layout &L = h->L;
    h->args.hash = HashArgs{nullptr, uid, at<uint64_t>(h, L.hkeys), at<int32_t>(h, L.hvals), p,
                            L.hsize};
    h->args.match = MatchArgs{nullptr, D, nullptr, nullptr, uid, hist, hcount,
                              at<uint64_t>(h, L.hkeys), at<int32_t>(h, L.hvals), partner, dpart,
                              p, p, p, L.hsize, h->P.hist_len, 0, 0, 0u, 0u};
    RC_TRY(upload_args(h, s));
    HIP_TRY(launch_hash(single(h, &ArgBlock::hash), 1, p, L.hsize, s));
    HIP_TRY(launch_match(single(h, &ArgBlock::match), 1, p, s));
    return PLSE_OK;
}

int plse_stage_aux(plse_handle h, int32_t p, int32_t gen, uint64_t seed, void *stream,
                   const uint8_t *S, const int32_t *partner, const int32_t *dpart,
                   uint8_t *S_off) {
    if (!h || !S || !partner || !dpart || !S_off || gen < 1 || gen >= (1 << 24))
        return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    RC_TRY(stage_prepare(h, p, s));
    h->args.aux = AuxArgs{nullptr, S, partner, dpart, S_off, p, h->nv, h->stride, gen,
                          h->P.crossover, h->P.beta_num, h->P.beta_den, (uint32_t)seed,
                          (uint32_t)(seed >> 32)};
    RC_TRY(upload_args(h, s));
    HIP_TRY(launch_aux(single(h, &ArgBlock::aux), 1, p, s));
    return PLSE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Serving: continuous batching over a device arena (include/plse.h).
// ---------------------------------------------------------------------------
namespace {

struct Request {
    uint64_t ticket = 0;
    plse_instance *h = nullptr;
    int p = 0, G = 0;
    uint64_t seed = 0;
    size_t off = 0, bytes = 0;
    int steps = 0;   // generations finished on the device
    int queued = 0;  // generations enqueued
    Session *S = nullptr;       // the request's own session (graphs, events)
    hipStream_t st = nullptr;   // the request's own stream
    int status = PLSE_PENDING;
    double t_submit = 0, t_admit = -1, t_done = -1;
    std::vector<double> t_gen;  // wall time at the end of each generation
    std::vector<int8_t> grid;
    int filled = 0, best_gen = 0;
    uint64_t moves = 0;
    std::atomic<bool> cancel{false};  // plse_server_cancel on a resident request
    int caller_max_gens = 0;  // the handle's own setting, restored when the request ends
};

// Results of one finished request (its stream has drained).  The
// statistics cover the generations the device ran, which can exceed those
// the worker saw end (generations still queued at a cancel or a stop): their
// end times come from their end events, relative to the last generation the
// worker saw end (or to the first search's start event).
int collect(Request &r, hipStream_t s) {
    plse_instance *h = r.h;
    Ctl c{};
    HIP_TRY(hipMemcpyAsync(&c, at<Ctl>(h, h->L.ctl), sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (c.gens_run < 0 || c.gens_run > h->max_gens) return PLSE_E_HIP;
    std::vector<GenStat> gs((size_t)std::max(c.gens_run, 1));
    std::vector<uint8_t> star((size_t)h->stride);
    HIP_TRY(hipMemcpyAsync(gs.data(), at<GenStat>(h, h->L.stats), sizeof(GenStat) * gs.size(),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(star.data(), at<uint8_t>(h, h->L.Sstar), h->stride,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int gens = c.gens_run;
    RunResult rr = summarize(c, gs.data(), gens);
    h->last = rr.stats;
    h->gen_best = std::move(rr.gen_best);
    h->gen_cnt = std::move(rr.gen_cnt);
    r.best_gen = c.best_gen;
    r.moves = h->last.totals[C_MOVES];
    r.steps = std::max(r.steps, gens);  // generations run, seen ending or not
    if (r.S && (int)r.t_gen.size() < gens && (size_t)3 * gens <= r.S->ev.size()) {
        const size_t k = r.t_gen.size();
        const hipEvent_t ref = k ? r.S->ev[3 * (k - 1) + 2] : r.S->ev[0];
        const double base = k ? r.t_gen.back() : r.t_admit;
        for (int g = (int)k; g < gens; ++g) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ref, r.S->ev[3 * (size_t)g + 2]) != hipSuccess) break;
            r.t_gen.push_back(base + 1e-3 * ms);
        }
        (void)hipGetLastError();
    }
    r.grid.assign((size_t)h->n * h->n, 0);
    r.filled = best_grid(h->n, h->cell_v, h->grid, star.data(), gens, r.grid.data());
    return PLSE_OK;
}

}  // namespace

struct plse_server_s {
    uint8_t *arena = nullptr;
    size_t budget = 0;
    int max_slots = 1;
    hipStream_t stream = nullptr;
    hipEvent_t ready = nullptr;  // recorded on `stream` at creation
    int device = 0;
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request *> waiting;
    std::vector<Request *> resident;
    std::map<uint64_t, Request *> finished;
    std::set<uint64_t> live;  // submitted and not yet finished (waiting, admitting, resident)
    std::set<uint64_t> cancelled;  // cancel requests for tickets being admitted
    FirstFitArena blocks{0, kAlign};  // the arena's free blocks
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    // First-fit placement in the arena (256-byte granules); merge on release.
    bool place(Request *r) { return blocks.place(r->bytes, &r->off); }
    void release(Request *r) { blocks.release(r->off, r->bytes); }

    void finish(Request *r, int status) {
        cancelled.erase(r->ticket);
        r->status = status;
        r->t_done = now();
        r->h->ws = nullptr;
        r->h->ws_bytes = 0;
        r->h->max_gens = r->caller_max_gens;
        r->h->in_session = false;
        release(r);
        live.erase(r->ticket);
        finished[r->ticket] = r;
    }

    // The request's stream (ordered after work already on the server's
    // stream) and session: upload, initial population, generation graphs.
    int start(Request *r) {
        HIP_TRY(hipStreamCreateWithFlags(&r->st, hipStreamNonBlocking));
        HIP_TRY(hipStreamWaitEvent(r->st, ready, 0));
        r->S = new Session();
        r->S->hs = {r->h};
        r->S->p = r->p;
        HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&r->S->stop_host),
                              sizeof(int32_t) * Session::kStopRing));
        for (int q = 0; q < Session::kStopRing; ++q) r->S->stop_host[q] = 0;
        return session_begin(*r->S, &r->seed, r->st);
    }

    // Session and stream of a request (the stream drains first).
    void retire(Request *r) {
        if (r->st) (void)hipStreamSynchronize(r->st);
        delete r->S;
        r->S = nullptr;
        if (r->st) {
            (void)hipStreamDestroy(r->st);
            r->st = nullptr;
        }
    }

    void loop();
};

// Admission, then independent progress: every resident request has its own
// stream and session and keeps up to kAhead generations enqueued, so
// requests of different sizes overlap on the device and none waits for the
// generations of another.
void plse_server_s::loop() {
    (void)hipSetDevice(device);
    constexpr int kAhead = 2;
    static_assert(kAhead < Session::kStopRing, "stop flags of queued generations would collide");
    for (;;) {
        std::vector<Request *> fresh;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (resident.empty())
                cv.wait(lk, [&] { return stop || !waiting.empty(); });
            if (stop) return;
            // admission in arrival order, while the workspace fits the free
            // arena and a slot is free
            while (!waiting.empty() && (int)(resident.size() + fresh.size()) < max_slots) {
                Request *r = waiting.front();
                if (!place(r)) break;
                waiting.pop_front();
                r->h->ws = arena + r->off;
                r->h->ws_bytes = r->bytes;
                fresh.push_back(r);
            }
        }
        bool progressed = !fresh.empty();
        for (Request *r : fresh) {
            const int e = start(r);
            std::lock_guard<std::mutex> lk(mu);
            if (e) {
                retire(r);
                finish(r, e);
            } else {
                r->t_admit = now();
                if (cancelled.erase(r->ticket)) r->cancel.store(true);
                resident.push_back(r);
            }
        }
        std::vector<Request *> run;
        {
            std::lock_guard<std::mutex> lk(mu);
            run = resident;
        }
        std::vector<std::pair<Request *, int>> done;
        for (Request *r : run) {
            int rc = PLSE_OK;
            bool stopped = false;  // bound or iteration budget reached on the device
            while (r->steps < r->queued && !stopped) {
                const hipError_t q = hipEventQuery(r->S->ev[3 * (size_t)r->steps + 2]);
                if (q == hipErrorNotReady) break;
                if (q != hipSuccess) {
                    rc = hip_fail(q, "hipEventQuery");
                    break;
                }
                // this generation's copy of the flag landed before its end
                // event (at most kAhead generations are enqueued beyond it)
                stopped = __atomic_load_n(r->S->stop_host + r->steps % Session::kStopRing,
                                          __ATOMIC_ACQUIRE) != 0;
                r->steps += 1;
                r->t_gen.push_back(now());
                progressed = true;
            }
            const int fail_at = r->h->fail_at;
            const bool fault = fail_at && r->steps >= fail_at && r->steps < r->G;
            const bool cancel = r->cancel.load() && r->steps < r->G && !stopped;
            if (rc || fault || stopped || cancel || r->steps >= r->G) {
                // the request's stream drains before its workspace is released
                const hipError_t q = hipStreamSynchronize(r->st);
                if (!rc && q != hipSuccess) rc = hip_fail(q, "hipStreamSynchronize");
                if (!rc && fault) rc = PLSE_E_FAULT;
                if (!rc) rc = collect(*r, r->st);
                // cancelled: the best grid so far is returned with its status
                if (!rc && cancel) rc = PLSE_E_CANCELLED;
                done.emplace_back(r, rc);
                progressed = true;
                continue;
            }
            while (r->queued < r->G && r->queued - r->steps < kAhead &&
                   !(fail_at && r->queued >= fail_at)) {
                rc = session_step(*r->S, 1, r->st);
                if (rc) break;
                r->queued += 1;
            }
            if (rc) {
                (void)hipStreamSynchronize(r->st);
                done.emplace_back(r, rc);
                progressed = true;
            }
        }
        for (auto &d : done) retire(d.first);
        {
            std::lock_guard<std::mutex> lk(mu);
            for (auto &d : done) {
                resident.erase(std::find(resident.begin(), resident.end(), d.first));
                finish(d.first, d.second);
            }
        }
        if (!progressed) {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait_for(lk, std::chrono::microseconds(200),
                        [&] { return stop || !waiting.empty(); });
        }
    }
}

extern "C" {

int plse_server_create(size_t budget, void *device_ptr, int32_t max_slots, void *stream,
                       plse_server *out) {
    if (!out || !device_ptr || budget == 0 || max_slots < 1 || ((uintptr_t)device_ptr % kAlign))
        return PLSE_E_ARG;
    plse_server_s *s = new plse_server_s();
    s->arena = reinterpret_cast<uint8_t *>(device_ptr);
    s->budget = budget / kAlign * kAlign;
    s->max_slots = max_slots;
    s->stream = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetDevice(&s->device);
    s->t0 = std::chrono::steady_clock::now();
    s->blocks = FirstFitArena(s->budget, kAlign);
    set_attributes_once();
    hipError_t e = hipEventCreateWithFlags(&s->ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(s->ready, s->stream);
    if (e != hipSuccess) {
        if (s->ready) (void)hipEventDestroy(s->ready);
        delete s;
        return hip_fail(e, "plse_server_create");
    }
    s->worker = std::thread([s] { s->loop(); });
    *out = s;
    return PLSE_OK;
}

int plse_server_submit(plse_server s, plse_handle h, int32_t p, int32_t G, uint64_t seed,
                       uint64_t *ticket) {
    if (!s || !h || !ticket || p < 2 || p > PLSE_MAX_POPULATION || G < 1 ||
        G > PLSE_MAX_GENERATIONS)
        return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok || h->in_session) return PLSE_E_BUSY;
    Request *r = new Request();
    r->h = h;
    r->p = p;
    r->G = G;
    r->seed = seed;
    // the request's statistics records are sized by its generation budget
    r->caller_max_gens = h->max_gens;
    h->max_gens = G;
    r->bytes = round_up(plan(h, p).total, kAlign);
    if (r->bytes > s->budget) {
        h->max_gens = r->caller_max_gens;
        delete r;
        return PLSE_E_CAPACITY;
    }
    h->in_session = true;  // the server owns the handle until it is polled
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    r->t_submit = s->now();
    *ticket = r->ticket;
    s->live.insert(r->ticket);
    s->waiting.push_back(r);
    s->cv.notify_one();
    return PLSE_OK;
}

int plse_server_poll(plse_server s, uint64_t ticket, int8_t *best_grid, int32_t *filled,
                     plse_timing *t) {
    if (!s) return PLSE_E_ARG;
    Request *r = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->finished.find(ticket);
        if (it == s->finished.end()) return s->live.count(ticket) ? PLSE_PENDING : PLSE_E_ARG;
        r = it->second;
        s->finished.erase(it);
    }
    if (best_grid && !r->grid.empty()) std::memcpy(best_grid, r->grid.data(), r->grid.size());
    if (filled) *filled = r->filled;
    if (t) {
        t->submit_s = r->t_submit;
        t->admit_s = r->t_admit;
        t->done_s = r->t_done;
        t->best_s = time_to_best(r->t_gen, r->steps, r->best_gen, r->t_done);
        t->generations = r->steps;
        t->best_generation = r->best_gen;
        t->filled = r->filled;
        t->status = r->status;
        t->moves = r->moves;
    }
    const int st = r->status;
    delete r;
    return st;
}

int plse_server_cancel(plse_server s, uint64_t ticket) {
    if (!s) return PLSE_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->live.count(ticket)) return PLSE_E_ARG;  // unknown, or already finished
    for (auto it = s->waiting.begin(); it != s->waiting.end(); ++it) {
        Request *r = *it;
        if (r->ticket != ticket) continue;
        // never admitted: no workspace, no stream, no result
        s->waiting.erase(it);
        r->status = PLSE_E_CANCELLED;
        r->t_done = s->now();
        r->h->max_gens = r->caller_max_gens;
        r->h->in_session = false;
        s->live.erase(ticket);
        s->finished[ticket] = r;
        return PLSE_OK;
    }
    // admitted: the worker stops it at its next generation end; being
    // admitted: the cancellation is applied when it becomes resident
    for (Request *r : s->resident)
        if (r->ticket == ticket) {
            r->cancel.store(true);
            return PLSE_OK;
        }
    s->cancelled.insert(ticket);
    return PLSE_OK;
}

int plse_server_status(plse_server s, int32_t *waiting, int32_t *resident, int32_t *finished) {
    if (!s) return PLSE_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (waiting) *waiting = (int32_t)s->waiting.size();
    if (resident) *resident = (int32_t)s->resident.size();
    if (finished) *finished = (int32_t)s->finished.size();
    return PLSE_OK;
}

int plse_server_destroy(plse_server s) {
    if (!s) return PLSE_E_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    for (Request *r : s->waiting) {
        r->h->max_gens = r->caller_max_gens;
        r->h->in_session = false;
        delete r;
    }
    for (Request *r : s->resident) {
        s->retire(r);
        r->h->max_gens = r->caller_max_gens;
        r->h->in_session = false;
        r->h->ws = nullptr;
        delete r;
    }
    for (auto &kv : s->finished) delete kv.second;
    (void)hipEventDestroy(s->ready);
    delete s;
    return PLSE_OK;
}

}  // extern "C"

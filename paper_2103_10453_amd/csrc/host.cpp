// host.cpp -- libplse host side: instance preprocessing (Section 2.2, Alg. 1),
// workspace planning, the per-generation HIP graph (Alg. 2) and the C ABI of
// include/plse.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/plse.h"
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
int colour_bits(int n) {
    int b = 0;
    while ((1 << b) <= n) ++b;
    return b;
}

// Offsets of every device array of one handle, for a population p.
struct Layout {
    size_t vrc, vrec, dom, rowl, coll, rowc, colc;
    size_t ctl, stats, Sstar;
    size_t S_all, S_off, S_tmp, f_all, f_tmp, uid, uid_tmp, hist, hist_tmp, hc, hc_tmp, cnt;
    size_t tabu, planes, D, deg, adj, keys, rej, acc, hkeys, hvals, partner, dpart;
    size_t total;
    int pow2_sel, hsize;
};

}  // namespace

struct plse_instance {
    int n = 0, nv = 0, l = 0, ub = 0, nd = 0, stride = 16;
    std::vector<int8_t> grid;
    std::vector<int> cell_v;  // -1 prefilled, -2 impossible, else vertex id
    // host images of the device instance tables
    std::vector<uint16_t> vrc;
    std::vector<uint32_t> vrec;  // 8 words per vertex
    std::vector<uint8_t> dom;    // domain colour lists
    std::vector<uint32_t> rowl, coll;
    std::vector<uint8_t> rowc, colc;

    Params P{};
    int lpv = 0;  // lanes per eligible vertex in PLITS; 0: automatic
    int wpb = 0;  // waves per block in PLITS; 0: automatic

    uint8_t *ws = nullptr;
    size_t ws_bytes = 0;

    // generation graphs: [gen_begin, plits] and [best .. aux]; HIP events
    // around the first measure the tabu-search kernel on the caller's stream
    hipGraphExec_t exec_ls = nullptr, exec_rest = nullptr;
    bool graph_valid = false;
    int graph_p = 0;
    uint64_t graph_seed = 0;

    // session (plse_begin / plse_step / plse_end)
    bool in_session = false;
    int sess_p = 0;
    uint64_t sess_seed = 0;
    int sess_steps = 0;
    std::vector<hipEvent_t> ev;  // 3 per generation: before plits, after, end of generation
    std::vector<float> ms_plits, ms_rest;

    plse_stats last{};
    std::vector<int32_t> gen_best;
    std::vector<uint64_t> gen_cnt;
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

std::once_flag g_attr_once;
int g_lds_limit = 65536;  // dynamic LDS per block every kernel may use

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

// PLITS per-wave LDS: S, row/column colour counts, eligibility bitmap,
// per-vertex tabu expiry, eligible-vertex list.
struct PlitsLds {
    int per_wave, off_h, off_bm, off_tm, off_el;
};

PlitsLds plits_lds(const plse_instance *h) {
    PlitsLds L;
    const int W = (h->nv + 31) / 32;
    L.off_h = h->stride;
    L.off_bm = L.off_h + (int)round_up((size_t)2 * h->n * (h->n + 1), 16);
    L.off_tm = L.off_bm + (int)round_up((size_t)W * 4, 16);
    L.off_el = L.off_tm + (int)round_up((size_t)h->nv * 4, 16);
    L.per_wave = L.off_el + (int)round_up((size_t)h->nv * 2, 16);
    return L;
}

// Waves per block maximising resident waves per CU under the LDS budget.
int choose_wpb(const plse_instance *h) {
    if (h->wpb) return h->wpb;
    const int per = plits_lds(h).per_wave;
    const int lim = max_lds_per_block();
    int best = 1, best_waves = 0;
    for (int w : {1, 2, 4}) {
        if (w * per > lim) continue;
        const int waves = (lim / (w * per)) * w;
        if (waves >= best_waves) {
            best = w;
            best_waves = waves;
        }
    }
    return best;
}

// Lanes per eligible vertex: about four domain colours per lane.
int choose_lpv(const plse_instance *h) {
    if (h->lpv) return h->lpv;
    const double mean = h->nv ? (double)h->nd / h->nv : 1.0;
    if (mean <= 6.0) return 1;
    if (mean <= 12.0) return 2;
    if (mean <= 24.0) return 4;
    return 8;
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
    L.dom = take(nd + 16);
    L.rowl = take(4 * n * n);
    L.coll = take(4 * n * n);
    L.rowc = take(n);
    L.colc = take(n);
    L.ctl = take(sizeof(Ctl));
    L.stats = take(sizeof(GenStat) * PLSE_MAX_GENERATIONS);
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
    L.tabu = take((size_t)p * (nd + nv) * 4);
    L.planes = take(m * W * B * 4);
    L.D = take(m * m * 2);
    L.deg = take(4 * m);
    L.adj = take(2 * m * kAdj);
    L.pow2_sel = next_pow2(std::max<int>(4, (int)m));
    L.keys = take(8 * (size_t)L.pow2_sel);
    L.rej = take(4 * m);
    L.acc = take(4 * (size_t)p);
    L.hsize = next_pow2(std::max<int>(4, (int)m));
    L.hkeys = take(8 * (size_t)L.hsize);
    L.hvals = take(4 * (size_t)L.hsize);
    L.partner = take(4 * (size_t)p);
    L.dpart = take(4 * (size_t)p);
    L.total = o;
    return L;
}

template <typename T>
T *at(plse_instance *h, size_t off) {
    return reinterpret_cast<T *>(h->ws + off);
}

DevInstance dev_instance(plse_instance *h, const Layout &L) {
    DevInstance I;
    I.n = h->n;
    I.nv = h->nv;
    I.nd = h->nd;
    I.stride = h->stride;
    I.l = h->l;
    I.ub = h->ub;
    I.vrc = at<uint16_t>(h, L.vrc);
    I.vrec = at<void>(h, L.vrec);
    I.dom = at<uint8_t>(h, L.dom);
    I.rowl = at<uint32_t>(h, L.rowl);
    I.coll = at<uint32_t>(h, L.coll);
    I.rowc = at<uint8_t>(h, L.rowc);
    I.colc = at<uint8_t>(h, L.colc);
    return I;
}

int upload_instance(plse_instance *h, const Layout &L, hipStream_t s) {
    auto put = [&](size_t off, const void *src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync(h->ws + off, src, bytes, hipMemcpyHostToDevice, s);
    };
    HIP_TRY(put(L.vrc, h->vrc.data(), 2 * h->vrc.size()));
    HIP_TRY(put(L.vrec, h->vrec.data(), 4 * h->vrec.size()));
    HIP_TRY(put(L.dom, h->dom.data(), h->dom.size()));
    HIP_TRY(put(L.rowl, h->rowl.data(), 4 * h->rowl.size()));
    HIP_TRY(put(L.coll, h->coll.data(), 4 * h->coll.size()));
    HIP_TRY(put(L.rowc, h->rowc.data(), h->rowc.size()));
    HIP_TRY(put(L.colc, h->colc.data(), h->colc.size()));
    return PLSE_OK;
}

PlitsArgs plits_args(plse_instance *h, const Layout &L, int p, int gen_fixed, uint64_t seed,
                     const uint8_t *S_in, uint8_t *S_out, int32_t *f_out, uint64_t *cnt,
                     const Ctl *ctl) {
    PlitsArgs a{};
    a.I = dev_instance(h, L);
    a.P = h->P;
    a.S_in = S_in;
    a.S_out = S_out;
    a.f_out = f_out;
    a.cnt_out = cnt;
    a.tabu = at<uint32_t>(h, L.tabu);
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
    return a;
}

int launch_select_stage(plse_instance *h, const Layout &L, int p, int gen_fixed, uint64_t seed,
                        const Ctl *ctl, const int32_t *f_all, const int16_t *D, int ld,
                        int32_t *acc, hipStream_t s) {
    const int m = 2 * p;
    CloseArgs ca{ctl, D, at<int32_t>(h, L.deg), at<uint16_t>(h, L.adj), m, ld, h->nv,
                 h->P.spacing};
    HIP_TRY(launch_close(ca, s));
    SelectArgs sa{};
    sa.ctl = ctl;
    sa.f_all = f_all;
    sa.D = D;
    sa.deg = at<int32_t>(h, L.deg);
    sa.adj = at<uint16_t>(h, L.adj);
    sa.keys_g = at<uint64_t>(h, L.keys);
    sa.rej = at<int32_t>(h, L.rej);
    sa.acc = acc;
    sa.p = p;
    sa.m = m;
    sa.ld = ld;
    sa.nv = h->nv;
    sa.pow2 = L.pow2_sel;
    sa.keys_in_lds =
        select_lds_bytes(m, L.pow2_sel, true) <= (size_t)max_lds_per_block() ? 1 : 0;
    sa.gen_fixed = gen_fixed;
    sa.spacing = h->P.spacing;
    sa.seed_lo = (uint32_t)seed;
    sa.seed_hi = (uint32_t)(seed >> 32);
    HIP_TRY(launch_select(sa, s));
    return PLSE_OK;
}

int launch_match_stage(plse_instance *h, const Layout &L, int p, const Ctl *ctl,
                       const int16_t *D, int ld, const int32_t *idx, const uint64_t *uid,
                       uint64_t *hist, int32_t *hc, int32_t *partner, int32_t *dpart,
                       hipStream_t s) {
    HashArgs ha{ctl, uid, at<uint64_t>(h, L.hkeys), at<int32_t>(h, L.hvals), p, L.hsize};
    MatchArgs ma{ctl, D, idx, uid, hist, hc, at<uint64_t>(h, L.hkeys), at<int32_t>(h, L.hvals),
                 partner, dpart, p, ld, L.hsize, h->P.hist_len};
    HIP_TRY(launch_match(ha, ma, s));
    return PLSE_OK;
}

// One generation of Alg. 2 on the device; every kernel reads the generation
// number and the stop flag from the control block.
int enqueue_local_search(plse_instance *h, const Layout &L, int p, uint64_t seed,
                         hipStream_t s) {
    Ctl *ctl = at<Ctl>(h, L.ctl);
    const int st = h->stride;
    uint8_t *S_new = at<uint8_t>(h, L.S_all) + (size_t)p * st;
    int32_t *f_all = at<int32_t>(h, L.f_all);
    HIP_TRY(launch_gen_begin(ctl, s));
    PlitsArgs pa = plits_args(h, L, p, 0, seed, at<uint8_t>(h, L.S_off), S_new, f_all + p,
                              at<uint64_t>(h, L.cnt), ctl);
    HIP_TRY(launch_plits(pa, choose_lpv(h), choose_wpb(h), s));
    return PLSE_OK;
}

int enqueue_rest(plse_instance *h, const Layout &L, int p, uint64_t seed, hipStream_t s) {
    Ctl *ctl = at<Ctl>(h, L.ctl);
    const int st = h->stride, m = 2 * p;
    uint8_t *S_all = at<uint8_t>(h, L.S_all);
    uint8_t *S_new = S_all + (size_t)p * st;
    int32_t *f_all = at<int32_t>(h, L.f_all);
    BestArgs ba{ctl, at<GenStat>(h, L.stats), f_all + p, S_new, at<uint64_t>(h, L.cnt),
                at<uint8_t>(h, L.Sstar), p, st, h->n * h->n - h->l, h->ub, h->P.stop_at_ub};
    HIP_TRY(launch_best(ba, s));
    HIP_TRY(launch_distances(ctl, S_all, at<uint32_t>(h, L.planes), at<int16_t>(h, L.D), m,
                             h->nv, st, m, colour_bits(h->n), s));
    int rc = launch_select_stage(h, L, p, 0, seed, ctl, f_all, at<int16_t>(h, L.D), m,
                                 at<int32_t>(h, L.acc), s);
    if (rc) return rc;
    GatherArgs ga{ctl, at<int32_t>(h, L.acc), S_all, f_all, at<uint64_t>(h, L.uid),
                  at<uint64_t>(h, L.hist), at<int32_t>(h, L.hc), at<uint8_t>(h, L.S_tmp),
                  at<int32_t>(h, L.f_tmp), at<uint64_t>(h, L.uid_tmp),
                  at<uint64_t>(h, L.hist_tmp), at<int32_t>(h, L.hc_tmp), p, st};
    HIP_TRY(launch_gather(ga, s));
    rc = launch_match_stage(h, L, p, ctl, at<int16_t>(h, L.D), m, at<int32_t>(h, L.acc),
                            at<uint64_t>(h, L.uid), at<uint64_t>(h, L.hist), at<int32_t>(h, L.hc),
                            at<int32_t>(h, L.partner), at<int32_t>(h, L.dpart), s);
    if (rc) return rc;
    AuxArgs xa{ctl, S_all, at<int32_t>(h, L.partner), at<int32_t>(h, L.dpart),
               at<uint8_t>(h, L.S_off), p, h->nv, st, 0, h->P.beta_num, h->P.beta_den,
               (uint32_t)seed, (uint32_t)(seed >> 32)};
    HIP_TRY(launch_aux(xa, s));
    return PLSE_OK;
}

void drop_graph(plse_instance *h) {
    if (h->exec_ls) (void)hipGraphExecDestroy(h->exec_ls);
    if (h->exec_rest) (void)hipGraphExecDestroy(h->exec_rest);
    h->exec_ls = h->exec_rest = nullptr;
    h->graph_valid = false;
}

template <typename F>
int capture(F &&enqueue, hipGraphExec_t *out) {
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e);
    }
    const int rc = enqueue(cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e);
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        *out = nullptr;
        return hip_fail(e);
    }
    return PLSE_OK;
}

int capture_generation(plse_instance *h, const Layout &L, int p, uint64_t seed) {
    drop_graph(h);
    int rc = capture([&](hipStream_t cs) { return enqueue_local_search(h, L, p, seed, cs); },
                     &h->exec_ls);
    if (rc) return rc;
    rc = capture([&](hipStream_t cs) { return enqueue_rest(h, L, p, seed, cs); }, &h->exec_rest);
    if (rc) {
        drop_graph(h);
        return rc;
    }
    h->graph_valid = true;
    h->graph_p = p;
    h->graph_seed = seed;
    return PLSE_OK;
}

int ensure_events(plse_instance *h, size_t count) {
    while (h->ev.size() < count) {
        hipEvent_t e = nullptr;
        HIP_TRY(hipEventCreate(&e));
        h->ev.push_back(e);
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

int check_ws(plse_instance *h, int p, Layout *L) {
    if (p < 2 || p > PLSE_MAX_POPULATION) return PLSE_E_ARG;
    *L = plan(h, p);
    if (!h->ws || h->ws_bytes < L->total) return PLSE_E_WORKSPACE;
    set_attributes_once();
    return PLSE_OK;
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
    h->rowc.assign(n, 0);
    h->colc.assign(n, 0);
    h->rowl.assign((size_t)n * n, 0);
    h->coll.assign((size_t)n * n, 0);
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
            h->rowl[(size_t)i * n + h->rowc[i]++] = (uint32_t)v | ((uint32_t)j << 16);
            h->coll[(size_t)j * n + h->colc[j]++] = (uint32_t)v | ((uint32_t)i << 16);
        }
    h->ub = (h->l == 1) ? n * n - 2 : n * n - h->l;
    // vertex records: 128-bit domain mask, first tabu slot (sum of earlier
    // domain sizes), coordinates
    h->vrec.assign((size_t)h->nv * 8, 0);
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
        for (int k = 1; k <= n; ++k)
            if ((dmask[2 * v + (k >> 6)] >> (k & 63)) & 1ull) h->dom.push_back((uint8_t)k);
        off += d;
    }
    h->nd = (int)off;
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
    h->P.hist_len = kHist;
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
    if (!g.ok) return PLSE_E_BUSY;
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
    } else if (k == "nn_history") {
        if (v < 0 || v > kHist) return PLSE_E_PARAM;
        P.hist_len = (int32_t)v;
    } else if (k == "lanes_per_vertex") {
        if (v != 0 && v != 1 && v != 2 && v != 4 && v != 8) return PLSE_E_PARAM;
        h->lpv = (int)v;
    } else if (k == "waves_per_block") {
        if (v != 0 && v != 1 && v != 2 && v != 4) return PLSE_E_PARAM;
        h->wpb = (int)v;
    } else {
        return PLSE_E_PARAM;
    }
    drop_graph(h);
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
    else if (k == "nn_history") *v = P.hist_len;
    else if (k == "lanes_per_vertex") *v = choose_lpv(h);
    else if (k == "waves_per_block") *v = h->wpb ? h->wpb : choose_wpb(h);
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
    if (!g.ok) return PLSE_E_BUSY;
    drop_graph(h);
    h->ws = reinterpret_cast<uint8_t *>(ptr);
    h->ws_bytes = ptr ? bytes : 0;
    return PLSE_OK;
}

int plse_begin(plse_handle h, int32_t p, uint64_t seed, void *stream) {
    if (!h) return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    Layout L;
    int rc = check_ws(h, p, &L);
    if (rc) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    rc = upload_instance(h, L, s);
    if (rc) return rc;
    Ctl *ctl = at<Ctl>(h, L.ctl);
    HIP_TRY(launch_ctl_reset(ctl, s));
    InitArgs ia{dev_instance(h, L), at<uint8_t>(h, L.S_all), at<int32_t>(h, L.f_all), p,
                next_pow2(std::max(4, h->nv)), (uint32_t)seed, (uint32_t)(seed >> 32)};
    HIP_TRY(launch_init(ia, s));
    HIP_TRY(launch_pop_setup(p, h->stride, at<uint64_t>(h, L.uid), at<int32_t>(h, L.hc),
                             at<uint8_t>(h, L.S_all), at<uint8_t>(h, L.S_off), s));
    HIP_TRY(launch_fill_zero(at<uint32_t>(h, L.tabu), (size_t)p * (h->nd + h->nv), s));
    if (!h->graph_valid || h->graph_p != p || h->graph_seed != seed) {
        rc = capture_generation(h, L, p, seed);
        if (rc) return rc;
    }
    h->in_session = true;
    h->sess_p = p;
    h->sess_seed = seed;
    h->sess_steps = 0;
    return PLSE_OK;
}

int plse_step(plse_handle h, int32_t generations, void *stream) {
    if (!h || generations < 0) return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    if (!h->in_session || !h->graph_valid) return PLSE_E_ARG;
    if (h->sess_steps + generations > PLSE_MAX_GENERATIONS) return PLSE_E_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int rc = ensure_events(h, 3 * (size_t)(h->sess_steps + generations));
    if (rc) return rc;
    for (int g = 0; g < generations; ++g) {
        const size_t k = 3 * (size_t)(h->sess_steps + g);
        HIP_TRY(hipEventRecord(h->ev[k], s));
        HIP_TRY(hipGraphLaunch(h->exec_ls, s));
        HIP_TRY(hipEventRecord(h->ev[k + 1], s));
        HIP_TRY(hipGraphLaunch(h->exec_rest, s));
        HIP_TRY(hipEventRecord(h->ev[k + 2], s));
    }
    h->sess_steps += generations;
    return PLSE_OK;
}

int plse_end(plse_handle h, void *stream, int8_t *best_grid, int32_t *filled) {
    if (!h || !best_grid || !filled) return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    if (!h->in_session) return PLSE_E_ARG;
    h->in_session = false;
    const Layout L = plan(h, h->sess_p);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int st = h->stride;
    const int G = std::max(h->sess_steps, 1);
    Ctl hc{};
    std::vector<GenStat> gs((size_t)G);
    std::vector<uint8_t> sstar((size_t)st);
    HIP_TRY(hipMemcpyAsync(&hc, at<Ctl>(h, L.ctl), sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(gs.data(), at<GenStat>(h, L.stats), sizeof(GenStat) * G,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(sstar.data(), at<uint8_t>(h, L.Sstar), st, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int gens = hc.gens_run;
    h->gen_best.assign((size_t)gens, 0);
    h->gen_cnt.assign((size_t)gens * kCounters, 0);
    plse_stats &ls = h->last;
    std::memset(&ls, 0, sizeof(ls));
    for (int g = 0; g < gens; ++g) {
        h->gen_best[g] = gs[g].best_f;
        for (int q = 0; q < kCounters; ++q) {
            h->gen_cnt[(size_t)g * kCounters + q] = gs[g].cnt[q];
            ls.totals[q] += gs[g].cnt[q];
        }
    }
    ls.generations_run = gens;
    ls.best_f = hc.fstar;
    ls.best_generation = hc.best_gen;
    h->ms_plits.assign((size_t)h->sess_steps, 0.f);
    h->ms_rest.assign((size_t)h->sess_steps, 0.f);
    for (int g = 0; g < h->sess_steps; ++g) {
        HIP_TRY(hipEventElapsedTime(&h->ms_plits[g], h->ev[3 * g], h->ev[3 * g + 1]));
        HIP_TRY(hipEventElapsedTime(&h->ms_rest[g], h->ev[3 * g + 1], h->ev[3 * g + 2]));
    }
    // best grid: prefilled cells plus S* on the vertices
    const int n = h->n;
    int cnt = 0;
    for (int c = 0; c < n * n; ++c) {
        const int v = h->cell_v[c];
        const int8_t val =
            (v == -1) ? h->grid[c] : ((v >= 0 && gens > 0) ? (int8_t)sstar[v] : (int8_t)0);
        best_grid[c] = val;
        cnt += (val != 0);
    }
    *filled = cnt;
    return PLSE_OK;
}

int plse_solve(plse_handle h, int32_t p, int32_t G, uint64_t seed, void *stream,
               int8_t *best_grid, int32_t *filled) {
    if (!h || !best_grid || !filled || G < 1 || G > PLSE_MAX_GENERATIONS) return PLSE_E_ARG;
    int rc = plse_begin(h, p, seed, stream);
    if (rc) return rc;
    rc = plse_step(h, G, stream);
    if (rc) {
        int8_t *tmp = new int8_t[(size_t)h->n * h->n];
        int32_t f = 0;
        (void)plse_end(h, stream, tmp, &f);
        delete[] tmp;
        return rc;
    }
    return plse_end(h, stream, best_grid, filled);
}

int plse_last_timing(plse_handle h, int32_t *steps, float *plits_ms, float *rest_ms) {
    if (!h || !steps) return PLSE_E_ARG;
    *steps = (int32_t)h->ms_plits.size();
    if (plits_ms) std::copy(h->ms_plits.begin(), h->ms_plits.end(), plits_ms);
    if (rest_ms) std::copy(h->ms_rest.begin(), h->ms_rest.end(), rest_ms);
    return PLSE_OK;
}

int plse_last_stats(plse_handle h, plse_stats *out, int32_t *per_gen_best_f,
                    uint64_t *per_gen_counters) {
    if (!h || !out) return PLSE_E_ARG;
    *out = h->last;
    if (per_gen_best_f)
        std::copy(h->gen_best.begin(), h->gen_best.end(), per_gen_best_f);
    if (per_gen_counters)
        std::copy(h->gen_cnt.begin(), h->gen_cnt.end(), per_gen_counters);
    return PLSE_OK;
}

void plse_destroy(plse_handle h) {
    if (!h) return;
    drop_graph(h);
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
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
    Layout L;
    int rc = check_ws(h, p, &L);
    if (rc) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    rc = upload_instance(h, L, s);
    if (rc) return rc;
    InitArgs ia{dev_instance(h, L), S, f, p, next_pow2(std::max(4, h->nv)), (uint32_t)seed,
                (uint32_t)(seed >> 32)};
    HIP_TRY(launch_init(ia, s));
    return PLSE_OK;
}

int plse_stage_plits(plse_handle h, int32_t p, int32_t gen, uint64_t seed, void *stream,
                     const uint8_t *S_in, uint8_t *S_out, int32_t *f_out, uint64_t *counters) {
    if (!h || !S_in || !S_out || !f_out || !counters || S_in == S_out || gen < 1 ||
        gen >= (1 << 24))
        return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    Layout L;
    int rc = check_ws(h, p, &L);
    if (rc) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    rc = upload_instance(h, L, s);
    if (rc) return rc;
    PlitsArgs a = plits_args(h, L, p, gen, seed, S_in, S_out, f_out, counters, nullptr);
    HIP_TRY(launch_fill_zero(at<uint32_t>(h, L.tabu), (size_t)p * (h->nd + h->nv), s));
    HIP_TRY(launch_plits(a, choose_lpv(h), choose_wpb(h), s));
    return PLSE_OK;
}

int plse_stage_distances(plse_handle h, int32_t m, void *stream, const uint8_t *S, int16_t *D) {
    if (!h || !S || !D || m < 1) return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    Layout L;
    int rc = check_ws(h, std::max(2, (m + 1) / 2), &L);
    if (rc) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(launch_distances(nullptr, S, at<uint32_t>(h, L.planes), D, m, h->nv, h->stride, m,
                             colour_bits(h->n), s));
    return PLSE_OK;
}

int plse_stage_select(plse_handle h, int32_t p, int32_t gen, uint64_t seed, void *stream,
                      const int32_t *f_all, const int16_t *D_all, int32_t *accepted) {
    if (!h || !f_all || !D_all || !accepted || gen < 1 || gen >= (1 << 24)) return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    Layout L;
    int rc = check_ws(h, p, &L);
    if (rc) return rc;
    return launch_select_stage(h, L, p, gen, seed, nullptr, f_all, D_all, 2 * p, accepted,
                               reinterpret_cast<hipStream_t>(stream));
}

int plse_stage_match(plse_handle h, int32_t p, void *stream, const int16_t *D,
                     const uint64_t *uid, uint64_t *hist, int32_t *hcount, int32_t *partner,
                     int32_t *dpart) {
    if (!h || !D || !uid || !hist || !hcount || !partner || !dpart) return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    Layout L;
    int rc = check_ws(h, p, &L);
    if (rc) return rc;
    return launch_match_stage(h, L, p, nullptr, D, p, nullptr, uid, hist, hcount, partner, dpart,
                              reinterpret_cast<hipStream_t>(stream));
}

int plse_stage_aux(plse_handle h, int32_t p, int32_t gen, uint64_t seed, void *stream,
                   const uint8_t *S, const int32_t *partner, const int32_t *dpart,
                   uint8_t *S_off) {
    if (!h || !S || !partner || !dpart || !S_off || gen < 1 || gen >= (1 << 24))
        return PLSE_E_ARG;
    BusyGuard guard(h);
    if (!guard.ok) return PLSE_E_BUSY;
    Layout L;
    int rc = check_ws(h, p, &L);
    if (rc) return rc;
    AuxArgs xa{nullptr, S, partner, dpart, S_off, p, h->nv, h->stride, gen, h->P.beta_num,
               h->P.beta_den, (uint32_t)seed, (uint32_t)(seed >> 32)};
    HIP_TRY(launch_aux(xa, reinterpret_cast<hipStream_t>(stream)));
    return PLSE_OK;
}

}  // extern "C"

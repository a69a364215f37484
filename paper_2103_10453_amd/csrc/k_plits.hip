// k_plits.hip -- PLITS, the two-phase tabu search of Section 3.3 (Alg. 3),
// one wave64 per individual on gfx950.
//
// Conflict counts in factored form.  In the Latin square graph the neighbours
// of a cell are exactly the other cells of its row and of its column
// (Section 2.1), so the incremental evaluation table of Section 3.3,
// conf[v][k] = #neighbours of v coloured k, equals
//     rowcnt[r(v)][k] + colcnt[c(v)][k] - 2 [S(v) = k]
// with rowcnt/colcnt the number of vertices of each colour per row and per
// column.  These 2 n (n+1) byte counters replace the sum_v |D*(v)| table, live
// in LDS, and a move updates four of them instead of every neighbour's entry.
//
// Candidate rows.  The moves of vertex v are the colours of {0} u D*(v)
// (0: uncolour), kept ascending at cand[v][0 .. d] with d = |D*(v)|, TS
// positions per vertex; the tabu expiry of each move sits at the same
// position of tabu[v].  An iteration cuts the rows of its eligible vertices
// into chunks of CH consecutive positions and deals the chunks to the 64
// lanes round by round, so every lane evaluates CH moves per round whatever
// the domain sizes are.
//
// Per wave (LDS): S[stride] colours, rowcnt|colcnt, the eligibility bitmap of
//   V_0 u C(S), tm8[|V|] (per vertex: whether this phase wrote its tabu row,
//   and its latest tabu expiry relative to a base advanced by 128 iterations
//   at a time, 255 = "treat as live"; a vertex not live has no tabu move),
//   the 64 eligible vertices being dealt, a ring of chunk descriptors, the
//   colour halves of the iteration's tie values and bit planes of the
//   vertices' chunk counts.
// Per individual (HBM): tabu[|V|][TS] "allowed from" iteration of every move,
//   read only for vertices with a live entry; all zero between phases (each
//   phase clears the rows it wrote).
//
// One iteration:
//   1. eligible vertices V_0 u C(S) from the bitmap (wave prefix sum);
//   2. chunks of their candidate rows, CH moves per lane and round: move value
//      from the row/column counts, admissibility from tabu and aspiration,
//      best key per lane: (value, tie value) above the move id v (n+1) + k,
//      the tie value being the top half of fmix32(w1 ^ v) ^ fmix32(w2 ^ k)
//      for the iteration's random words w1, w2;
//   3. a DPP wave minimum of the upper key words, then (only when several
//      lanes hold it) of their move ids, picks the unique best admissible
//      move;
//   4. counts, colour, eligibility bits of the row/column vertices holding the
//      old or new colour, tenure, tabu entry, best-solution snapshot.
#include "device_common.h"
#include "kernels.h"

namespace plse {

namespace {

struct WaveState {
    uint8_t *S;
    uint8_t *H;        // rowcnt [n][n+1] then colcnt [n][n+1]
    uint32_t *bm;
    uint8_t *tm8;      // [|V|] 0: no tabu entry this phase; 1: entries, all expired;
                       // m in 2..254: latest expiry = base + m - 1; 255: treat as live
    uint16_t *stage;   // [kPlitsStage] eligible vertices of consecutive ranks
    uint32_t *ring;    // chunk descriptors: vertex | chunk index << 16 | live << 31
    uint16_t *hk;      // [n+1] colour halves of the iteration's tie values
    uint32_t *planes;  // [B][W] bit b of floor(|D*(v)| / CH) (chunks per row - 1)
    int nplanes;
};

// Per-individual counters of one launch (moves = iterations - idle ones).
// Iterations per phase are at most 2^31 - 1, so the per-iteration ones fit 32
// bits; eligible-vertex and update sums take 64.
struct Cnt {
    uint32_t iters, idle, snaps, repairs;
    uint64_t elig, nupd, cupd;
};

struct Scal {
    int64_t F, Fbest;
    int32_t f, c, nC;  // uncoloured, conflicting edges, conflicting vertices
    int32_t fbest, cbest;
};

// Position of colour k in a candidate row with 128-bit domain mask a: 0 for
// k = 0, else 1 + the number of domain colours below k.
__device__ __forceinline__ uint32_t position_in(const u32x4 a, int k) {
    if (k == 0) return 0u;
    const uint64_t m0 = ((uint64_t)a.y << 32) | a.x;
    const uint64_t m1 = ((uint64_t)a.w << 32) | a.z;
    if (k < 64) return 1u + (uint32_t)__popcll(m0 & ((1ull << k) - 1ull));
    return 1u + (uint32_t)__popcll(m0) + (uint32_t)__popcll(m1 & ((1ull << (k - 64)) - 1ull));
}

// S from `src`; row/column colour counts; eligibility bitmap; f, c, |C(S)|.
__device__ void setup_state(const DevInstance &I, const uint8_t *src, const WaveState &ws,
                            Scal &sc) {
    const int lane = lane_id();
    const int n = I.n, nv = I.nv, np1 = n + 1;
    for (int q = lane; q < (I.stride >> 4); q += 64)
        reinterpret_cast<u32x4 *>(ws.S)[q] = gload4(reinterpret_cast<const u32x4 *>(src) + q);
    const int hbytes = 2 * n * np1;
    uint32_t *h32 = reinterpret_cast<uint32_t *>(ws.H);
    for (int q = lane; q < (hbytes + 3) / 4; q += 64) h32[q] = 0u;
    PLSE_WAVE_SYNC();
    for (int v = lane; v < nv; v += 64) {
        const int s = ws.S[v];
        if (s) {
            const uint32_t rc = gptr(I.vrc)[v];
            const int a = (int)(rc & 0xFFu) * np1 + s;
            const int b = n * np1 + (int)(rc >> 8) * np1 + s;
            atomicAdd(&h32[a >> 2], 1u << ((a & 3) * 8));
            atomicAdd(&h32[b >> 2], 1u << ((b & 3) * 8));
        }
    }
    PLSE_WAVE_SYNC();
    const uint8_t *rowH = ws.H, *colH = ws.H + n * np1;
    const int W = (nv + 31) >> 5;
    uint32_t f = 0, c2 = 0, nC = 0;
    for (int w = lane; w < W; w += 64) {
        uint32_t bits = 0u;
        const int vend = min(nv, (w + 1) * 32);
        for (int v = w * 32; v < vend; ++v) {
            const int s = ws.S[v];
            int own = 0;
            if (s) {
                const uint32_t rc = gptr(I.vrc)[v];
                own = (int)rowH[(rc & 0xFFu) * np1 + s] + (int)colH[(rc >> 8) * np1 + s] - 2;
            }
            if (s == 0 || own > 0) bits |= 1u << (v & 31);
            f += (s == 0);
            c2 += (uint32_t)own;
            nC += (s != 0 && own > 0);
        }
        ws.bm[w] = bits;
    }
    for (int q = lane; q < (nv + 3) >> 2; q += 64) reinterpret_cast<uint32_t *>(ws.tm8)[q] = 0u;
    PLSE_WAVE_SYNC();
    sc.f = (int32_t)wave_sum_u32_dpp(f);
    sc.c = (int32_t)(wave_sum_u32_dpp(c2) >> 1);  // each conflicting edge seen twice
    sc.nC = (int32_t)wave_sum_u32_dpp(nC);
}

__device__ __forceinline__ void snapshot(const DevInstance &I, const uint8_t *S, uint8_t *dst) {
    for (int q = lane_id(); q < (I.stride >> 4); q += 64)
        gstore4(reinterpret_cast<u32x4 *>(dst) + q, reinterpret_cast<const u32x4 *>(S)[q]);
}

// Zero the tabu rows this phase wrote (vertices with a nonzero mark).
__device__ void clear_tabu(const DevInstance &I, uint32_t *tabu, const WaveState &ws) {
    const int q4 = I.ts >> 2;
    for (int v = lane_id(); v < I.nv; v += 64) {
        if (ws.tm8[v] != 0) {
            u32x4 *tb = reinterpret_cast<u32x4 *>(tabu + (size_t)v * I.ts);
            for (int t = 0; t < q4; ++t) gstore4(tb + t, u32x4{0u, 0u, 0u, 0u});
        }
    }
}

// CH consecutive candidate colours (bytes) and their tabu expiries.
template <int CH>
struct Chunk;

template <>
struct Chunk<2> {
    static __device__ __forceinline__ uint32_t colours(const uint8_t *p) {
        return *gptr(reinterpret_cast<const uint16_t *>(p));
    }
    static __device__ __forceinline__ void tabu(const uint32_t *p, uint32_t *t) {
        const u32x2 a = gload2(p);
        t[0] = a.x;
        t[1] = a.y;
    }
};

template <>
struct Chunk<4> {
    static __device__ __forceinline__ uint32_t colours(const uint8_t *p) {
        return *gptr(reinterpret_cast<const uint32_t *>(p));
    }
    static __device__ __forceinline__ void tabu(const uint32_t *p, uint32_t *t) {
        const u32x4 a = gload4(p);
        t[0] = a.x;
        t[1] = a.y;
        t[2] = a.z;
        t[3] = a.w;
    }
};

template <>
struct Chunk<8> {
    static __device__ __forceinline__ uint64_t colours(const uint8_t *p) {
        return *gptr(reinterpret_cast<const uint64_t *>(p));
    }
    static __device__ __forceinline__ void tabu(const uint32_t *p, uint32_t *t) {
        const u32x4 a = gload4(p);
        const u32x4 b = gload4(p + 4);
        t[0] = a.x;
        t[1] = a.y;
        t[2] = a.z;
        t[3] = a.w;
        t[4] = b.x;
        t[5] = b.y;
        t[6] = b.z;
        t[7] = b.w;
    }
};

// PH 1, 2: the two phases of Section 3.3.  PH 3: PartialCol (Section 3.7),
// the search of Partial-MPMA over legal partial colourings: the eligible
// vertices are the uncoloured ones (a legal colouring has no conflicts), a
// move colours one of them and uncolours its neighbours holding the colour,
// which then may not take it back for T iterations.
template <int CH, int PH>
__device__ void run_phase(const PlitsArgs &a, int64_t iters, uint32_t slot,
                          uint32_t gen, const uint8_t *src, uint8_t *out, uint32_t *tabu,
                          const WaveState &ws, Scal &sc, Cnt &ucnt, uint32_t &lane_cands) {
    const DevInstance I = a.I;  // by value: the pointers the search uses stay in registers
    const int lane = lane_id();
    const int n = I.n, nv = I.nv, np1 = n + 1, TS = I.ts;
    // F = phi_den f + phi_num c: phase 1 phi = 1/2, phase 2 phi = |V|;
    // PartialCol: F = f (c stays 0)
    const int32_t phi_num = (PH == 1 || PH == 3) ? 1 : nv;
    const int32_t phi_den = (PH == 1) ? 2 : 1;
    const uint32_t tag = PH == 1 ? TAG_PLITS1 : (PH == 2 ? TAG_PLITS2 : TAG_PARTIAL);
    // Move values on a 16-bit scale e ordered like delta: e = delta when the
    // phase's values fit (phase 1, and phase 2 with |V| <= 64); otherwise
    // e = 4 dc + df, which orders moves as |V| dc + df does since |df| <= 1
    // and |V| >= 3.  Keys carry e + 2^15.
    const bool squeeze = (PH == 2 && nv > 64);
    const int32_t eA = (PH != 2) ? 1 : (squeeze ? 4 : nv);  // per unit of dc
    const int32_t eB = (PH == 1) ? 2 : 1;                   // per unit of df
    const uint32_t alpha_n = (uint32_t)a.P.alpha_num, alpha_d = (uint32_t)a.P.alpha_den;
    const uint32_t m_alpha = 0xFFFFFFFFu / alpha_d;
    uint8_t *rowH = ws.H;
    uint8_t *colH = ws.H + n * np1;

    setup_state(I, src, ws, sc);
    if (src != out) snapshot(I, ws.S, out);
    sc.F = (int64_t)phi_den * sc.f + (int64_t)phi_num * sc.c;
    sc.Fbest = sc.F;
    sc.fbest = sc.f;
    sc.cbest = sc.c;
    const int W = (nv + 31) >> 5;
    uint32_t wx = 0u, wy = 0u, wz = 0u;  // random words of iterations (it & ~63) + lane
    // The tabu entry of a move is written at the start of the next
    // iteration's candidate loads (lane 0 holds it; the others hold ~0): its
    // completion then overlaps those loads instead of stalling the move.
    uint32_t pend_off = 0xFFFFFFFFu, pend_val = 0u;
    // likewise the expiry mark of the moved vertex, raised at the start of
    // the next iteration (under the eligibility scan)
    uint32_t pend_tv = 0xFFFFFFFFu, pend_tu = 0u;
    uint32_t tbase = 0u;  // base of the relative expiry marks
    // lane roles of the count updates (all ones / all zeros)
    const uint32_t ln_new = lane >= 2 ? 0xFFFFFFFFu : 0u;  // entering colour
    const uint32_t ln_odd = (lane & 1) ? 0xFFFFFFFFu : 0u;  // column count
    PLSE_WAVE_SYNC();

    for (int64_t it = 0; it < iters; ++it) {
        const uint32_t itu = (uint32_t)it;
        if ((itu & 63u) == 0u) {
            const U4 rw = draw(a.seed_lo, a.seed_hi, slot, gen, tag, itu + (uint32_t)lane);
            wx = rw.x;
            wy = rw.y;
            wz = rw.z;
        }
        if ((itu & 127u) == 0u && itu != 0u) {
            // advance the base: marks drop by 128 (expired ones to 1), 255 stays
            tbase += 128u;
            PLSE_WAVE_SYNC();
            for (int q = lane; q < (nv + 3) >> 2; q += 64) {
                const uint32_t x = reinterpret_cast<uint32_t *>(ws.tm8)[q];
                uint32_t y = 0u;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const uint32_t b = (x >> (8 * t)) & 0xFFu;
                    y |= (b == 255u ? 255u : (b > 128u ? b - 128u : (b != 0u ? 1u : 0u))) << (8 * t);
                }
                reinterpret_cast<uint32_t *>(ws.tm8)[q] = y;
            }
            PLSE_WAVE_SYNC();
        }
        if (lane == 0 && pend_tv != 0xFFFFFFFFu) {
            const uint32_t rel = pend_tu - tbase;  // >= 0
            const uint32_t mark = rel > 253u ? 255u : rel + 1u;
            if (mark > ws.tm8[pend_tv]) ws.tm8[pend_tv] = (uint8_t)mark;
        }
        const uint32_t w0 = readlane_u32(wx, (int)(itu & 63u));
        const uint32_t w1 = readlane_u32(wy, (int)(itu & 63u));
        const uint32_t w2 = readlane_u32(wz, (int)(itu & 63u));
        // colour halves of the tie values (written first: independent of the
        // eligibility scan, which covers their latency)
        if (lane <= n) ws.hk[lane] = (uint16_t)(fmix32(w2 ^ (uint32_t)lane) >> 16);
        if (lane + 64 <= n) ws.hk[lane + 64] = (uint16_t)(fmix32(w2 ^ (uint32_t)(lane + 64)) >> 16);
        // 1. eligible vertices (ascending rank over the bitmap): their number
        //    m, and the first kPlitsStage of them staged for dealing
        uint32_t m = 0;
        for (int wb = 0; wb < W; wb += 64) {
            const int w = wb + lane;
            uint32_t bits = (w < W) ? ws.bm[w] : 0u;
            uint32_t total;
            uint32_t pos = m + wave_excl_scan_dpp((uint32_t)__popc(bits), &total);
#pragma unroll 1
            while (bits && pos < (uint32_t)kPlitsStage) {
                const int b = __ffs(bits) - 1;
                bits &= bits - 1u;
                ws.stage[pos++] = (uint16_t)(w * 32 + b);
            }
            m += total;
        }
        if (m == 0) break;  // F = 0: complete legal colouring
        PLSE_WAVE_SYNC();
        ucnt.iters++;
        ucnt.elig += m;

        // 2. best admissible one-move per lane over the chunk rounds.
        //    Aspiration F + delta < F* is e + 2^15 < teb.
        int32_t te;
        if (!squeeze) {
            const int64_t gap = sc.Fbest - sc.F;  // <= 0
            te = gap < -(1ll << 30) ? -(1 << 30) : (int32_t)gap;
        } else {
            te = squeezed_bound(sc.fbest - sc.f, sc.cbest - sc.c, nv);
        }
        const int32_t teb = te + 0x8000;
        // per lane: upper key word of its best move (value, tie value), the
        // move's vertex and colour, and the vertex's payload.  A lane meets
        // its moves in ascending id order, so keeping the first of equal
        // upper words keeps the smallest id among them.
        uint32_t lhi = 0xFFFFFFFFu, lv = 0u, lk = 0u, lpay = 0u;
        if (pend_off != 0xFFFFFFFFu) gptr(tabu)[pend_off] = pend_val;
        uint32_t head = 0u, tail = 0u, g = 0u;
        uint32_t sbase = 0u;  // rank of stage[0]
        for (;;) {
            // once the ring is empty, deal the rows of the next 64 eligible
            // vertices into it
            if (head == tail && g < m) {
                head = tail = 0u;
                if (g >= sbase + (uint32_t)kPlitsStage) {
                    // stage eligible vertices of rank g .. g+kPlitsStage-1
                    // (the bitmap does not change within the iteration)
                    PLSE_WAVE_SYNC();
                    sbase = g;
                    const uint32_t gend = g + (uint32_t)kPlitsStage;
                    uint32_t base = 0;
                    for (int wb = 0; wb < W && base < gend; wb += 64) {
                        const int w = wb + lane;
                        uint32_t bits = (w < W) ? ws.bm[w] : 0u;
                        uint32_t total;
                        uint32_t pos = base + wave_excl_scan_dpp((uint32_t)__popc(bits), &total);
#pragma unroll 1
                        while (bits && pos < gend) {
                            const int b = __ffs(bits) - 1;
                            bits &= bits - 1u;
                            if (pos >= g) ws.stage[pos - g] = (uint16_t)(w * 32 + b);
                            ++pos;
                        }
                        base += total;
                    }
                    PLSE_WAVE_SYNC();
                }
                const uint32_t e = g + (uint32_t)lane;
                uint32_t v = 0u, nch = 0u, ent = 0u;
                if (e < m) {
                    v = ws.stage[e - sbase];
                    // chunk count and liveness of v, read together: planes 0
                    // and 1 (or 0 twice), further planes only when present
                    const int vw = (int)(v >> 5);
                    const bool p0ok = ws.nplanes > 0, p1ok = ws.nplanes > 1;
                    const uint32_t q0 = p0ok ? ws.planes[vw] : 0u;
                    const uint32_t q1 = p1ok ? ws.planes[W + vw] : 0u;
                    const uint32_t tm = ws.tm8[v];
                    uint32_t code = ((q0 >> (v & 31u)) & 1u) | (((q1 >> (v & 31u)) & 1u) << 1);
                    if (ws.nplanes > 2) {
#pragma unroll
                        for (int b = 2; b < 6; ++b)
                            if (b < ws.nplanes)
                                code |= ((ws.planes[b * W + vw] >> (v & 31u)) & 1u) << b;
                    }
                    nch = code + 1u;  // ceil((d + 1) / CH)
                    // a vertex not live has no tabu move this iteration
                    const bool live = tm == 255u || tm > itu - tbase + 1u;
                    ent = v | ((uint32_t)live << 31);
                }
                uint32_t total;
                const uint32_t at = tail + wave_excl_scan_dpp(nch, &total);
#pragma unroll 1
                for (uint32_t t = 0; t < nch; ++t) ws.ring[at + t] = ent | (t << 16);
                tail += total;
                g += 64u;
                PLSE_WAVE_SYNC();
            }
            if (head == tail) break;
            const uint32_t x = head + (uint32_t)lane;
            head = min(head + 64u, tail);
            if (x < tail) {
                // ring entry: vertex | chunk index << 16 | live << 31
                const uint32_t ent = ws.ring[x];
                const int v = (int)(ent & 0xFFFFu);
                const int p0 = (int)((ent >> 16) & 0x7FFFu) * CH;
                const bool live = (ent >> 31) != 0u;
                const int s = ws.S[v];
                const uint32_t vi = gptr(I.vinfo)[v];
                const auto cw = Chunk<CH>::colours(I.cand + (size_t)v * TS + p0);
                uint32_t tv[CH];
#pragma unroll
                for (int t = 0; t < CH; ++t) tv[t] = 0u;
                if (live) Chunk<CH>::tabu(tabu + (size_t)v * TS + p0, tv);
                const int r = (int)(vi & 0xFFu), c = (int)((vi >> 8) & 0xFFu);
                if (p0 == 0) lane_cands += (vi >> 16) & 0xFFu;
                const uint8_t *rH = rowH + r * np1;
                const uint8_t *cH = colH + c * np1;
                const int32_t cur = s ? ((int32_t)rH[s] + (int32_t)cH[s] - 2) : 0;
                // e = eB df + eA (conf(v,k) - cur), df = -1 when v was
                // uncoloured, +1 for the uncolour move (k = 0, position 0)
                const int32_t base = 0x8000 + (s ? 0 : -eB) - eA * cur;
                const uint32_t hv = fmix32(w1 ^ (uint32_t)v) >> 16;
                // winner payload: row, column, current colour, degree
                const uint32_t vpay =
                    (uint32_t)r | ((uint32_t)c << 8) | ((uint32_t)s << 16) | (vi & 0xFF000000u);
                // all LDS reads of the chunk issued together
                int kk[CH], cnt[CH];
                uint32_t hkv[CH];
#pragma unroll
                for (int t = 0; t < CH; ++t) kk[t] = (int)((cw >> (8 * t)) & 0xFFu);
#pragma unroll
                for (int t = 0; t < CH; ++t) cnt[t] = (int)rH[kk[t]] + (int)cH[kk[t]];
#pragma unroll
                for (int t = 0; t < CH; ++t) hkv[t] = ws.hk[kk[t]];
                bool took = false;
#pragma unroll
                for (int t = 0; t < CH; ++t) {
                    const int k = kk[t];
                    const int32_t b = (t == 0 && p0 == 0) ? base + eB : base;
                    const int32_t eb = eA * cnt[t] + b;
                    // positions past the domain repeat its last colour and
                    // that colour's tabu entry: they never beat the original,
                    // which this lane met first
                    const bool ok = (k != s) && (itu >= tv[t] || eb < teb);
                    const uint32_t hi = ((uint32_t)eb << 16) | (hv ^ hkv[t]);
                    const bool take = ok && hi < lhi;
                    lhi = take ? hi : lhi;
                    lk = take ? (uint32_t)k : lk;
                    took = took || take;
                }
                lv = took ? (uint32_t)v : lv;
                lpay = took ? vpay : lpay;
            }
            PLSE_WAVE_SYNC();
        }
        // 3. unique best over the wave: minimum of the upper key words, then
        //    of the move ids among the lanes holding it
        const uint32_t ghi = wave_min_u32_dpp(lhi);
        if (ghi == 0xFFFFFFFFu) {
            ucnt.idle++;
            continue;
        }
        // the move id of the lane holding the minimum (a second minimum over
        // move ids only when several lanes share the upper word)
        uint64_t who = ballot(lhi == ghi);
        if (__popcll(who) != 1) {
            const uint32_t lcid = lv * (uint32_t)np1 + lk;
            const uint32_t glo = wave_min_u32_dpp(lhi == ghi ? lcid : 0xFFFFFFFFu);
            who = ballot(lhi == ghi && lcid == glo);
        }
        const int wl = (int)__ffsll((unsigned long long)who) - 1;
        const uint32_t pay = readlane_u32(lpay, wl);
        const int v = (int)readlane_u32(lv, wl);
        const int k = (int)readlane_u32(lk, wl);
        const int r = (int)(pay & 0xFFu);
        const int c = (int)((pay >> 8) & 0xFFu);
        const int old = (int)((pay >> 16) & 0xFFu);
        const int deg = (int)(pay >> 24);
        // the counts of the two colours in v's row and column, then the memory
        // the apply needs, fetched together: v's first 64 neighbours and its
        // domain mask (the tabu position of the colour it leaves)
        uint8_t *rH = rowH + r * np1;
        uint8_t *cH = colH + c * np1;
        const int32_t hk_r = rH[k], hk_c = cH[k], ho_r = rH[old], ho_c = cH[old];
        const uint32_t *nb = I.nbr + (size_t)v * I.nl;
        const uint32_t ent0 = lane < deg ? gptr(nb)[lane] : 0u;
        u32x4 dmask{0u, 0u, 0u, 0u};
        if constexpr (PH != 3) dmask = gload4(reinterpret_cast<const u32x4 *>(I.vrec) + 2 * v);
        const int32_t cvk = k ? hk_r + hk_c : 0;
        const int32_t cvo = old ? ho_r + ho_c - 2 : 0;
        const bool vC = (k != 0) && (cvk > 0);
        PLSE_WAVE_SYNC();
        if constexpr (PH == 3) {
            // PartialCol: v (uncoloured) takes k; its cvk neighbours holding k
            // (at most one per row and column) are uncoloured and may not take
            // k back before `until`
            if (lane < 4) {
                const uint32_t col = (ln_new & (uint32_t)k) | (~ln_new & (uint32_t)old);
                const uint32_t hb = ((ln_odd & (uint32_t)(cH - ws.H)) |
                                     (~ln_odd & (uint32_t)(rH - ws.H))) + col;
                const uint32_t add = col != 0u ? ((ln_new & 2u) - 1u) << ((hb & 3u) * 8u) : 0u;
                atomicAdd(reinterpret_cast<uint32_t *>(ws.H) + (hb >> 2), add);
            }
            if (lane == 0) {
                ws.S[v] = (uint8_t)k;
                atomicAdd(&ws.bm[v >> 5], 0u - (1u << (v & 31)));
            }
            sc.f += cvk - 1;
            sc.F = sc.f;
            ucnt.cupd += 2u + 2u * (uint32_t)cvk;
            const uint32_t mp = (uint32_t)sc.f;
            const uint32_t T = scale32(w0, 10u) + udiv_by(alpha_n * mp, alpha_d, m_alpha);
            const uint32_t until = itu + 1u + T;
            PLSE_WAVE_SYNC();
            // conflict-table entries: v's neighbours, then each uncoloured
            // vertex's neighbours
            uint32_t nupd_l = 0u;
            for (int t0 = 0; t0 < deg; t0 += 64) {
                const int t = t0 + lane;
                const uint32_t ent = t0 == 0 ? ent0 : (t < deg ? gptr(nb)[t] : 0u);
                const int u = (int)(ent & 0xFFFFu), other = (int)((ent >> 16) & 0x7FFFu);
                if (t < deg && ws.S[u] == k) {
                    nupd_l += gptr(I.vinfo)[u] >> 24;
                    const bool inrow = (ent >> 31) == 0;
                    const int ur = inrow ? r : other, uc = inrow ? other : c;
                    const int rb = ur * np1 + k, cb = n * np1 + uc * np1 + k;
                    uint32_t *H32 = reinterpret_cast<uint32_t *>(ws.H);
                    ws.S[u] = 0;
                    atomicAdd(H32 + (rb >> 2), 0u - (1u << ((rb & 3) * 8)));
                    atomicAdd(H32 + (cb >> 2), 0u - (1u << ((cb & 3) * 8)));
                    atomicOr(&ws.bm[u >> 5], 1u << (u & 31));
                    // tabu entry (u, k), repeated over the rest of the chunk
                    // when k is u's last domain colour
                    const u32x4 dm = gload4(reinterpret_cast<const u32x4 *>(I.vrec) + 2 * u);
                    const uint32_t po = position_in(dm, k);
                    const uint32_t du = (uint32_t)(__popcll(((uint64_t)dm.y << 32) | dm.x) +
                                                   __popcll(((uint64_t)dm.w << 32) | dm.z));
                    const uint32_t nrep = po == du ? (uint32_t)CH - du % (uint32_t)CH : 1u;
                    for (uint32_t q = 0; q < nrep; ++q)
                        gptr(tabu)[(size_t)u * TS + po + q] = until;
                    const uint32_t rel = until - tbase;
                    const uint32_t mark = rel > 253u ? 255u : rel + 1u;
                    if (mark > ws.tm8[u]) ws.tm8[u] = (uint8_t)mark;
                }
            }
            ucnt.nupd += (uint64_t)deg + wave_sum_u32_dpp(nupd_l);
        } else {
            // 4. apply.  Counts: lanes 0-1 the leaving colour's row and column
            //    count (-1), lanes 2-3 the entering colour's (+1), as LDS adds on
            //    the bytes of u32 words (exact: counts stay within 0..n, nothing
            //    carries), an add of 0 for colour 0.  Lane 0: v's colour, and v's
            //    eligibility bit cleared (an exact add: v was eligible) unless v
            //    stays in V_0 u C.  Lane roles are bit masks, not branches.
            if (lane < 4) {
                const uint32_t col = (ln_new & (uint32_t)k) | (~ln_new & (uint32_t)old);
                const uint32_t hb = ((ln_odd & (uint32_t)(cH - ws.H)) |
                                     (~ln_odd & (uint32_t)(rH - ws.H))) + col;
                const uint32_t add = col != 0u ? ((ln_new & 2u) - 1u) << ((hb & 3u) * 8u) : 0u;
                atomicAdd(reinterpret_cast<uint32_t *>(ws.H) + (hb >> 2), add);
            }
            if (lane == 0) {
                ws.S[v] = (uint8_t)k;
                atomicAdd(&ws.bm[v >> 5], (k == 0 || vC) ? 0u : 0u - (1u << (v & 31)));
            }
            PLSE_WAVE_SYNC();
            // eligibility of the row/column vertices holding the old or new colour:
            // all reads unconditional, one toggle where it changes
            int32_t dC = 0;
            for (int t0 = 0; t0 < deg; t0 += 64) {
                const int t = t0 + lane;
                const uint32_t ent = t0 == 0 ? ent0 : (t < deg ? gptr(nb)[t] : 0u);
                const bool inrow = (ent >> 31) == 0;
                const int u = (int)(ent & 0xFFFFu), other = (int)((ent >> 16) & 0x7FFFu);
                const int su = ws.S[u];
                const uint32_t bw = ws.bm[u >> 5];
                const int rrow = inrow ? r : other, rcol = inrow ? other : c;
                const int cu = (int)rowH[rrow * np1 + su] + (int)colH[rcol * np1 + su] - 2;
                const bool hit = t < deg && su != 0 && (su == old || su == k);
                const bool was = (bw >> (u & 31)) & 1u;
                const bool now = cu > 0;
                const bool flip = hit && (now != was);
                if (flip) atomicXor(&ws.bm[u >> 5], 1u << (u & 31));
                dC += (int32_t)__popcll(ballot(flip && now)) - (int32_t)__popcll(ballot(flip && !now));
            }
            const int32_t df = (k == 0 ? 1 : 0) - (old == 0 ? 1 : 0);
            sc.nC += dC + (vC ? 1 : 0) - (old ? 1 : 0);
            sc.f += df;
            sc.c += cvk - cvo;
            sc.F += (int64_t)phi_den * df + (int64_t)phi_num * (cvk - cvo);
            const uint32_t ends = (uint32_t)(old != 0) + (uint32_t)(k != 0);
            ucnt.cupd += 2u * ends;
            ucnt.nupd += (uint32_t)deg * ends;
            // tenure T = L + alpha (|V_0| + |C|) after the move; moving v back to
            // `old` is tabu for T iterations
            const uint32_t mp = (uint32_t)(sc.f + sc.nC);
            const uint32_t T = scale32(w0, 10u) + udiv_by(alpha_n * mp, alpha_d, m_alpha);
            const uint32_t until = itu + 1u + T;
            pend_tv = (uint32_t)v;
            pend_tu = until;
            {
                // the entry of the last domain colour is repeated over the rest
                // of its chunk, where the candidate row repeats that colour
                const uint32_t po = position_in(dmask, old);
                const uint32_t dv = (uint32_t)(__popcll(((uint64_t)dmask.y << 32) | dmask.x) +
                                               __popcll(((uint64_t)dmask.w << 32) | dmask.z));
                const uint32_t nrep = po == dv ? (uint32_t)CH - dv % (uint32_t)CH : 1u;
                pend_off = (uint32_t)lane < nrep ? (uint32_t)v * (uint32_t)TS + po + (uint32_t)lane
                                                 : 0xFFFFFFFFu;
                pend_val = until;
            }
        }
        PLSE_WAVE_SYNC();
        if (sc.F < sc.Fbest) {
            sc.Fbest = sc.F;
            sc.fbest = sc.f;
            sc.cbest = sc.c;
            snapshot(I, ws.S, out);
            ucnt.snaps++;
        }
    }
    // the last move's tabu entry and mark: the mark tells clear_tabu the row
    // was written
    if (pend_off != 0xFFFFFFFFu) gptr(tabu)[pend_off] = pend_val;
    if (lane == 0 && pend_tv != 0xFFFFFFFFu && ws.tm8[pend_tv] == 0) ws.tm8[pend_tv] = 1;
    PLSE_WAVE_SYNC();
    clear_tabu(I, tabu, ws);
    PLSE_WAVE_SYNC();
}

// Greedy conflict removal (Section 3.7): uncolour the vertex with the most
// conflicts (ties: lowest id) until the colouring is legal; `from` -> `out`.
__device__ void repair(const PlitsArgs &a, const uint8_t *from, uint8_t *out, const WaveState &ws,
                       Scal &sc, Cnt &ucnt) {
    const DevInstance &I = a.I;
    const int lane = lane_id();
    const int n = I.n, nv = I.nv, np1 = n + 1;
    setup_state(I, from, ws, sc);
    uint8_t *rowH = ws.H, *colH = ws.H + n * np1;
    for (;;) {
        uint32_t lkey = 0u;
        for (int v = lane; v < nv; v += 64) {
            const int s = ws.S[v];
            if (s) {
                const uint32_t rc = gptr(I.vrc)[v];
                const int own =
                    (int)rowH[(rc & 0xFFu) * np1 + s] + (int)colH[(rc >> 8) * np1 + s] - 2;
                if (own > 0) {
                    const uint32_t key = ((uint32_t)own << 16) | (0xFFFFu - (uint32_t)v);
                    lkey = key > lkey ? key : lkey;
                }
            }
        }
        const uint32_t g = wave_max_u32(lkey);
        if (g == 0u) break;
        const int v = (int)(0xFFFFu - (g & 0xFFFFu));
        if (lane == 0) {
            const uint32_t rc = gptr(I.vrc)[v];
            const int old = ws.S[v];
            rowH[(rc & 0xFFu) * np1 + old] -= 1;
            colH[(rc >> 8) * np1 + old] -= 1;
            ws.S[v] = 0;
        }
        ucnt.repairs++;
        PLSE_WAVE_SYNC();
    }
    snapshot(I, ws.S, out);
    PLSE_WAVE_SYNC();
}

// The search of individual `ind` of one instance in generation `gen`, by one
// wave whose LDS starts at `base`.
template <int CH, bool PARTIAL>
__device__ __forceinline__ void plits_individual(const PlitsArgs &a, int ind, int gen, uint8_t *base) {
    WaveState ws;
    ws.S = base;
    ws.H = base + a.off_h;
    ws.bm = reinterpret_cast<uint32_t *>(base + a.off_bm);
    ws.tm8 = base + a.off_tm;
    ws.stage = reinterpret_cast<uint16_t *>(base + a.off_el);
    ws.ring = reinterpret_cast<uint32_t *>(base + a.off_ring);
    ws.hk = reinterpret_cast<uint16_t *>(base + a.off_hk);
    ws.planes = reinterpret_cast<uint32_t *>(base + a.off_planes);
    ws.nplanes = a.nplanes;
    {
        // chunk-count planes: bit b of floor(|D*(v)| / CH) per vertex
        const int W = (a.I.nv + 31) >> 5;
        for (int w = lane_id(); w < W; w += 64) {
            uint32_t pl[6] = {0u, 0u, 0u, 0u, 0u, 0u};
            const int vend = min(a.I.nv, (w + 1) * 32);
            for (int v = w * 32; v < vend; ++v) {
                const uint32_t code = ((gptr(a.I.vinfo)[v] >> 16) & 0xFFu) / CH;
#pragma unroll
                for (int b = 0; b < 6; ++b) pl[b] |= ((code >> b) & 1u) << (v & 31);
            }
            for (int b = 0; b < a.nplanes; ++b) ws.planes[b * W + w] = pl[b];
        }
    }
    const DevInstance &I = a.I;
    uint32_t *tabu = a.tabu + (size_t)ind * I.nv * I.ts;
    const uint8_t *src = a.S_in + (size_t)ind * I.stride;
    uint8_t *out = a.S_out + (size_t)ind * I.stride;

    Cnt ucnt{0u, 0u, 0u, 0u, 0ull, 0ull, 0ull};
    uint32_t lane_cands = 0;
    Scal sc;
    const uint32_t slot = (uint32_t)readfirst(ind);
    int32_t f_final;
    if constexpr (PARTIAL) {
        // Partial-MPMA (Section 3.7): the offspring repaired into a legal
        // partial colouring, then PartialCol for the whole depth
        repair(a, src, out, ws, sc, ucnt);
        run_phase<CH, 3>(a, a.P.depth1 + a.P.depth2, slot, (uint32_t)gen, out, out, tabu, ws,
                         sc, ucnt, lane_cands);
        f_final = sc.fbest;
    } else {
        // phase 1 from the offspring, phase 2 from phase 1's best (both write
        // their best into `out`)
        run_phase<CH, 1>(a, a.P.depth1, slot, (uint32_t)gen, src, out, tabu, ws, sc, ucnt,
                         lane_cands);
        run_phase<CH, 2>(a, a.P.depth2, slot, (uint32_t)gen, out, out, tabu, ws, sc, ucnt,
                         lane_cands);
        f_final = sc.fbest;
        if (sc.cbest > 0) {
            repair(a, out, out, ws, sc, ucnt);
            f_final = sc.f + (int32_t)ucnt.repairs;
        }
    }
    const uint64_t cands = wave_sum_u64(lane_cands);
    const int lane = lane_id();
    if (lane < kCounters) {
        uint64_t v = 0;
        switch (lane) {
            case C_ITERS: v = ucnt.iters; break;
            case C_MOVES: v = ucnt.iters - ucnt.idle; break;
            case C_IDLE: v = ucnt.idle; break;
            case C_CANDS: v = cands; break;
            case C_ELIG: v = ucnt.elig; break;
            case C_NUPD: v = ucnt.nupd; break;
            case C_SNAPS: v = ucnt.snaps; break;
            case C_REPAIRS: v = ucnt.repairs; break;
            default: v = ucnt.cupd; break;
        }
        gptr(a.cnt_out)[(size_t)ind * kCounters + lane] = v;
    }
    if (lane == 0) gptr(a.f_out)[ind] = f_final;
}

}  // namespace

template <int CH, bool PARTIAL>
__global__ __launch_bounds__(256, 4) void plits_kernel(const ArgList L) {
    extern __shared__ __align__(16) uint8_t lds[];
    // by reference: fields needed only before or after a phase are read when
    // needed instead of being held in registers through the search
    const PlitsArgs &a = *static_cast<const PlitsArgs *>(L.p[blockIdx.y]);
    const int wv = (int)(threadIdx.x >> 6);
    const int ind = (int)blockIdx.x * (int)(blockDim.x >> 6) + wv;
    if (ind >= a.p) return;
    int gen = a.gen_fixed;
    if (gen == 0) {
        if (gptr(a.ctl)->stop) return;
        gen = gptr(a.ctl)->gen;
    }
    plits_individual<CH, PARTIAL>(a, ind, gen, lds + (size_t)wv * a.lds_per_wave);
}

// Persistent form for many instances: every wave takes (instance,
// individual) items from a queue until it runs dry.  Items run instance by
// instance in the order of the argument list (longest estimated work first),
// individuals in order within an instance; stopped instances are skipped.
// Every wave of the launch uses `lds_per_wave` bytes (the largest instance's).
template <int CH, bool PARTIAL>
__global__ __launch_bounds__(256, 4) void plits_persistent_kernel(const ArgList L, int count, int p,
                                                                  int lds_per_wave,
                                                                  uint32_t *queue) {
    extern __shared__ __align__(16) uint8_t lds[];
    uint8_t *base = lds + (size_t)(threadIdx.x >> 6) * lds_per_wave;
    const uint32_t total = (uint32_t)count * (uint32_t)p;
    for (;;) {
        uint32_t item = 0u;
        if (lane_id() == 0) item = atomicAdd(queue, 1u);
        item = readlane_u32(item, 0);
        if (item >= total) break;
        const uint32_t inst = item / (uint32_t)p, ind = item - inst * (uint32_t)p;
        const PlitsArgs &a = *static_cast<const PlitsArgs *>(L.p[inst]);
        int gen = a.gen_fixed;
        if (gen == 0) {
            if (gptr(a.ctl)->stop) continue;
            gen = gptr(a.ctl)->gen;
        }
        plits_individual<CH, PARTIAL>(a, (int)ind, gen, base);
        PLSE_WAVE_SYNC();
    }
}

__global__ void queue_reset_kernel(uint32_t *queue) {
    if (threadIdx.x == 0) *gptr(queue) = 0u;
}

// The PLITS kernel of a chunk size, MPMA or Partial-MPMA; null for other sizes.
const void *plits_fn(int slots_per_lane, bool partial) {
    switch (slots_per_lane) {
        case 2: return partial ? (const void *)plits_kernel<2, true> : (const void *)plits_kernel<2, false>;
        case 4: return partial ? (const void *)plits_kernel<4, true> : (const void *)plits_kernel<4, false>;
        case 8: return partial ? (const void *)plits_kernel<8, true> : (const void *)plits_kernel<8, false>;
        default: return nullptr;
    }
}

// Zero a tabu region (a fresh workspace, before the first phase uses it).
__global__ void fill_zero_kernel(const ArgList L) {
    const FillArgs a = arg_of<FillArgs>(L);
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t nq = a.n / 4;
    for (size_t i = t; i < nq; i += (size_t)gridDim.x * blockDim.x)
        gstore4(reinterpret_cast<u32x4 *>(a.p) + i, u32x4{0u, 0u, 0u, 0u});
    for (size_t i = nq * 4 + t; i < a.n; i += (size_t)gridDim.x * blockDim.x) gptr(a.p)[i] = 0u;
}

hipError_t launch_plits(const ArgList &L, int count, int p, int lds_per_wave,
                        int slots_per_lane, int waves_per_block, bool partial, bool lean,
                        hipStream_t stream) {
    const int blocks = (p + waves_per_block - 1) / waves_per_block;
    const size_t lds = (size_t)lds_per_wave * waves_per_block;
    const dim3 grid(blocks, count), block(64 * waves_per_block);
    const void *fn = lean ? plits_lean_fn(slots_per_lane) : plits_fn(slots_per_lane, partial);
    if (!fn) return hipErrorInvalidValue;
    void *args[] = {const_cast<ArgList *>(&L)};
    return hipLaunchKernel(fn, grid, block, args, lds, stream);
}

const void *plits_persistent_fn(int slots_per_lane, bool partial) {
    switch (slots_per_lane) {
        case 2: return partial ? (const void *)plits_persistent_kernel<2, true>
                               : (const void *)plits_persistent_kernel<2, false>;
        case 4: return partial ? (const void *)plits_persistent_kernel<4, true>
                               : (const void *)plits_persistent_kernel<4, false>;
        case 8: return partial ? (const void *)plits_persistent_kernel<8, true>
                               : (const void *)plits_persistent_kernel<8, false>;
        default: return nullptr;
    }
}

hipError_t launch_plits_persistent(const ArgList &L, int count, int p, int lds_per_wave,
                                   int slots_per_lane, int waves_per_block, bool partial,
                                   int blocks, uint32_t *queue, hipStream_t stream) {
    const void *fn = plits_persistent_fn(slots_per_lane, partial);
    if (!fn || blocks < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, stream, queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)lds_per_wave * waves_per_block;
    ArgList Lc = L;
    void *args[] = {&Lc, &count, &p, &lds_per_wave, &queue};
    return hipLaunchKernel(fn, dim3(blocks), dim3(64 * waves_per_block), args, lds, stream);
}

hipError_t launch_fill_zero(const ArgList &L, int count, hipStream_t stream) {
    hipLaunchKernelGGL(fill_zero_kernel, dim3(1024, count), dim3(256), 0, stream, L);
    return hipGetLastError();
}

// Resident waves per CU of a PLITS launch shape (the runtime's occupancy
// calculation: registers, LDS and workgroup limits).
int plits_waves_per_cu(int slots_per_lane, int waves_per_block, int lds_per_wave, bool partial,
                       bool lean, bool persistent) {
    const void *fn = lean ? plits_lean_fn(slots_per_lane)
                          : (persistent ? plits_persistent_fn(slots_per_lane, partial)
                                        : plits_fn(slots_per_lane, partial));
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, 64 * waves_per_block,
                                                     (size_t)lds_per_wave * waves_per_block) !=
        hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return blocks * waves_per_block;
}

hipError_t plits_set_lds_limit(int bytes) {
    hipError_t e = hipSuccess;
    for (int spl : {2, 4, 8}) {
        for (bool partial : {false, true})
            if (e == hipSuccess) e = set_dynamic_lds_limit(plits_fn(spl, partial), bytes);
        if (e == hipSuccess) e = set_dynamic_lds_limit(plits_lean_fn(spl), bytes);
        for (bool partial : {false, true})
            if (e == hipSuccess) e = set_dynamic_lds_limit(plits_persistent_fn(spl, partial), bytes);
    }
    return e;
}

}  // namespace plse

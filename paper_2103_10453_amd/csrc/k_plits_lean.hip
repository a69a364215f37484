// k_plits_lean.hip -- PLITS (Section 3.3, Alg. 3) with the whole search state
// of an individual in LDS, for instances whose tabu marks fit there
// (gfx950, one wave64 per individual).
//
// A tabu-search iteration is a chain of short dependent steps (find the
// eligible vertices, evaluate their moves, take the wave minimum, apply), so
// a lone search is bound by how many instructions and memory round trips
// each step issues, not by bandwidth.  This kernel keeps every per-iteration
// access in LDS or in the small read-only instance tables (L1-resident), and
// spends no pass on dealing work to lanes:
//
//   * Tabu list: one byte per candidate move (vertex, position in its
//     candidate row) in LDS: the iteration from which the move is allowed,
//     relative to a base advanced by 128 iterations at a time (0: allowed,
//     m in 1..254: allowed from base + m - 1, 255: the exact iteration is in
//     the individual's global tabu area, used only for tenures beyond the
//     byte's range).  Moves of a vertex sit at consecutive positions, its
//     candidate row padded to a multiple of CH, so a lane fetches the marks of
//     CH moves in one LDS read.
//   * Eligible vertices V_0 u C(S) come from the eligibility bitmap, one per
//     lane; each lane derives its vertex's chunk count and offset (where its
//     row of marks starts) from per-word offsets and bit-plane popcounts.
//   * Chunks to lanes: when the iteration's chunks fit the wave (the usual
//     case) lane g takes chunk g; its vertex is the last chunk start at or
//     below g (a ballot over start flags and a bit count), and it pulls that
//     vertex's data across lanes (ds_bpermute).  Otherwise each lane takes
//     whole vertices.  A lane meets its moves in ascending move id, as the
//     tie rule needs.
//   * Apply: the moved vertex's row and column come from the instance's
//     row and column vertex lists (a few KB, shared by every individual).
//
// Conflict counts are kept factored as in the other PLITS kernel: conf[v][k]
// = rowcnt[r(v)][k] + colcnt[c(v)][k] - 2 [S(v) = k] (Section 2.1: the
// neighbours of a cell are the other cells of its row and column).
#include "device_common.h"
#include "kernels.h"

namespace plse {

namespace {

struct LeanState {
    uint8_t *S;        // [stride] colours
    uint8_t *H;        // rowcnt [n][n+1] then colcnt [n][n+1]
    uint32_t *bm;      // [W] eligibility bitmap of V_0 u C(S)
    uint8_t *mk;       // [npos] tabu marks
    uint32_t *dirty;   // [W] vertices with entries in the global tabu area
    uint32_t *planes;  // [nplanes][W] bit b of floor(|D*(v)| / CH)
    uint32_t *wpre;    // [W] chunk offset of each word's first vertex
    u32x2 *stage;      // [kLeanStage] u16 eligible vertices, then 64 chunk-start flags
    uint16_t *hk;      // [n+1] colour halves of the iteration's tie values
    int nplanes;
};

// Per-individual counters of one launch.  The per-iteration sums are held by
// lane 0 of the wave in vector registers (32-bit partial sums, folded into the
// 64-bit totals every 128 iterations), which keeps scalar registers free for
// the search itself.
struct Cnt {
    uint32_t iters, idle, snaps, repairs;
    uint64_t elig, nupd, cupd;
    uint32_t pelig, pnupd, pcupd;  // lane 0: partial sums
};

__device__ __forceinline__ void fold(Cnt &u) {
    u.elig += u.pelig;
    u.nupd += u.pnupd;
    u.cupd += u.pcupd;
    u.pelig = u.pnupd = u.pcupd = 0u;
}

struct Scal {
    int64_t F, Fbest;
    int32_t f, c, nC;
    int32_t fbest, cbest;
};

template <int CH>
struct LeanChunk;

template <>
struct LeanChunk<2> {
    static __device__ __forceinline__ uint64_t colours(const uint8_t *p) {
        return *gptr(reinterpret_cast<const uint16_t *>(p));
    }
    static __device__ __forceinline__ uint64_t marks(const uint8_t *p) {
        return *reinterpret_cast<const uint16_t *>(p);
    }
    static __device__ __forceinline__ bool any_far(uint64_t m) {
        return ((m & 0xFFu) == 0xFFu) || ((m & 0xFF00u) == 0xFF00u);
    }
};

template <>
struct LeanChunk<4> {
    static __device__ __forceinline__ uint64_t colours(const uint8_t *p) {
        return *gptr(reinterpret_cast<const uint32_t *>(p));
    }
    static __device__ __forceinline__ uint64_t marks(const uint8_t *p) {
        return *reinterpret_cast<const uint32_t *>(p);
    }
    static __device__ __forceinline__ bool any_far(uint64_t m) {
        const uint32_t x = (uint32_t)m;
        return (((x & 0x7F7F7F7Fu) + 0x01010101u) & x & 0x80808080u) != 0u;
    }
};

template <>
struct LeanChunk<8> {
    static __device__ __forceinline__ uint64_t colours(const uint8_t *p) {
        return *gptr(reinterpret_cast<const uint64_t *>(p));
    }
    static __device__ __forceinline__ uint64_t marks(const uint8_t *p) {
        return *reinterpret_cast<const uint64_t *>(p);
    }
    static __device__ __forceinline__ bool any_far(uint64_t m) {
        return (((m & 0x7F7F7F7F7F7F7F7Full) + 0x0101010101010101ull) & m &
                0x8080808080808080ull) != 0ull;
    }
};

// Position of colour k in a candidate row with 128-bit domain mask a: 0 for
// k = 0, else 1 + the number of domain colours below k.
__device__ __forceinline__ uint32_t lean_position(const u32x4 a, int k) {
    if (k == 0) return 0u;
    const uint64_t m0 = ((uint64_t)a.y << 32) | a.x;
    const uint64_t m1 = ((uint64_t)a.w << 32) | a.z;
    if (k < 64) return 1u + (uint32_t)__popcll(m0 & ((1ull << k) - 1ull));
    return 1u + (uint32_t)__popcll(m0) + (uint32_t)__popcll(m1 & ((1ull << (k - 64)) - 1ull));
}

// Chunk offset of vertex v (first chunk of its candidate row).
__device__ __forceinline__ uint32_t chunk_offset(const LeanState &ws, int W, int v) {
    const int w = v >> 5, b = v & 31;
    const uint32_t below = (1u << b) - 1u;
    uint32_t o = ws.wpre[w] + (uint32_t)b;
    for (int q = 0; q < ws.nplanes; ++q)
        o += (uint32_t)__popc(ws.planes[q * W + w] & below) << q;
    return o;
}

// S from `src`; row/column colour counts; eligibility bitmap; f, c, |C(S)|;
// tabu marks and the dirty set cleared.
__device__ void lean_setup(const DevInstance &I, const uint8_t *src, const LeanState &ws,
                           int npos, Scal &sc) {
    const int lane = lane_id();
    const int n = I.n, nv = I.nv, np1 = n + 1;
    for (int q = lane; q < (I.stride >> 4); q += 64)
        reinterpret_cast<u32x4 *>(ws.S)[q] = gload4(reinterpret_cast<const u32x4 *>(src) + q);
    const int hbytes = 2 * n * np1;
    uint32_t *h32 = reinterpret_cast<uint32_t *>(ws.H);
    for (int q = lane; q < (hbytes + 3) / 4; q += 64) h32[q] = 0u;
    for (int q = lane; q < (npos + 15) >> 4; q += 64)
        reinterpret_cast<u32x4 *>(ws.mk)[q] = u32x4{0u, 0u, 0u, 0u};
    const int W = (nv + 31) >> 5;
    for (int w = lane; w < W; w += 64) ws.dirty[w] = 0u;
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
    PLSE_WAVE_SYNC();
    sc.f = (int32_t)wave_sum_u32_dpp(f);
    sc.c = (int32_t)(wave_sum_u32_dpp(c2) >> 1);  // each conflicting edge seen twice
    sc.nC = (int32_t)wave_sum_u32_dpp(nC);
}

__device__ __forceinline__ void lean_snapshot(const DevInstance &I, const uint8_t *S,
                                              uint8_t *dst) {
    for (int q = lane_id(); q < (I.stride >> 4); q += 64)
        gstore4(reinterpret_cast<u32x4 *>(dst) + q, reinterpret_cast<const u32x4 *>(S)[q]);
}

// Advance the mark base by 128: marks of moves allowed within the next
// window drop by 128 (already allowed ones to 0); entries kept in the global
// tabu area come back into the byte range once they are near enough.
template <int CH>
__device__ void lean_rebase(const LeanState &ws, int npos, const uint32_t *gfar, uint32_t tbase) {
    const int lane = lane_id();
    for (int q = lane; q < (npos + 15) >> 4; q += 64) {
        u32x4 x = reinterpret_cast<u32x4 *>(ws.mk)[q];
        uint32_t far_any = 0u;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const uint32_t w = x[t];
            const uint32_t hi = w & 0x80808080u;
            const uint32_t lo = w & 0x7F7F7F7Fu;
            const uint32_t ff = (lo + 0x01010101u) & hi;  // bytes equal to 255
            x[t] = (lo & ((hi >> 7) * 0x7Fu)) | ff | ((ff >> 7) * 0x7Fu);
            far_any |= ff;
        }
        if (far_any) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                uint32_t w = x[t];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int pos = q * 16 + t * 4 + b;
                    if (((w >> (8 * b)) & 0xFFu) == 0xFFu && pos < npos) {
                        const uint32_t rel = gptr(gfar)[pos] - tbase;  // > 125
                        if (rel <= 253u) w = (w & ~(0xFFu << (8 * b))) | ((rel + 1u) << (8 * b));
                    }
                }
                x[t] = w;
            }
        }
        reinterpret_cast<u32x4 *>(ws.mk)[q] = x;
    }
}

// Zero the global tabu entries of the vertices marked dirty this phase.
template <int CH>
__device__ void lean_clear_far(const DevInstance &I, const LeanState &ws, uint32_t *gfar) {
    const int W = (I.nv + 31) >> 5;
    for (int w = lane_id(); w < W; w += 64) {
        uint32_t bits = ws.dirty[w];
        while (bits) {
            const int b = __ffs(bits) - 1;
            bits &= bits - 1u;
            const int v = w * 32 + b;
            const uint32_t co = chunk_offset(ws, W, v);
            uint32_t code = 0u;
            for (int q = 0; q < ws.nplanes; ++q)
                code |= ((ws.planes[q * W + w] >> b) & 1u) << q;
            for (uint32_t p = co * CH; p < (co + code + 1u) * CH; ++p) gptr(gfar)[p] = 0u;
        }
    }
}

// Per-vertex data of an eligible vertex v, computed by one lane: chunk
// count and offset, row/column count bases, current colour and conflicts,
// the base of its move values and its half of the tie values.
struct VData {
    int v, s, rb, cb;
    uint32_t nch, co, vpay, hv, d;
    int32_t base;
};

__device__ __forceinline__ VData vertex_data(const DevInstance &I, const LeanState &ws, int W,
                                             int v, uint32_t w1, int32_t eA, int32_t eB) {
    VData x;
    const int n = I.n, np1 = n + 1;
    const int w = v >> 5, b = v & 31;
    const uint32_t below = (1u << b) - 1u;
    const uint32_t vi = gptr(I.vinfo)[v];
    const int s = ws.S[v];
    uint32_t co = ws.wpre[w] + (uint32_t)b, code = 0u;
    for (int q = 0; q < ws.nplanes; ++q) {
        const uint32_t pq = ws.planes[q * W + w];
        co += (uint32_t)__popc(pq & below) << q;
        code |= ((pq >> b) & 1u) << q;
    }
    const int r = (int)(vi & 0xFFu), c = (int)((vi >> 8) & 0xFFu);
    x.v = v;
    x.s = s;
    x.rb = r * np1;
    x.cb = n * np1 + c * np1;
    x.nch = code + 1u;
    x.co = co;
    x.d = (vi >> 16) & 0xFFu;
    x.vpay = (uint32_t)r | ((uint32_t)c << 8) | ((uint32_t)s << 16) | (vi & 0xFF000000u);
    x.hv = fmix32(w1 ^ (uint32_t)v) >> 16;
    const int32_t cur = s ? ((int32_t)ws.H[x.rb + s] + (int32_t)ws.H[x.cb + s] - 2) : 0;
    x.base = 0x8000 + (s ? 0 : -eB) - eA * cur;
    return x;
}

// Best admissible move of chunk j of vertex x into the lane's running best
// (lhi: value and tie value; ties keep the earlier, i.e. smaller, move id).
template <int CH>
__device__ __forceinline__ void eval_chunk(const DevInstance &I, const LeanState &ws,
                                           const uint32_t *gfar, const VData &x, uint32_t j,
                                           uint32_t itu, uint32_t relit, int32_t teb, int32_t eA,
                                           int32_t eB, uint32_t &lhi, uint32_t &lk, bool &took) {
    const int p0 = (int)j * CH;
    const uint64_t cw = LeanChunk<CH>::colours(I.cand + (size_t)x.v * I.ts + p0);
    const uint32_t mpos = (x.co + j) * CH;
    const uint64_t mw = LeanChunk<CH>::marks(ws.mk + mpos);
    // moves allowed by entries kept in the global tabu area
    uint32_t farok = 0u;
    if (LeanChunk<CH>::any_far(mw)) {
#pragma unroll
        for (int t = 0; t < CH; ++t)
            if (((mw >> (8 * t)) & 0xFFu) == 0xFFu && itu >= gptr(gfar)[mpos + t]) farok |= 1u << t;
    }
    int kk[CH], cnt[CH];
    uint32_t hkv[CH];
#pragma unroll
    for (int t = 0; t < CH; ++t) kk[t] = (int)((cw >> (8 * t)) & 0xFFu);
#pragma unroll
    for (int t = 0; t < CH; ++t) cnt[t] = (int)ws.H[x.rb + kk[t]] + (int)ws.H[x.cb + kk[t]];
#pragma unroll
    for (int t = 0; t < CH; ++t) hkv[t] = ws.hk[kk[t]];
#pragma unroll
    for (int t = 0; t < CH; ++t) {
        const int k = kk[t];
        const int32_t b = (t == 0 && p0 == 0) ? x.base + eB : x.base;
        const int32_t eb = eA * cnt[t] + b;
        const uint32_t mt = (uint32_t)((mw >> (8 * t)) & 0xFFu);
        const bool allowed = mt <= relit || ((farok >> t) & 1u);
        // positions past the domain repeat its last colour and that colour's
        // mark: never better than the original, met first
        const bool ok = (k != x.s) && (allowed || eb < teb);
        const uint32_t hi = ((uint32_t)eb << 16) | (x.hv ^ hkv[t]);
        const bool take = ok && hi < lhi;
        lhi = take ? hi : lhi;
        lk = take ? (uint32_t)k : lk;
        took = took || take;
    }
}

// A zero the compiler cannot see through: added to a uniform address, it keeps
// a load in vector registers (its wait then falls at the first use).
__device__ __forceinline__ int vzero() {
    int z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    return z;
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
    return ((uint64_t)readlane_u32((uint32_t)(v >> 32), l) << 32) | readlane_u32((uint32_t)v, l);
}

__device__ __forceinline__ uint32_t pull(uint32_t v, int from) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute(from << 2, (int)v);
}

// The eligible list held in registers, one vertex per lane (m <= 64):
//   ev = v | S(v) << 16 | |D*(v)| << 24 (v = 0xFFFF: empty slot)
//   eb = rowcnt base | colcnt base << 16
//   ec = chunk offset | (chunks - 1) << 24
//   ep = row | column << 8 | degree << 24
constexpr uint32_t kEmpty = 0xFFFFu;

struct Slot {
    uint32_t ev, eb, ec, ep;
};

__device__ __forceinline__ Slot load_slot(const DevInstance &I, const LeanState &ws, int W, int v) {
    const int n = I.n, np1 = n + 1;
    const int w = v >> 5, b = v & 31;
    const uint32_t below = (1u << b) - 1u;
    const uint32_t vi = gptr(I.vinfo)[v];
    const uint32_t s = ws.S[v];
    uint32_t co = ws.wpre[w] + (uint32_t)b, code = 0u;
    for (int q = 0; q < ws.nplanes; ++q) {
        const uint32_t pq = ws.planes[q * W + w];
        co += (uint32_t)__popc(pq & below) << q;
        code |= ((pq >> b) & 1u) << q;
    }
    const uint32_t r = vi & 0xFFu, c = (vi >> 8) & 0xFFu;
    Slot x;
    x.ev = (uint32_t)v | (s << 16) | (((vi >> 16) & 0xFFu) << 24);
    x.eb = r * (uint32_t)np1 | (((uint32_t)n * np1 + c * (uint32_t)np1) << 16);
    x.ec = co | (code << 24);
    x.ep = r | (c << 8) | (vi & 0xFF000000u);
    return x;
}

__device__ __forceinline__ VData slot_data(const LeanState &ws, const Slot &e, uint32_t w1,
                                           int32_t eA, int32_t eB) {
    VData x;
    x.v = (int)(e.ev & 0xFFFFu);
    x.s = (int)((e.ev >> 16) & 0xFFu);
    x.d = e.ev >> 24;
    x.rb = (int)(e.eb & 0xFFFFu);
    x.cb = (int)(e.eb >> 16);
    x.co = e.ec & 0xFFFFFFu;
    x.nch = (e.ec >> 24) + 1u;
    x.vpay = e.ep | ((uint32_t)x.s << 16);
    x.hv = fmix32(w1 ^ (uint32_t)x.v) >> 16;
    const int32_t cur = x.s ? ((int32_t)ws.H[x.rb + x.s] + (int32_t)ws.H[x.cb + x.s] - 2) : 0;
    x.base = 0x8000 + (x.s ? 0 : -eB) - eA * cur;
    return x;
}

template <int CH, int PH>
__device__ void lean_phase(const PlitsArgs &a, uint32_t iters, uint32_t slot, uint32_t gen,
                           const uint8_t *src, uint8_t *out, uint32_t *gfar, const LeanState &ws,
                           Scal &sc, Cnt &ucnt, uint32_t &lane_cands) {
    const DevInstance I = a.I;  // by value: the pointers the search uses stay in registers
    const int lane = lane_id();
    const int n = I.n, nv = I.nv, np1 = n + 1;
    const int W = (nv + 31) >> 5;
    const int npos = a.npos;
    const int32_t phi_num = (PH == 1) ? 1 : nv;
    const int32_t phi_den = (PH == 1) ? 2 : 1;
    const uint32_t tag = PH == 1 ? TAG_PLITS1 : TAG_PLITS2;
    // move values on a 16-bit scale e ordered like delta (see the other PLITS
    // kernel): e = delta, or e = 4 dc + df in phase 2 with |V| > 64
    const bool squeeze = (PH == 2 && nv > 64);
    const int32_t eA = (PH == 1) ? 1 : (squeeze ? 4 : nv);
    const int32_t eB = (PH == 1) ? 2 : 1;
    const uint32_t alpha_n = (uint32_t)a.P.alpha_num, alpha_d = (uint32_t)a.P.alpha_den;
    const uint32_t m_alpha = 0xFFFFFFFFu / alpha_d;
    uint8_t *H = ws.H;
    const int colH0 = n * np1;

    lean_setup(I, src, ws, npos, sc);
    if (src != out) lean_snapshot(I, ws.S, out);
    sc.F = (int64_t)phi_den * sc.f + (int64_t)phi_num * sc.c;
    sc.Fbest = sc.F;
    sc.fbest = sc.f;
    sc.cbest = sc.c;
    uint32_t wx = 0u, wy = 0u, wz = 0u;
    uint32_t tbase = 0u;
    const uint32_t ln_new = lane >= 2 ? 0xFFFFFFFFu : 0u;
    const uint32_t ln_odd = (lane & 1) ? 0xFFFFFFFFu : 0u;
    const uint32_t lane0 = lane == 0 ? 0xFFFFFFFFu : 0u;
    uint16_t *stage = reinterpret_cast<uint16_t *>(ws.stage);
    uint8_t *flag = reinterpret_cast<uint8_t *>(ws.stage) + kLeanFlags;
    uint16_t *ins = reinterpret_cast<uint16_t *>(reinterpret_cast<uint8_t *>(ws.stage) + kLeanIns);
    const uint32_t *rclo = reinterpret_cast<const uint32_t *>(
        reinterpret_cast<const uint8_t *>(ws.stage) + kLeanRclo);
    // the eligible list (valid while `listed`: every eligible vertex in a slot)
    Slot e{kEmpty, 0u, 0u, 0u};
    bool listed = false;
    PLSE_WAVE_SYNC();

    for (uint32_t itu = 0; itu < iters; ++itu) {
        if ((itu & 63u) == 0u) {
            const U4 rw = draw(a.seed_lo, a.seed_hi, slot, gen, tag, itu + (uint32_t)lane);
            wx = rw.x;
            wy = rw.y;
            wz = rw.z;
        }
        if ((itu & 127u) == 0u && itu != 0u) {
            tbase += 128u;
            lean_rebase<CH>(ws, npos, gfar, tbase);
            fold(ucnt);
            PLSE_WAVE_SYNC();
        }
        const uint32_t w0 = readlane_u32(wx, (int)(itu & 63u));
        const uint32_t w1 = readlane_u32(wy, (int)(itu & 63u));
        const uint32_t w2 = readlane_u32(wz, (int)(itu & 63u));
        if (lane <= n) ws.hk[lane] = (uint16_t)(fmix32(w2 ^ (uint32_t)lane) >> 16);
        if (lane + 64 <= n) ws.hk[lane + 64] = (uint16_t)(fmix32(w2 ^ (uint32_t)(lane + 64)) >> 16);

        // 1. eligible vertices: from the list, or (when it is not valid) a
        //    scan of the bitmap, staging the first kLeanStage; at most 64 of
        //    them go (back) into the list
        uint32_t m = 0;
        if (listed) {
            m = (uint32_t)__popcll(ballot((e.ev & 0xFFFFu) != kEmpty));
        } else {
            for (int wb = 0; wb < W; wb += 64) {
                const int w = wb + lane;
                uint32_t bits = (w < W) ? ws.bm[w] : 0u;
                uint32_t total;
                uint32_t pos = m + wave_excl_scan_dpp((uint32_t)__popc(bits), &total);
#pragma unroll 1
                while (bits && pos < (uint32_t)kLeanStage) {
                    const int b = __ffs(bits) - 1;
                    bits &= bits - 1u;
                    stage[pos++] = (uint16_t)(w * 32 + b);
                }
                m += total;
            }
            PLSE_WAVE_SYNC();
            if (m <= 64u) {
                e = (uint32_t)lane < m ? load_slot(I, ws, W, (int)stage[lane])
                                       : Slot{kEmpty, 0u, 0u, 0u};
                listed = true;
            }
        }
        if (m == 0) break;  // F = 0: complete legal colouring
        ucnt.iters++;
        ucnt.pelig += m & lane0;

        // 2. best admissible one-move per lane; aspiration F + delta < F* is
        //    e + 2^15 < teb
        int32_t te;
        if (!squeeze) {
            const int64_t gap = sc.Fbest - sc.F;
            te = gap < -(1ll << 30) ? -(1 << 30) : (int32_t)gap;
        } else {
            te = squeezed_bound(sc.fbest - sc.f, sc.cbest - sc.c, nv);
        }
        const int32_t teb = te + 0x8000;
        const uint32_t relit = itu - tbase + 1u;
        uint32_t lhi = 0xFFFFFFFFu, lv = 0u, lk = 0u, lpay = 0u, lco = 0u;
        if (listed) {
            // lane g takes chunk g of the listed vertices when they fit the
            // wave: its vertex holds the last chunk start at or below g
            const bool act = (e.ev & 0xFFFFu) != kEmpty;
            const VData x = slot_data(ws, e, w1, eA, eB);
            const uint32_t nmine = act ? x.nch : 0u;
            if (act) lane_cands += x.d;
            uint32_t C;
            const uint32_t s0 = wave_excl_scan_dpp(nmine, &C);
            if (C <= 64u) {
                flag[lane] = 0;
                if (act) flag[s0] = 1;
                PLSE_WAVE_SYNC();
                const uint64_t starts = ballot(flag[lane] != 0);
                const int src_l = (int)(rank_below(starts) + (uint32_t)((starts >> lane) & 1ull)) - 1;
                // the lane of the src_l-th listed vertex
                const uint64_t occ = ballot(act);
                int owner = 0;
                {
                    // position of the (src_l)-th set bit of occ: lanes hold
                    // listed vertices in any order, so pull through their ranks
                    const uint32_t myrank = rank_below(occ);
                    flag[act ? myrank : 64 + (lane & 15)] = (uint8_t)lane;
                    PLSE_WAVE_SYNC();
                    owner = flag[src_l < 0 ? 0 : src_l];
                }
                VData y;
                y.v = (int)pull((uint32_t)x.v, owner);
                y.s = (int)pull((uint32_t)x.s, owner);
                y.rb = (int)pull((uint32_t)x.rb, owner);
                y.cb = (int)pull((uint32_t)x.cb, owner);
                y.co = pull(x.co, owner);
                y.vpay = pull(x.vpay, owner);
                y.hv = pull(x.hv, owner);
                y.base = (int32_t)pull((uint32_t)x.base, owner);
                const uint32_t j = (uint32_t)lane - pull(s0, owner);
                bool took = false;
                if ((uint32_t)lane < C)
                    eval_chunk<CH>(I, ws, gfar, y, j, itu, relit, teb, eA, eB, lhi, lk, took);
                lv = (uint32_t)y.v;
                lpay = y.vpay;
                lco = y.co;
            } else {
                bool took = false;
                for (uint32_t j = 0; j < nmine; ++j)
                    eval_chunk<CH>(I, ws, gfar, x, j, itu, relit, teb, eA, eB, lhi, lk, took);
                lv = (uint32_t)x.v;
                lpay = x.vpay;
                lco = x.co;
            }
        } else {
            // more than 64 eligible vertices (early in a phase): lanes take
            // whole vertices, kLeanStage staged at a time
            for (uint32_t g0 = 0; g0 < m; g0 += (uint32_t)kLeanStage) {
                if (g0 > 0) {
                    PLSE_WAVE_SYNC();
                    const uint32_t gend = g0 + (uint32_t)kLeanStage;
                    uint32_t basec = 0;
                    for (int wb = 0; wb < W && basec < gend; wb += 64) {
                        const int w = wb + lane;
                        uint32_t bits = (w < W) ? ws.bm[w] : 0u;
                        uint32_t total;
                        uint32_t pos = basec + wave_excl_scan_dpp((uint32_t)__popc(bits), &total);
#pragma unroll 1
                        while (bits && pos < gend) {
                            const int b = __ffs(bits) - 1;
                            bits &= bits - 1u;
                            if (pos >= g0) stage[pos - g0] = (uint16_t)(w * 32 + b);
                            ++pos;
                        }
                        basec += total;
                    }
                    PLSE_WAVE_SYNC();
                }
                const uint32_t mb = min(m - g0, (uint32_t)kLeanStage);
                for (uint32_t pb = 0; pb < mb; pb += 64u) {
                    const uint32_t q = pb + (uint32_t)lane;
                    if (q < mb) {
                        const VData x = vertex_data(I, ws, W, (int)stage[q], w1, eA, eB);
                        lane_cands += x.d;
                        bool took = false;
                        for (uint32_t j = 0; j < x.nch; ++j)
                            eval_chunk<CH>(I, ws, gfar, x, j, itu, relit, teb, eA, eB, lhi, lk,
                                           took);
                        lv = took ? (uint32_t)x.v : lv;
                        lpay = took ? x.vpay : lpay;
                        lco = took ? x.co : lco;
                    }
                }
            }
        }
        // 3. unique best over the wave: minimum of the upper key words, then
        //    of the move ids among the lanes holding it
        const uint32_t ghi = wave_min_u32_dpp(lhi);
        if (ghi == 0xFFFFFFFFu) {
            ucnt.idle++;
            PLSE_WAVE_SYNC();
            continue;
        }
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
        const uint32_t vco = readlane_u32(lco, wl);
        const int r = (int)(pay & 0xFFu);
        const int c = (int)((pay >> 8) & 0xFFu);
        const int old = (int)((pay >> 16) & 0xFFu);
        const int deg = (int)(pay >> 24);
        const int rb = r * np1, cb = colH0 + c * np1;
        // counts of the two colours in v's row and column, the vertices of
        // that row and column, and v's domain mask (the tabu position of the
        // colour it leaves), fetched together
        // (uniform values read from LDS are moved to scalar registers, so the
        // work on them stays scalar and loops over them stay uniform)
        const int32_t hk_r = readfirst(H[rb + k]), hk_c = readfirst(H[cb + k]);
        const int32_t ho_r = readfirst(H[rb + old]), ho_c = readfirst(H[cb + old]);
        const uint32_t r0 = (uint32_t)readfirst((int)rclo[r]);
        const uint32_t nr = (uint32_t)readfirst((int)rclo[r + 1]) - r0;
        const uint32_t c0 = (uint32_t)readfirst((int)rclo[n + c]);
        const uint32_t nc = (uint32_t)readfirst((int)rclo[n + c + 1]) - c0;
        const uint32_t nrc = nr + nc;
        uint32_t ent0 = 0xFFFFu, ent1 = 0xFFFFu;
        {
            const uint32_t q0 = (uint32_t)lane, q1 = (uint32_t)lane + 64u;
            if (q0 < nrc) ent0 = gptr(I.rcl)[q0 < nr ? r0 + q0 : c0 + q0 - nr];
            if (q1 < nrc) ent1 = gptr(I.rcl)[q1 < nr ? r0 + q1 : c0 + q1 - nr];
        }
        // (read per lane so the wait for it falls where it is used)
        const u32x4 dmask = gload4(reinterpret_cast<const u32x4 *>(I.vrec) + 2 * v + vzero());
        const int32_t cvk = k ? hk_r + hk_c : 0;
        const int32_t cvo = old ? ho_r + ho_c - 2 : 0;
        const bool vC = (k != 0) && (cvk > 0);
        PLSE_WAVE_SYNC();
        // 4. apply.  Counts: lanes 0-1 the leaving colour's row and column
        //    count (-1), lanes 2-3 the entering colour's (+1), as LDS adds on
        //    the bytes of u32 words (exact: counts stay within 0..n), an add of
        //    0 for colour 0.  Lane 0: v's colour and eligibility bit.
        if (lane < 4) {
            const uint32_t col = (ln_new & (uint32_t)k) | (~ln_new & (uint32_t)old);
            const uint32_t hb = ((ln_odd & (uint32_t)cb) | (~ln_odd & (uint32_t)rb)) + col;
            const uint32_t add = col != 0u ? ((ln_new & 2u) - 1u) << ((hb & 3u) * 8u) : 0u;
            atomicAdd(reinterpret_cast<uint32_t *>(H) + (hb >> 2), add);
        }
        if (lane == 0) {
            ws.S[v] = (uint8_t)k;
            atomicAdd(&ws.bm[v >> 5], (k == 0 || vC) ? 0u : 0u - (1u << (v & 31)));
        }
        PLSE_WAVE_SYNC();
        // eligibility of the row and column vertices holding the old or the
        // new colour: one toggle where it changes; the vertices that become
        // eligible are noted for the list
        int32_t dC = 0;
        uint32_t nins = 0;
        for (uint32_t qb = 0; qb < nrc; qb += 64u) {
            const uint32_t qq = (uint32_t)lane + qb;
            uint32_t ent = qb == 0u ? ent0 : ent1;
            if (qb >= 128u)
                ent = qq < nrc ? gptr(I.rcl)[qq < nr ? r0 + qq : c0 + qq - nr] : 0xFFFFu;
            const int u = (int)(ent & 0xFFFFu), other = (int)(ent >> 16);
            const bool valid = ent != 0xFFFFu && u != v;
            const int uu = valid ? u : 0;
            const int su = ws.S[uu];
            const uint32_t bw = ws.bm[uu >> 5];
            // a row vertex (r, other); a column vertex (other, c)
            const bool inrow = qq < nr;
            const int ub = (inrow ? rb : other * np1) + su;
            const int uc = (inrow ? colH0 + other * np1 : cb) + su;
            const int cu = (int)H[ub] + (int)H[uc] - 2;
            const bool hit = valid && su != 0 && (su == old || su == k);
            const bool was = (bw >> (uu & 31)) & 1u;
            const bool now = cu > 0;
            const bool flip = hit && (now != was);
            if (flip) atomicXor(&ws.bm[uu >> 5], 1u << (uu & 31));
            const uint64_t up = ballot(flip && now);
            if (flip && now) ins[nins + rank_below(up)] = (uint16_t)uu;
            nins += (uint32_t)__popcll(up);
            dC += (int32_t)__popcll(up) - (int32_t)__popcll(ballot(flip && !now));
        }
        const int32_t df = (k == 0 ? 1 : 0) - (old == 0 ? 1 : 0);
        sc.nC += dC + (vC ? 1 : 0) - (old ? 1 : 0);
        sc.f += df;
        sc.c += cvk - cvo;
        sc.F += (int64_t)phi_den * df + (int64_t)phi_num * (cvk - cvo);
        const uint32_t ends = (uint32_t)(old != 0) + (uint32_t)(k != 0);
        ucnt.pcupd += (2u * ends) & lane0;
        ucnt.pnupd += ((uint32_t)deg * ends) & lane0;
        // tenure T = L + alpha (|V_0| + |C|) after the move; moving v back to
        // `old` is tabu for T iterations.  The mark of the last domain colour
        // is repeated over the rest of its chunk, where the candidate row
        // repeats that colour.
        const uint32_t mp = (uint32_t)(sc.f + sc.nC);
        const uint32_t T = scale32(w0, 10u) + udiv_by(alpha_n * mp, alpha_d, m_alpha);
        const uint32_t until = itu + 1u + T;
        {
            const uint32_t po = lean_position(dmask, old);
            const uint32_t dv = (uint32_t)(__popcll(((uint64_t)dmask.y << 32) | dmask.x) +
                                           __popcll(((uint64_t)dmask.w << 32) | dmask.z));
            const uint32_t nrep = po == dv ? (uint32_t)CH - dv % (uint32_t)CH : 1u;
            const uint32_t rel = until - tbase;
            const bool far = rel > 253u;
            const uint32_t mark = far ? 255u : rel + 1u;
            const uint32_t mpos = vco * CH + po;
            if ((uint32_t)lane < nrep) {
                ws.mk[mpos + lane] = (uint8_t)mark;
                if (far) gptr(gfar)[mpos + lane] = until;
            }
            if (far && lane == 0) atomicOr(&ws.dirty[v >> 5], 1u << (v & 31));
        }
        PLSE_WAVE_SYNC();
        if (listed) {
            // the list after the move: v's colour, the vertices that stopped
            // being eligible dropped, the new ones into empty slots
            const int ve = (int)(e.ev & 0xFFFFu);
            if (ve == v) e.ev = (e.ev & 0xFF00FFFFu) | ((uint32_t)k << 16);
            const bool keep = ve != (int)kEmpty && ((ws.bm[ve >> 5] >> (ve & 31)) & 1u);
            if (!keep) e.ev = kEmpty;
            const uint64_t empty = ballot(!keep);
            if (nins > (uint32_t)__popcll(empty)) {
                listed = false;  // more than 64: the next iteration scans
            } else if (nins > 0u) {
                const uint32_t er = rank_below(empty);
                if (!keep && er < nins) e = load_slot(I, ws, W, (int)ins[er]);
            }
        }
        if (sc.F < sc.Fbest) {
            sc.Fbest = sc.F;
            sc.fbest = sc.f;
            sc.cbest = sc.c;
            lean_snapshot(I, ws.S, out);
            ucnt.snaps++;
        }
    }
    fold(ucnt);
    PLSE_WAVE_SYNC();
    lean_clear_far<CH>(I, ws, gfar);
    PLSE_WAVE_SYNC();
}

// Greedy conflict removal (Section 3.7): uncolour the vertex with the most
// conflicts (ties: lowest id) until the colouring is legal; `from` -> `out`.
__device__ void lean_repair(const PlitsArgs &a, const uint8_t *from, uint8_t *out,
                            const LeanState &ws, Scal &sc, Cnt &ucnt) {
    const DevInstance &I = a.I;
    const int lane = lane_id();
    const int n = I.n, nv = I.nv, np1 = n + 1;
    lean_setup(I, from, ws, 0, sc);
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
    lean_snapshot(I, ws.S, out);
    PLSE_WAVE_SYNC();
}

}  // namespace

template <int CH>
__global__ __launch_bounds__(256) void plits_lean_kernel(const ArgList L) {
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
    const DevInstance &I = a.I;
    const int W = (I.nv + 31) >> 5;
    uint8_t *base = lds + (size_t)wv * a.lds_per_wave;
    LeanState ws;
    ws.S = base;
    ws.H = base + a.off_h;
    ws.bm = reinterpret_cast<uint32_t *>(base + a.off_bm);
    ws.mk = base + a.off_mk;
    ws.dirty = reinterpret_cast<uint32_t *>(base + a.off_dirty);
    ws.planes = reinterpret_cast<uint32_t *>(base + a.off_planes);
    ws.wpre = reinterpret_cast<uint32_t *>(base + a.off_wpre);
    ws.stage = reinterpret_cast<u32x2 *>(base + a.off_el);
    ws.hk = reinterpret_cast<uint16_t *>(base + a.off_hk);
    ws.nplanes = a.nplanes;
    {
        // chunk-count planes (bit b of floor(|D*(v)| / CH)) and each word's
        // chunk offset (wave prefix sum of the words' chunk totals)
        uint32_t run = 0u;
        for (int wb = 0; wb < W; wb += 64) {
            const int w = wb + lane_id();
            uint32_t pl[7] = {0u, 0u, 0u, 0u, 0u, 0u, 0u};
            uint32_t cnt = 0u;
            if (w < W) {
                const int vend = min(I.nv, (w + 1) * 32);
                for (int v = w * 32; v < vend; ++v) {
                    const uint32_t code = ((gptr(I.vinfo)[v] >> 16) & 0xFFu) / CH;
#pragma unroll
                    for (int b = 0; b < 7; ++b) pl[b] |= ((code >> b) & 1u) << (v & 31);
                    cnt += code + 1u;
                }
                for (int b = 0; b < a.nplanes; ++b) ws.planes[b * W + w] = pl[b];
            }
            uint32_t total;
            const uint32_t pre = run + wave_excl_scan_dpp(cnt, &total);
            if (w < W) ws.wpre[w] = pre;
            run += total;
        }
        // row/column list offsets
        uint32_t *rclo = reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(ws.stage) +
                                                      kLeanRclo);
        for (int q = lane_id(); q <= 2 * I.n; q += 64) rclo[q] = gptr(I.rclo)[q];
        PLSE_WAVE_SYNC();
    }
    uint32_t *gfar = a.tabu + (size_t)ind * I.nv * I.ts;
    const uint8_t *src = a.S_in + (size_t)ind * I.stride;
    uint8_t *out = a.S_out + (size_t)ind * I.stride;

    Cnt ucnt{0u, 0u, 0u, 0u, 0ull, 0ull, 0ull, 0u, 0u, 0u};
    uint32_t lane_cands = 0;
    Scal sc;
    const uint32_t slot = (uint32_t)readfirst(ind);
    // phase 1 from the offspring, phase 2 from phase 1's best (both write
    // their best into `out`), then the legality guard
    lean_phase<CH, 1>(a, (uint32_t)a.P.depth1, slot, (uint32_t)gen, src, out, gfar, ws, sc, ucnt,
                      lane_cands);
    lean_phase<CH, 2>(a, (uint32_t)a.P.depth2, slot, (uint32_t)gen, out, out, gfar, ws, sc, ucnt,
                      lane_cands);
    int32_t f_final = sc.fbest;
    if (sc.cbest > 0) {
        lean_repair(a, out, out, ws, sc, ucnt);
        f_final = sc.f + (int32_t)ucnt.repairs;
    }
    const uint64_t cands = wave_sum_u64(lane_cands);
    // lane 0's totals, read while every lane is active
    const uint64_t elig = readlane_u64(ucnt.elig, 0), nupd = readlane_u64(ucnt.nupd, 0),
                   cupd = readlane_u64(ucnt.cupd, 0);
    const int lane = lane_id();
    if (lane < kCounters) {
        uint64_t v = 0;
        switch (lane) {
            case C_ITERS: v = ucnt.iters; break;
            case C_MOVES: v = ucnt.iters - ucnt.idle; break;
            case C_IDLE: v = ucnt.idle; break;
            case C_CANDS: v = cands; break;
            case C_ELIG: v = elig; break;
            case C_NUPD: v = nupd; break;
            case C_SNAPS: v = ucnt.snaps; break;
            case C_REPAIRS: v = ucnt.repairs; break;
            default: v = cupd; break;
        }
        gptr(a.cnt_out)[(size_t)ind * kCounters + lane] = v;
    }
    if (lane == 0) gptr(a.f_out)[ind] = f_final;
}

const void *plits_lean_fn(int slots_per_lane) {
    switch (slots_per_lane) {
        case 2: return (const void *)plits_lean_kernel<2>;
        case 4: return (const void *)plits_lean_kernel<4>;
        case 8: return (const void *)plits_lean_kernel<8>;
        default: return nullptr;
    }
}

}  // namespace plse

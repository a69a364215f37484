// k_plits.hip -- PLITS, the two-phase tabu search of Section 3.3 (Alg. 3),
// one wave64 per individual on gfx950.
//
// Layout of one individual's state:
//   LDS (per wave): S[stride] colours, cs[stride] slot of the current colour in
//     D*(v) (kNoSlot if uncoloured), bm[W] eligibility bitmap (V_0 u C(S)), and
//     a scratch area that holds the eligible-vertex list during the search and
//     the row/column colour histograms while the conflict table is rebuilt.
//   HBM (per individual, in the workspace): conf[nd] conflict counts for every
//     (v, k in D*(v)) -- the incremental evaluation table of Section 3.3 -- and
//     tabu[nd + nv] "allowed from" iterations for every (v, k in D(v)).
//   Instance tables (domains, slot map, row/column vertex lists) are shared by
//   all waves and served from L1/L2.
//
// One iteration:
//   1. expand the eligibility bitmap into a list (wave prefix sum);
//   2. each lane evaluates every one-move of its eligible vertices: move value
//      from the conflict table, admissibility from the tabu table and the
//      aspiration test, and keeps its best (value, tie-hash) key;
//   3. wave min over 64-bit keys picks the unique best admissible move;
//   4. the lanes update the conflict counts of the moved vertex's row and
//      column neighbours and their eligibility bits;
//   5. tenure, tabu entry, best-solution snapshot.
#include "device_common.h"
#include "kernels.h"

namespace plse {


namespace {

struct WaveState {
    uint8_t *S;
    uint8_t *cs;
    uint32_t *bm;
    uint8_t *scr;
};

struct Scal {
    int64_t F, Fbest;
    int32_t f, c, nC;        // uncoloured, conflicting edges, conflicting vertices
    int32_t fbest, cbest;
};

// Build S (from `src`), the conflict table, the current-slot array and the
// eligibility bitmap from scratch; returns f, c and |C(S)|.  conf[v][k] is the
// number of neighbours of v coloured k = (row count of k) + (column count of
// k) - 2 [S(v) = k], from per-row and per-column colour histograms.
template <typename ConfT>
__device__ void setup_state(const DevInstance &I, const uint8_t *src, ConfT *conf,
                            const WaveState &ws, Scal &sc) {
    const int lane = lane_id();
    const int n = I.n, nv = I.nv, np1 = n + 1;
    const int nchunks = I.stride >> 4;
    for (int q = lane; q < nchunks; q += 64)
        reinterpret_cast<uint4 *>(ws.S)[q] = reinterpret_cast<const uint4 *>(src)[q];
    // histograms: row r colour k at byte r*np1+k, column c colour k after them
    const int hbytes = 2 * n * np1;
    uint32_t *h32 = reinterpret_cast<uint32_t *>(ws.scr);
    for (int q = lane; q < (hbytes + 3) / 4; q += 64) h32[q] = 0u;
    PLSE_WAVE_SYNC();
    for (int v = lane; v < nv; v += 64) {
        const int s = ws.S[v];
        if (s) {
            const int a = I.vrow[v] * np1 + s;
            const int b = n * np1 + I.vcol[v] * np1 + s;
            atomicAdd(&h32[a >> 2], 1u << ((a & 3) * 8));
            atomicAdd(&h32[b >> 2], 1u << ((b & 3) * 8));
        }
    }
    PLSE_WAVE_SYNC();
    const uint8_t *rowH = ws.scr;
    const uint8_t *colH = ws.scr + n * np1;
    const int W = (nv + 31) >> 5;
    int32_t f = 0, c2 = 0, nC = 0;
    for (int w = lane; w < W; w += 64) {
        uint32_t bits = 0u;
        const int vend = min(nv, (w + 1) * 32);
        for (int v = w * 32; v < vend; ++v) {
            const int s = ws.S[v];
            const int r = I.vrow[v] * np1, cc = I.vcol[v] * np1;
            const uint32_t off = I.doff[v], d = I.doff[v + 1] - off;
            uint8_t js = kNoSlot;
            int own = 0;
            for (uint32_t j = 0; j < d; ++j) {
                const int k = I.dom[off + j];
                const int x = (int)rowH[r + k] + (int)colH[cc + k] - (k == s ? 2 : 0);
                conf[off + j] = (ConfT)x;
                if (k == s) {
                    js = (uint8_t)j;
                    own = x;
                }
            }
            ws.cs[v] = js;
            if (s == 0 || own > 0) bits |= 1u << (v & 31);
            f += (s == 0);
            c2 += own;
            nC += (s != 0 && own > 0);
        }
        ws.bm[w] = bits;
    }
    PLSE_WAVE_SYNC();
    sc.f = (int32_t)wave_sum_u32((uint32_t)f);
    sc.c = (int32_t)(wave_sum_u32((uint32_t)c2) >> 1);  // each conflicting edge counted twice
    sc.nC = (int32_t)wave_sum_u32((uint32_t)nC);
}

__device__ __forceinline__ void snapshot(const DevInstance &I, const uint8_t *S, uint8_t *dst) {
    const int nchunks = I.stride >> 4;
    for (int q = lane_id(); q < nchunks; q += 64)
        reinterpret_cast<uint4 *>(dst)[q] = reinterpret_cast<const uint4 *>(S)[q];
}

// One phase of PLITS.  `src` is the start solution, `out` receives the
// phase's best solution (the snapshot target).
template <typename ConfT>
__device__ void run_phase(const PlitsArgs &a, int phase, int64_t iters, uint32_t slot,
                          uint32_t gen, const uint8_t *src, uint8_t *out, ConfT *conf,
                          uint32_t *tabu, const WaveState &ws, Scal &sc, uint64_t *ucnt,
                          uint32_t &lane_cands, uint32_t &lane_nupd) {
    const DevInstance &I = a.I;
    const int lane = lane_id();
    const int n = I.n, nv = I.nv, np1 = n + 1;
    // F = phi_den * f + phi_num * c: phase 1 phi = 1/2, phase 2 phi = |V|.
    const int32_t phi_num = (phase == 1) ? 1 : nv;
    const int32_t phi_den = (phase == 1) ? 2 : 1;
    const uint32_t tag = (phase == 1) ? TAG_PLITS1 : TAG_PLITS2;

    setup_state<ConfT>(I, src, conf, ws, sc);
    if (src != out) snapshot(I, ws.S, out);
    {
        const int ntab = I.nd + nv;
        for (int q = lane; q < ntab; q += 64) tabu[q] = 0u;
    }
    sc.F = (int64_t)phi_den * sc.f + (int64_t)phi_num * sc.c;
    sc.Fbest = sc.F;
    sc.fbest = sc.f;
    sc.cbest = sc.c;
    const int W = (nv + 31) >> 5;
    uint16_t *elist = reinterpret_cast<uint16_t *>(ws.scr);
    PLSE_WAVE_SYNC();

    for (int64_t it = 0; it < iters; ++it) {
        // 1. eligible vertices V_0 u C(S), in ascending order
        uint32_t m = 0;
        for (int wb = 0; wb < W; wb += 64) {
            const int w = wb + lane;
            uint32_t bits = (w < W) ? ws.bm[w] : 0u;
            uint32_t total;
            uint32_t pos = m + wave_excl_scan((uint32_t)__popc(bits), &total);
            while (bits) {
                const int b = __ffs(bits) - 1;
                bits &= bits - 1u;
                elist[pos++] = (uint16_t)(w * 32 + b);
            }
            m += total;
        }
        if (m == 0) break;  // F = 0: complete legal colouring
        PLSE_WAVE_SYNC();
        ucnt[C_ITERS]++;
        ucnt[C_ELIG] += m;
        const U4 rw = draw(a.seed_lo, a.seed_hi, slot, gen, tag, (uint32_t)it);
        const uint32_t itu = (uint32_t)it;

        // 2. best admissible one-move per lane
        uint64_t lbest = ~0ull;
        uint32_t lpay = 0u;
        for (uint32_t e = lane; e < m; e += 64) {
            const int v = elist[e];
            const int s = ws.S[v];
            const int js = ws.cs[v];
            const uint32_t off = I.doff[v], d = I.doff[v + 1] - off;
            const uint32_t *tb = tabu + off + v;  // [0] colour 0, [1+j] slot j
            const int32_t cur = s ? (int32_t)conf[off + js] : 0;
            const int32_t dfb = s ? 0 : -phi_den;
            const uint32_t cid0 = (uint32_t)(v * np1);
            lane_cands += d;
            for (uint32_t j = 0; j < d; ++j) {
                if ((int)j == js) continue;
                const int32_t delta = dfb + phi_num * ((int32_t)conf[off + j] - cur);
                const bool adm = (itu >= tb[1 + j]) || (sc.F + delta < sc.Fbest);
                if (adm) {
                    const uint64_t key =
                        ((uint64_t)((uint32_t)delta + 0x80000000u) << 32) |
                        fmix32(rw.y ^ (cid0 + I.dom[off + j]));
                    if (key < lbest) {
                        lbest = key;
                        lpay = ((uint32_t)v << 8) | (j + 1);
                    }
                }
            }
            if (s) {  // a conflicting vertex may also become uncoloured
                const int32_t delta = phi_den - phi_num * cur;
                const bool adm = (itu >= tb[0]) || (sc.F + delta < sc.Fbest);
                if (adm) {
                    const uint64_t key =
                        ((uint64_t)((uint32_t)delta + 0x80000000u) << 32) | fmix32(rw.y ^ cid0);
                    if (key < lbest) {
                        lbest = key;
                        lpay = (uint32_t)v << 8;
                    }
                }
            }
        }
        // 3. unique best over the wave
        const uint64_t gmin = wave_min_u64(lbest);
        if (gmin == ~0ull) {
            ucnt[C_IDLE]++;
            continue;
        }
        const uint64_t who = ballot(lbest == gmin);
        const uint32_t pay = shfl_u32(lpay, __ffsll((unsigned long long)who) - 1);
        const int v = (int)(pay >> 8);
        const int jp = (int)(pay & 0xFFu);
        const int32_t delta = (int32_t)((uint32_t)(gmin >> 32) - 0x80000000u);
        const int old = ws.S[v];
        const int jold = ws.cs[v];
        const uint32_t voff = I.doff[v];
        const int k = jp ? I.dom[voff + jp - 1] : 0;
        const int32_t cvk = jp ? (int32_t)conf[voff + jp - 1] : 0;
        const int32_t cvo = old ? (int32_t)conf[voff + jold] : 0;

        // 4. conflict counts of the row and column neighbours
        const int r = I.vrow[v], c = I.vcol[v];
        const int nr = I.rowc[r], nc = I.colc[c];
        int32_t dC = 0;
        for (int t0 = 0; t0 < nr + nc; t0 += 64) {
            const int t = t0 + lane;
            bool leave = false, enter = false;
            if (t < nr + nc) {
                const int u = (t < nr) ? I.rowv[r * n + t] : I.colv[c * n + (t - nr)];
                if (u != v) {
                    const int su = ws.S[u];
                    const uint32_t uoff = I.doff[u];
                    const uint8_t *us = I.slot + (size_t)u * np1;
                    if (old) {
                        const int so = us[old];
                        if (so != kNoSlot) {
                            const int x = (int)conf[uoff + so];
                            conf[uoff + so] = (ConfT)(x - 1);
                            lane_nupd++;
                            if (su == old && x == 1) {
                                leave = true;
                                atomicAnd(&ws.bm[u >> 5], ~(1u << (u & 31)));
                            }
                        }
                    }
                    if (k) {
                        const int sk = us[k];
                        if (sk != kNoSlot) {
                            const int x = (int)conf[uoff + sk];
                            conf[uoff + sk] = (ConfT)(x + 1);
                            lane_nupd++;
                            if (su == k && x == 0) {
                                enter = true;
                                atomicOr(&ws.bm[u >> 5], 1u << (u & 31));
                            }
                        }
                    }
                }
            }
            dC += (int32_t)__popcll(ballot(enter)) - (int32_t)__popcll(ballot(leave));
        }
        const bool vC = (k != 0) && (cvk > 0);
        if (lane == 0) {
            ws.S[v] = (uint8_t)k;
            ws.cs[v] = jp ? (uint8_t)(jp - 1) : kNoSlot;
            if (k == 0 || vC)
                atomicOr(&ws.bm[v >> 5], 1u << (v & 31));
            else
                atomicAnd(&ws.bm[v >> 5], ~(1u << (v & 31)));
        }
        sc.nC += dC + (vC ? 1 : 0) - (old ? 1 : 0);
        sc.f += (k == 0 ? 1 : 0) - (old == 0 ? 1 : 0);
        sc.c += cvk - cvo;
        sc.F += delta;

        // 5. tenure T = L + alpha (|V_0| + |C|) after the move; the move back
        //    to `old` is tabu for T iterations
        const int64_t mp = (int64_t)sc.f + sc.nC;
        const uint32_t T = scale32(rw.x, 10u) + (uint32_t)((a.P.alpha_num * mp) / a.P.alpha_den);
        if (lane == 0) tabu[voff + v + (old ? (uint32_t)jold + 1u : 0u)] = itu + 1u + T;
        ucnt[C_MOVES]++;
        PLSE_WAVE_SYNC();
        if (sc.F < sc.Fbest) {
            sc.Fbest = sc.F;
            sc.fbest = sc.f;
            sc.cbest = sc.c;
            snapshot(I, ws.S, out);
            ucnt[C_SNAPS]++;
        }
        PLSE_WAVE_SYNC();
    }
    PLSE_WAVE_SYNC();
}

// Greedy conflict removal (Section 3.7): uncolour the vertex with the most
// conflicts (ties: lowest id) until the colouring is legal.
template <typename ConfT>
__device__ void repair(const PlitsArgs &a, uint8_t *out, ConfT *conf, const WaveState &ws,
                       Scal &sc, uint64_t *ucnt) {
    const DevInstance &I = a.I;
    const int lane = lane_id();
    const int n = I.n, nv = I.nv, np1 = n + 1;
    setup_state<ConfT>(I, out, conf, ws, sc);
    for (;;) {
        uint32_t lkey = 0u;
        for (int v = lane; v < nv; v += 64) {
            const int s = ws.S[v];
            if (s) {
                const uint32_t cv = conf[I.doff[v] + ws.cs[v]];
                if (cv) {
                    const uint32_t key = (cv << 16) | (0xFFFFu - (uint32_t)v);
                    lkey = key > lkey ? key : lkey;
                }
            }
        }
        const uint32_t g = wave_max_u32(lkey);
        if (g == 0u) break;
        const int v = (int)(0xFFFFu - (g & 0xFFFFu));
        const int old = ws.S[v];
        const int r = I.vrow[v], c = I.vcol[v];
        const int nr = I.rowc[r], nc = I.colc[c];
        for (int t = lane; t < nr + nc; t += 64) {
            const int u = (t < nr) ? I.rowv[r * n + t] : I.colv[c * n + (t - nr)];
            if (u == v) continue;
            const int so = I.slot[(size_t)u * np1 + old];
            if (so != kNoSlot) {
                const uint32_t uoff = I.doff[u];
                conf[uoff + so] = (ConfT)((int)conf[uoff + so] - 1);
            }
        }
        if (lane == 0) {
            ws.S[v] = 0;
            ws.cs[v] = kNoSlot;
        }
        ucnt[C_REPAIRS]++;
        PLSE_WAVE_SYNC();
    }
    snapshot(I, ws.S, out);
    PLSE_WAVE_SYNC();
}

}  // namespace

template <typename ConfT>
__global__ __launch_bounds__(256) void plits_kernel(const PlitsArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    const int wv = (int)(threadIdx.x >> 6);
    const int ind = (int)blockIdx.x * (int)(blockDim.x >> 6) + wv;
    if (ind >= a.p) return;
    int gen = a.gen_fixed;
    if (gen == 0) {
        if (a.ctl->stop) return;
        gen = a.ctl->gen;
    }
    uint8_t *base = lds + (size_t)wv * a.lds_per_wave;
    WaveState ws;
    ws.S = base;
    ws.cs = base + a.off_cs;
    ws.bm = reinterpret_cast<uint32_t *>(base + a.off_bm);
    ws.scr = base + a.off_scr;
    const DevInstance &I = a.I;
    ConfT *conf = reinterpret_cast<ConfT *>(a.conf) + (size_t)ind * I.nd;
    uint32_t *tabu = a.tabu + (size_t)ind * (I.nd + I.nv);
    const uint8_t *src = a.S_in + (size_t)ind * I.stride;
    uint8_t *out = a.S_out + (size_t)ind * I.stride;

    uint64_t ucnt[kCounters];
#pragma unroll
    for (int q = 0; q < kCounters; ++q) ucnt[q] = 0;
    uint32_t lane_cands = 0, lane_nupd = 0;
    Scal sc;
    // phase 1 from the offspring, phase 2 from phase 1's best (both write their
    // best into `out`)
    run_phase<ConfT>(a, 1, a.P.depth1, (uint32_t)ind, (uint32_t)gen, src, out, conf, tabu, ws, sc,
                     ucnt, lane_cands, lane_nupd);
    run_phase<ConfT>(a, 2, a.P.depth2, (uint32_t)ind, (uint32_t)gen, out, out, conf, tabu, ws, sc,
                     ucnt, lane_cands, lane_nupd);
    int32_t f_final = sc.fbest;
    if (sc.cbest > 0) {
        repair<ConfT>(a, out, conf, ws, sc, ucnt);
        f_final = sc.f + (int32_t)ucnt[C_REPAIRS];
    }
    ucnt[C_CANDS] = wave_sum_u64(lane_cands);
    ucnt[C_NUPD] = wave_sum_u64(lane_nupd);
    const int lane = lane_id();
    if (lane < kCounters) {
        uint64_t v = 0;
#pragma unroll
        for (int q = 0; q < kCounters; ++q)
            if (q == lane) v = ucnt[q];
        a.cnt_out[(size_t)ind * kCounters + lane] = v;
    }
    if (lane == 0) a.f_out[ind] = f_final;
}

hipError_t launch_plits(const PlitsArgs &a, int conf_bytes, int waves_per_block,
                        hipStream_t stream) {
    const int blocks = (a.p + waves_per_block - 1) / waves_per_block;
    const size_t lds = (size_t)a.lds_per_wave * waves_per_block;
    if (conf_bytes == 1)
        hipLaunchKernelGGL(plits_kernel<uint8_t>, dim3(blocks), dim3(64 * waves_per_block), lds,
                           stream, a);
    else
        hipLaunchKernelGGL(plits_kernel<int16_t>, dim3(blocks), dim3(64 * waves_per_block), lds,
                           stream, a);
    return hipGetLastError();
}

hipError_t plits_set_lds_limit(int bytes) {
    hipError_t e = set_dynamic_lds_limit((const void *)plits_kernel<uint8_t>, bytes);
    if (e != hipSuccess) return e;
    return set_dynamic_lds_limit((const void *)plits_kernel<int16_t>, bytes);
}

}  // namespace plse

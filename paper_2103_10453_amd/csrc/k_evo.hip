// k_evo.hip -- the per-generation kernels around the tabu search on gfx950:
// best-solution saving, Hamming distances (Eq. 8) as bit-sliced tiles, the
// population update (Alg. 4), nearest-neighbour parent matching
// (Section 3.5.1) and the AUX crossover (Alg. 5, Eq. 9), plus the small
// control kernels of the generation graph.
#include "device_common.h"
#include "kernels.h"

namespace plse {

// ---------------------------------------------------------------------------
// control
// ---------------------------------------------------------------------------
__global__ void ctl_reset_kernel(const ArgList L) {
    Ctl *ctl = static_cast<Ctl *>(const_cast<void *>(L.p[blockIdx.y]));
    if (threadIdx.x == 0) {
        ctl->gen = 0;
        ctl->stop = 0;
        ctl->fstar = INT32_MAX;
        ctl->best_gen = 0;
        ctl->gens_run = 0;
        ctl->stop_reason = 0;
        ctl->iters = 0;
    }
}

__global__ void gen_begin_kernel(const ArgList L) {
    Ctl *ctl = static_cast<Ctl *>(const_cast<void *>(L.p[blockIdx.y]));
    if (threadIdx.x == 0 && !ctl->stop) ctl->gen += 1;
}

// Fresh population bookkeeping: uid = slot, empty partner history, and the
// first offspring population is the initial population itself (Alg. 2).
__global__ void pop_setup_kernel(const ArgList L) {
    const PopSetupArgs a = arg_of<PopSetupArgs>(L);
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (size_t)a.p) {
        a.uid[i] = i;
        a.hc[i] = 0;
    }
    const size_t nq = (size_t)a.p * (a.stride >> 4);
    for (size_t q = i; q < nq; q += (size_t)gridDim.x * blockDim.x)
        reinterpret_cast<uint4 *>(a.S_off)[q] = reinterpret_cast<const uint4 *>(a.S)[q];
}

// ---------------------------------------------------------------------------
// best-solution saving (Alg. 2): argmin f over the improved offspring, ties to
// the lowest slot; S* replaced only on strict improvement.  Also sums the
// per-individual counters of the generation and sets the bound stop flag.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(1024) void best_kernel(const ArgList L) {
    const BestArgs a = arg_of<BestArgs>(L);
    if (a.ctl->stop) return;
    const int g = a.ctl->gen;
    __shared__ uint64_t kmin[16];
    __shared__ uint64_t csum[16][kCounters];
    __shared__ int improved;
    const int tid = (int)threadIdx.x, lane = tid & 63, wv = tid >> 6;
    uint64_t key = ~0ull;
    uint64_t c[kCounters];
#pragma unroll
    for (int q = 0; q < kCounters; ++q) c[q] = 0;
    for (int i = tid; i < a.p; i += blockDim.x) {
        const uint64_t k = ((uint64_t)(uint32_t)a.f_new[i] << 32) | (uint32_t)i;
        key = k < key ? k : key;
#pragma unroll
        for (int q = 0; q < kCounters; ++q) c[q] += a.cnt[(size_t)i * kCounters + q];
    }
    key = wave_min_u64(key);
#pragma unroll
    for (int q = 0; q < kCounters; ++q) c[q] = wave_sum_u64(c[q]);
    if (lane == 0) {
        kmin[wv] = key;
#pragma unroll
        for (int q = 0; q < kCounters; ++q) csum[wv][q] = c[q];
    }
    __syncthreads();
    if (tid == 0) {
        uint64_t k = ~0ull;
        uint64_t s[kCounters] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            k = kmin[w] < k ? kmin[w] : k;
            for (int q = 0; q < kCounters; ++q) s[q] += csum[w][q];
        }
        const int32_t fb = (int32_t)(k >> 32);
        improved = 0;
        if (fb < a.ctl->fstar) {
            a.ctl->fstar = fb;
            a.ctl->best_gen = g;
            improved = 1 + (int)(uint32_t)k;  // slot + 1
        }
        GenStat &gs = a.stats[g - 1];
        gs.best_f = a.ctl->fstar;
        for (int q = 0; q < kCounters; ++q) gs.cnt[q] = s[q];
        a.ctl->gens_run = g;
        a.ctl->iters += s[0];
        if (a.stop_at_ub && a.nsq_minus_l - a.ctl->fstar == a.ub) {
            a.ctl->stop = 1;
            a.ctl->stop_reason = 1;
        } else if (a.max_iters > 0 && a.ctl->iters >= (uint64_t)a.max_iters) {
            // iteration budget (Section 4.3), known at generation ends only
            a.ctl->stop = 1;
            a.ctl->stop_reason = 2;
        }
    }
    __syncthreads();
    if (improved) {
        const uint8_t *src = a.S_new + (size_t)(improved - 1) * a.stride;
        for (int q = tid; q < (a.stride >> 4); q += blockDim.x)
            reinterpret_cast<uint4 *>(a.Sstar)[q] = reinterpret_cast<const uint4 *>(src)[q];
    }
}

// ---------------------------------------------------------------------------
// Hamming distances (Eq. 8), bit-sliced.  pack: colour bit b of vertices
// 32w..32w+31 of row x -> planes[(x*W + w)*B + b].  A pair differs at v iff
// some plane differs, so D = sum_w popcount(OR_b (a_b XOR c_b)).
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void pack_kernel(const ArgList L) {
    const PackArgs a = arg_of<PackArgs>(L);
    if (a.ctl && a.ctl->stop) return;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)a.m * a.W) return;
    const int x = a.row0 + (int)(t / a.W), w = (int)(t % a.W);
    const uint8_t *row = a.S + (size_t)x * a.stride;
    uint32_t pl[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int v0 = w * 32;
    const int vend = min(a.nv, v0 + 32);
    for (int v = v0; v < vend; ++v) {
        const uint32_t s = row[v];
#pragma unroll
        for (int b = 0; b < 8; ++b) pl[b] |= ((s >> b) & 1u) << (v - v0);
    }
    uint32_t *dst = a.planes + ((size_t)x * a.W + w) * a.B;
    for (int b = 0; b < a.B; ++b) dst[b] = pl[b];
}

constexpr int kTile = kDistTile;  // rows and columns per distance tile
constexpr int kCW = 8;      // words of 32 vertices staged per step


// One 64x64 tile (I <= J) per 256-thread workgroup; each thread owns a 4x4
// block of pairs (rows ty+16i, columns tx+16j).  The output tile reuses the
// operand LDS, so more workgroups fit per CU.  Both D[I][J] and its mirror
// are written through that LDS tile so that stores are row-contiguous.
template <int B>
__global__ __launch_bounds__(256) void dist_kernel(const ArgList L) {
    const DistArgs a = arg_of<DistArgs>(L);
    if (a.ctl && a.ctl->stop) return;
    // even pitch with 64-bit reads: 16 rows at a pitch of kCW*B + 2 words
    // (50 for B = 6) start in distinct even banks, so the bank pairs of a
    // 64-bit read never collide; plane pairs stay 8-byte aligned
    constexpr int PITCH = (B % 2 == 0) ? kCW * B + 2 : kCW * B + 1;
    constexpr int OPW = 2 * kTile * PITCH;             // operand words
    constexpr int DTW = kTile * (kTile + 2) / 2;       // output tile words
    __shared__ uint32_t AB[OPW > DTW ? OPW : DTW];
    uint32_t *As = AB, *Bs = AB + kTile * PITCH;
    int16_t(*Dt)[kTile + 2] = reinterpret_cast<int16_t(*)[kTile + 2]>(AB);
    // triangular tile index -> (I, J), I <= J
    const long t = (long)blockIdx.x + a.tile0;
    long J = (long)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((J + 1) * (J + 2) / 2 <= t) ++J;
    while (J * (J + 1) / 2 > t) --J;
    const long I = t - J * (J + 1) / 2;
    const int r0 = (int)I * kTile, c0 = (int)J * kTile;
    const int tid = (int)threadIdx.x, tx = tid & 15, ty = tid >> 4;
    uint32_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0u;

    for (int w0 = 0; w0 < a.W; w0 += kCW) {
        const int nw = min(kCW, a.W - w0);
        // stage kTile rows x nw words x B planes for both sides
        if constexpr (B % 2 == 0) {
            // plane pairs: 8-byte global loads and LDS stores (rows of B
            // words per vertex word keep pairs 8-byte aligned on both sides)
            constexpr int HP = kCW * B / 2;  // pairs per staged row
            for (int q = tid; q < kTile * HP; q += 256) {
                const int row = q / HP, rem = 2 * (q % HP);
                const int wc = rem / B;
                u32x2 va{0u, 0u}, vb{0u, 0u};
                if (wc < nw) {
                    const int ra = r0 + row, rb = c0 + row;
                    if (ra < a.m)
                        va = *gptr(reinterpret_cast<const u32x2 *>(
                            a.planes + ((size_t)ra * a.W + w0) * B + rem));
                    if (rb < a.m)
                        vb = *gptr(reinterpret_cast<const u32x2 *>(
                            a.planes + ((size_t)rb * a.W + w0) * B + rem));
                }
                *reinterpret_cast<u32x2 *>(As + row * PITCH + rem) = va;
                *reinterpret_cast<u32x2 *>(Bs + row * PITCH + rem) = vb;
            }
        } else {
            for (int q = tid; q < kTile * kCW * B; q += 256) {
                const int row = q / (kCW * B), rem = q % (kCW * B);
                const int wc = rem / B;
                uint32_t va = 0u, vb = 0u;
                if (wc < nw) {
                    const int ra = r0 + row, rb = c0 + row;
                    if (ra < a.m) va = *gptr(a.planes + ((size_t)ra * a.W + w0) * B + rem);
                    if (rb < a.m) vb = *gptr(a.planes + ((size_t)rb * a.W + w0) * B + rem);
                }
                As[row * PITCH + rem] = va;
                Bs[row * PITCH + rem] = vb;
            }
        }
        __syncthreads();
#pragma unroll 1
        for (int wc = 0; wc < nw; ++wc) {
            uint32_t ra[4][B], rb[4][B];
            if constexpr (B % 2 == 0) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int b = 0; b < B; b += 2) {
                        const u32x2 x = *reinterpret_cast<const u32x2 *>(
                            As + (ty + 16 * i) * PITCH + wc * B + b);
                        const u32x2 y = *reinterpret_cast<const u32x2 *>(
                            Bs + (tx + 16 * i) * PITCH + wc * B + b);
                        ra[i][b] = x.x;
                        ra[i][b + 1] = x.y;
                        rb[i][b] = y.x;
                        rb[i][b + 1] = y.y;
                    }
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        ra[i][b] = As[(ty + 16 * i) * PITCH + wc * B + b];
                        rb[i][b] = Bs[(tx + 16 * i) * PITCH + wc * B + b];
                    }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    // OR over planes of the XOR: one 3-input op per plane
                    // (v_bitop3 with table 0xBE = (s0 ^ s1) | s2)
                    uint32_t x = ra[i][0] ^ rb[j][0];
#pragma unroll
                    for (int b = 1; b < B; ++b)
                        x = __builtin_amdgcn_bitop3_b32(ra[i][b], rb[j][b], x, 0xBE);
                    acc[i][j] += (uint32_t)__popc(x);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) Dt[ty + 16 * i][tx + 16 * j] = (int16_t)acc[i][j];
    __syncthreads();
    // rows of the tile: D[r0 + row][c0 .. c0+63]
    for (int q = tid; q < kTile * kTile; q += 256) {
        const int row = q >> 6, col = q & 63;
        const int gr = r0 + row, gc = c0 + col;
        if (gr < a.m && gc < a.m) *gptr(a.D + (size_t)gr * a.ld + gc) = Dt[row][col];
    }
    if (I != J) {
        for (int q = tid; q < kTile * kTile; q += 256) {
            const int row = q >> 6, col = q & 63;  // mirror: D[c0 + row][r0 + col]
            const int gr = c0 + row, gc = r0 + col;
            if (gr < a.m && gc < a.m) *gptr(a.D + (size_t)gr * a.ld + gc) = Dt[col][row];
        }
    }
}


// ---------------------------------------------------------------------------
// Population update (Alg. 4)
// ---------------------------------------------------------------------------
// close lists: for candidate x, the candidates y != x with spacing*D(x,y) <= |V|
// (those x excludes once accepted); deg[x] counts them, adj keeps the first kAdj.

__global__ __launch_bounds__(256) void close_kernel(const ArgList L) {
    const CloseArgs a = arg_of<CloseArgs>(L);
    if (a.ctl && a.ctl->stop) return;
    const int x = (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (x >= a.m) return;
    const int lane = lane_id();
    const int16_t *row = a.D + (size_t)x * a.ld;
    uint32_t cnt = 0;
    if ((a.ld & 7) == 0 && (a.m & 7) == 0) {
        // eight distances per lane and load (16-byte rows of D), close list
        // still in ascending order: lanes in order, then the lane's eight
        for (int y0 = 0; y0 < a.m; y0 += 512) {
            const int yb = y0 + lane * 8;
            uint32_t fl = 0u;
            if (yb < a.m) {
                const u32x4 q = gload4(reinterpret_cast<const u32x4 *>(row + yb));
                const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int16_t d = (int16_t)((w[t >> 1] >> (16 * (t & 1))) & 0xFFFFu);
                    const bool cl = (yb + t != x) && (a.spacing * (int64_t)d <= (int64_t)a.nv);
                    fl |= (uint32_t)cl << t;
                }
            }
            uint32_t total;
            uint32_t pos = cnt + wave_excl_scan_dpp((uint32_t)__popc(fl), &total);
            while (fl) {
                const int t = __ffs(fl) - 1;
                fl &= fl - 1u;
                if (pos < (uint32_t)kAdj) *gptr(a.adj + (size_t)x * kAdj + pos) = (uint16_t)(yb + t);
                ++pos;
            }
            cnt += total;
        }
        if (lane == 0) *gptr(a.deg + x) = (int32_t)cnt;
        return;
    }
    for (int y0 = 0; y0 < a.m; y0 += 64) {
        const int y = y0 + lane;
        const bool cl = (y < a.m) && (y != x) && (a.spacing * (int64_t)row[y] <= (int64_t)a.nv);
        const uint64_t msk = ballot(cl);
        const uint32_t pos = cnt + rank_below(msk);
        if (cl && pos < (uint32_t)kAdj) a.adj[(size_t)x * kAdj + pos] = (uint16_t)y;
        cnt += (uint32_t)__popcll(msk);
    }
    if (lane == 0) a.deg[x] = (int32_t)cnt;
}


// One workgroup: keys (f, SELECT draw, index) sorted by a bitonic network,
// then wave 0 scans them in order.  A candidate is accepted iff the population
// is not full and no accepted candidate is close to it; the blocked set (the
// union of the close lists of accepted candidates) lives in an LDS bitmap.
// Lanes take 64 candidates at a time: the candidates up to the first
// unblocked one with a non-empty close list are decided together.
// Selection keys of P^all: f << 48 | SELECT draw << 16 | index (the order of
// Alg. 4: e, then a random key, then the index), ~0 beyond m.
__device__ __forceinline__ void select_keys(const SelectArgs &a, uint32_t gen, int q,
                                            uint64_t *K) {
    const int x0 = q * 4;
    U4 w{0, 0, 0, 0};
    if (x0 < a.m) w = draw(a.seed_lo, a.seed_hi, 0u, gen, TAG_SELECT, (uint32_t)q);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int x = x0 + t;
        K[x] = (x < a.m) ? (((uint64_t)(uint32_t)a.f_all[x] << 48) |
                            ((uint64_t)word_of(w, t) << 16) | (uint32_t)x)
                         : ~0ull;
    }
}

__device__ __forceinline__ bool select_gen(const SelectArgs &a, uint32_t *gen) {
    int g = a.gen_fixed;
    if (g == 0) {
        if (a.ctl->stop) return false;
        g = a.ctl->gen;
    }
    *gen = (uint32_t)g;
    return true;
}

// Key sort for populations whose keys exceed LDS: a bitonic network over the
// global key array, tile-local stages (partner distance < kSortTile) in LDS.
constexpr int kSortTile = 4096;

__global__ __launch_bounds__(256) void select_keys_kernel(const ArgList L) {
    const SelectArgs a = arg_of<SelectArgs>(L);
    uint32_t gen;
    if (!select_gen(a, &gen)) return;
    const int q = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q < (a.pow2 >> 2)) select_keys(a, gen, q, a.keys_g);
}

// Pair i of a bitonic step with partner distance j: lower index.
__device__ __forceinline__ int bitonic_lo(int i, int j) { return ((i & ~(j - 1)) << 1) | (i & (j - 1)); }

__global__ __launch_bounds__(1024) void sort_tile_kernel(const ArgList L, int k_lo, int k_hi) {
    __shared__ uint64_t t[kSortTile];
    const SelectArgs a = arg_of<SelectArgs>(L);
    uint32_t gen;
    if (!select_gen(a, &gen)) return;
    const int base = (int)blockIdx.x * kSortTile;
    for (int q = (int)threadIdx.x; q < kSortTile; q += (int)blockDim.x) t[q] = a.keys_g[base + q];
    __syncthreads();
    for (int k = k_lo; k <= k_hi; k <<= 1) {
        for (int j = min(k >> 1, kSortTile >> 1); j > 0; j >>= 1) {
            for (int i = (int)threadIdx.x; i < (kSortTile >> 1); i += (int)blockDim.x) {
                const int lo = bitonic_lo(i, j), hi = lo + j;
                const bool up = ((base + lo) & k) == 0;
                const uint64_t x = t[lo], y = t[hi];
                if ((x > y) == up) {
                    t[lo] = y;
                    t[hi] = x;
                }
            }
            __syncthreads();
        }
    }
    for (int q = (int)threadIdx.x; q < kSortTile; q += (int)blockDim.x) a.keys_g[base + q] = t[q];
}

__global__ __launch_bounds__(256) void sort_global_kernel(const ArgList L, int k, int j) {
    const SelectArgs a = arg_of<SelectArgs>(L);
    uint32_t gen;
    if (!select_gen(a, &gen)) return;
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= (a.pow2 >> 1)) return;
    const int lo = bitonic_lo(i, j), hi = lo + j;
    const bool up = (lo & k) == 0;
    uint64_t *K = a.keys_g;
    const uint64_t x = K[lo], y = K[hi];
    if ((x > y) == up) {
        K[lo] = y;
        K[hi] = x;
    }
}

__global__ __launch_bounds__(1024) void select_kernel(const ArgList L) {
    extern __shared__ __align__(16) uint8_t lds[];
    const SelectArgs a = arg_of<SelectArgs>(L);
    int gen = a.gen_fixed;
    if (gen == 0) {
        if (a.ctl->stop) return;
        gen = a.ctl->gen;
    }
    const int tid = (int)threadIdx.x, nthr = (int)blockDim.x;
    const int m = a.m, P2 = a.pow2;
    uint32_t *blocked = reinterpret_cast<uint32_t *>(lds);          // [(m+31)/32]
    const int nbw = (m + 31) / 32;
    // keys in LDS: generated and sorted here; else already sorted in global
    // memory by select_keys_kernel / sort_*_kernel
    const int off_keys = (nbw * 4 + 15) & ~15;
    uint64_t *K = a.keys_in_lds ? reinterpret_cast<uint64_t *>(lds + off_keys) : a.keys_g;
    // close lists of the 64 candidates being scanned, staged per block, and
    // each candidate's lane in the block being scanned (0xFF: not in it)
    uint16_t *adjs = reinterpret_cast<uint16_t *>(lds + off_keys + (a.keys_in_lds ? P2 * 8 : 0));
    uint8_t *inb = reinterpret_cast<uint8_t *>(adjs + 64 * kAdj);
    if (a.keys_in_lds)
        for (int q = tid; q < (P2 >> 2); q += nthr) select_keys(a, (uint32_t)gen, q, K);
    for (int q = tid; q < nbw; q += nthr) blocked[q] = 0u;
    for (int q = tid; q < m; q += nthr) *gptr(a.pos + q) = -1;
    for (int q = tid; q < m; q += nthr) inb[q] = 0xFF;
    __syncthreads();
    for (int k = 2; k <= (a.keys_in_lds ? P2 : 1); k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < P2; i += nthr) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const uint64_t x = K[i], y = K[ixj];
                    const bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        K[i] = y;
                        K[ixj] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (tid >= 64) return;
    const int lane = tid;
    int na = 0, nr = 0;
    bool full = false;
    // Loads run one block ahead of the decisions: while a block is decided,
    // the next block's candidates, degrees and close lists (all kAdj entries,
    // whatever the degree) and the keys of the block after it are in flight.
    auto key_at = [&](int r) -> uint64_t {
        return r < m ? (a.keys_in_lds ? K[r] : *gptr(a.keys_g + r)) : 0ull;
    };
    constexpr int kAdjV = kAdj / 8;  // 16-byte vectors per close list
    u32x4 an[kAdjV];
    int xn = (int)(key_at(lane) & 0xFFFFull);
    int dn = lane < m ? *gptr(a.deg + xn) : 0;
#pragma unroll
    for (int q = 0; q < kAdjV; ++q)
        an[q] = gload4(reinterpret_cast<const u32x4 *>(a.adj + (size_t)xn * kAdj) + q);
    uint64_t krn = key_at(64 + lane);
    for (int base = 0; base < m && !full; base += 64) {
        const int r = base + lane;
        const bool valid = r < m;
        const int x = xn, d = dn;
        if (d > 0 && d <= kAdj) {
            u32x4 *dst = reinterpret_cast<u32x4 *>(adjs + lane * kAdj);
#pragma unroll
            for (int q = 0; q < kAdjV; ++q) dst[q] = an[q];
        }
        xn = (int)(krn & 0xFFFFull);
        dn = base + 64 + lane < m ? *gptr(a.deg + xn) : 0;
#pragma unroll
        for (int q = 0; q < kAdjV; ++q)
            an[q] = gload4(reinterpret_cast<const u32x4 *>(a.adj + (size_t)xn * kAdj) + q);
        krn = key_at(base + 128 + lane);
        PLSE_WAVE_SYNC();
        if (ballot(valid && d > kAdj) == 0) {
            // every close list is complete: decide the block in scan order on
            // 64-bit masks.  mk: the later candidates of this block that this
            // one's close list holds; bl: the candidates blocked so far.
            if (valid) inb[x] = (uint8_t)lane;
            PLSE_WAVE_SYNC();
            uint64_t mk = 0;
            for (int q0 = 0; q0 < d; q0 += 8) {
                // eight entries per 16-byte read, their lanes read together
                const u32x4 e = reinterpret_cast<const u32x4 *>(adjs + lane * kAdj)[q0 >> 3];
                const uint32_t ew[4] = {e.x, e.y, e.z, e.w};
                uint32_t js[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    // entries past d are not part of the list: clamp their index
                    const uint32_t y = (ew[t >> 1] >> (16 * (t & 1))) & 0xFFFFu;
                    js[t] = inb[min(y, (uint32_t)(m - 1))];
                }
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    if (q0 + t < d && js[t] != 0xFFu && (int)js[t] > lane) mk |= 1ull << js[t];
            }
            PLSE_WAVE_SYNC();
            if (valid) inb[x] = 0xFF;
            uint64_t bl = ballot(valid && ((blocked[x >> 5] >> (x & 31)) & 1u));
            const int nvalid = (int)__popcll(ballot(valid));
            uint64_t accm = 0, rejm = 0;
            int room = a.p - na;
            for (int i = 0; i < nvalid; ++i) {
                if ((bl >> i) & 1ull) {
                    rejm |= 1ull << i;
                    continue;
                }
                accm |= 1ull << i;
                const uint32_t lo = readlane_u32((uint32_t)mk, i);
                const uint32_t hi = readlane_u32((uint32_t)(mk >> 32), i);
                bl |= ((uint64_t)hi << 32) | lo;
                if (--room == 0) {
                    full = true;
                    break;
                }
            }
            const bool am = (accm >> lane) & 1ull, rm = (rejm >> lane) & 1ull;
            if (am) *gptr(a.acc + na + (int)rank_below(accm)) = x;
            if (rm) *gptr(a.rej + nr + (int)rank_below(rejm)) = x;
            na += (int)__popcll(accm);
            nr += (int)__popcll(rejm);
            // accepted candidates block their close lists for later blocks
            if (am)
                for (int q = 0; q < d; ++q) {
                    const int y = adjs[lane * kAdj + q];
                    atomicOr(&blocked[y >> 5], 1u << (y & 31));
                }
            PLSE_WAVE_SYNC();
            continue;
        }
        // a close list longer than kAdj in the block: step from one
        // unblocked candidate with a non-empty close list to the next
        int pos = 0;
        while (pos < 64) {
            const bool blk = valid && ((blocked[x >> 5] >> (x & 31)) & 1u);
            const bool act = valid && lane >= pos;
            const uint64_t dep = ballot(act && !blk && d > 0);
            const int L = dep ? (__ffsll((unsigned long long)dep) - 1) : 64;
            const bool inr = act && lane < L;
            const uint64_t accm = ballot(inr && !blk), rejm = ballot(inr && blk);
            const int room = a.p - na;
            const uint32_t ra = rank_below(accm);
            if (inr && !blk && (int)ra < room) *gptr(a.acc + na + (int)ra) = x;
            const uint32_t rr = rank_below(rejm);
            if (inr && blk) *gptr(a.rej + nr + (int)rr) = x;
            const int nacc = (int)__popcll(accm);
            na += nacc < room ? nacc : room;
            nr += (int)__popcll(rejm);
            if (na >= a.p) {
                full = true;
                break;
            }
            if (L == 64) break;
            const int xL = (int)shfl_u32((uint32_t)x, L), dL = (int)shfl_u32((uint32_t)d, L);
            if (lane == 0) *gptr(a.acc + na) = xL;
            ++na;
            if (na >= a.p) {
                full = true;
                break;
            }
            if (dL <= kAdj) {
                if (lane < dL) {
                    const int y = adjs[L * kAdj + lane];
                    atomicOr(&blocked[y >> 5], 1u << (y & 31));
                }
            } else {
                const int16_t *row = a.D + (size_t)xL * a.ld;
                for (int y = lane; y < m; y += 64)
                    if (y != xL && a.spacing * (int64_t)*gptr(row + y) <= (int64_t)a.nv)
                        atomicOr(&blocked[y >> 5], 1u << (y & 31));
            }
            PLSE_WAVE_SYNC();
            pos = L + 1;
        }
    }
    // fill rule: rejected candidates in scan order complete a short population
    PLSE_WAVE_SYNC();
    for (int t = lane; t < a.p - na; t += 64) *gptr(a.acc + na + t) = *gptr(a.rej + t);
}

size_t select_lds_bytes(int m, int pow2, bool keys_in_lds) {
    const size_t b = ((size_t)((m + 31) / 32) * 4 + 15) & ~(size_t)15;
    return b + (keys_in_lds ? (size_t)pow2 * 8 : 0) + (size_t)64 * kAdj * 2 +
           (((size_t)m + 15) & ~(size_t)15);
}



// New population P_{t+1} = accepted candidates in acceptance order: rows,
// f, uid ((gen << 32) | slot for members of P'), partner history (empty for
// members of P').  Written to the tmp arrays, then copied back.

__global__ __launch_bounds__(256) void gather_kernel(const ArgList L) {
    const GatherArgs a = arg_of<GatherArgs>(L);
    if (a.ctl->stop) return;
    const int r = (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (r >= a.p) return;
    const int lane = lane_id();
    const int x = min(max(a.acc[r], 0), 2 * a.p - 1);
    const uint4 *src = reinterpret_cast<const uint4 *>(a.S_all + (size_t)x * a.stride);
    uint4 *dst = reinterpret_cast<uint4 *>(a.S_tmp + (size_t)r * a.stride);
    for (int q = lane; q < (a.stride >> 4); q += 64) dst[q] = src[q];
    const bool old = x < a.p;
    if (lane == 0) {
        a.f_tmp[r] = a.f_all[x];
        a.uid_tmp[r] = old ? a.uid[x] : (((uint64_t)(uint32_t)a.ctl->gen << 32) | (uint32_t)(x - a.p));
        a.hc_tmp[r] = old ? a.hc[x] : 0;
        *gptr(a.pos + x) = r;
    }
    if (old) a.hist_tmp[(size_t)r * kHist + lane] = a.hist[(size_t)x * kHist + lane];
}

__global__ __launch_bounds__(256) void copyback_kernel(const ArgList L) {
    const GatherArgs a = arg_of<GatherArgs>(L);
    if (a.ctl->stop) return;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t nq = (size_t)a.p * (a.stride >> 4);
    uint4 *S = reinterpret_cast<uint4 *>(const_cast<uint8_t *>(a.S_all));
    for (size_t q = t; q < nq; q += (size_t)gridDim.x * blockDim.x)
        S[q] = reinterpret_cast<const uint4 *>(a.S_tmp)[q];
    uint64_t *hist = const_cast<uint64_t *>(a.hist);
    for (size_t q = t; q < (size_t)a.p * kHist; q += (size_t)gridDim.x * blockDim.x)
        hist[q] = a.hist_tmp[q];
    if (t < (size_t)a.p) {
        const_cast<int32_t *>(a.f_all)[t] = a.f_tmp[t];
        const_cast<uint64_t *>(a.uid)[t] = a.uid_tmp[t];
        const_cast<int32_t *>(a.hc)[t] = a.hc_tmp[t];
    }
}


// ---------------------------------------------------------------------------
// Parent matching (Section 3.5.1): nearest neighbour (D, then slot) among the
// individuals not yet crossed with S_i; plain nearest neighbour when all are.
// uid -> slot through an open-addressing table rebuilt every generation.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t hash_uid(uint64_t u) {
    u ^= u >> 33;
    u *= 0xFF51AFD7ED558CCDull;
    u ^= u >> 33;
    return (uint32_t)u;
}


__global__ void hash_clear_kernel(const ArgList L) {
    const HashArgs a = arg_of<HashArgs>(L);
    if (a.ctl && a.ctl->stop) return;
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    for (int q = t; q < a.hsize; q += gridDim.x * blockDim.x) a.hkeys[q] = ~0ull;
}

__global__ void hash_insert_kernel(const ArgList L) {
    const HashArgs a = arg_of<HashArgs>(L);
    if (a.ctl && a.ctl->stop) return;
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= a.p) return;
    const uint64_t u = a.uid[i];
    uint32_t h = hash_uid(u) & (uint32_t)(a.hsize - 1);
    for (;;) {
        const unsigned long long prev =
            atomicCAS((unsigned long long *)&a.hkeys[h], ~0ull, (unsigned long long)u);
        if (prev == ~0ull || prev == u) {
            a.hvals[h] = i;
            return;
        }
        h = (h + 1) & (uint32_t)(a.hsize - 1);
    }
}


__global__ __launch_bounds__(256) void match_kernel(const ArgList L) {
    extern __shared__ __align__(16) uint8_t lds[];
    const MatchArgs a = arg_of<MatchArgs>(L);
    if (a.ctl && a.ctl->stop) return;
    const int wv = (int)(threadIdx.x >> 6), lane = lane_id();
    const int i = (int)blockIdx.x * 4 + wv;
    const int nbw = (a.p + 31) / 32;
    uint32_t *excl = reinterpret_cast<uint32_t *>(lds) + (size_t)wv * nbw;
    if (i >= a.p) return;
    for (int q = lane; q < nbw; q += 64) excl[q] = 0u;
    PLSE_WAVE_SYNC();
    const int hcount = max(*gptr(a.hc + i), 0);
    const int nh = min(hcount, a.hist_len);
    for (int t = lane; t < nh; t += 64) {
        const uint64_t u = *gptr(a.hist + (size_t)i * kHist + t);
        uint32_t h = hash_uid(u) & (uint32_t)(a.hsize - 1);
        for (;;) {
            const uint64_t k = *gptr(a.hkeys + h);
            if (k == u) {
                const int s = *gptr(a.hvals + h);
                atomicOr(&excl[s >> 5], 1u << (s & 31));
                break;
            }
            if (k == ~0ull) break;
            h = (h + 1) & (uint32_t)(a.hsize - 1);
        }
    }
    PLSE_WAVE_SYNC();
    const int ai = a.idx ? *gptr(a.idx + i) : i;
    const int16_t *row = a.D + (size_t)ai * a.ld;
    uint64_t best = ~0ull;
    if (a.mode == 1) {
        // random matching (Section 5.3): uniform over the other p - 1
        int gen = a.gen_fixed;
        if (gen == 0) gen = a.ctl->gen;
        const U4 w = draw(a.seed_lo, a.seed_hi, (uint32_t)i, (uint32_t)gen, TAG_MATCH, 0u);
        int j = (int)(((uint64_t)w.x * (uint64_t)(uint32_t)(a.p - 1)) >> 32);
        j += (j >= i) ? 1 : 0;
        const int aj = a.idx ? *gptr(a.idx + j) : j;
        best = ((uint64_t)(uint16_t)*gptr(row + aj) << 32) | (uint32_t)j;
    }
    for (int pass = 0; pass < 2 && best == ~0ull; ++pass) {
        // branch-free body, unrolled: several index and distance loads in
        // flight per lane
        uint64_t lb = ~0ull;
        if (a.idx && (a.ld & 7) == 0 && (a.m & 7) == 0) {
            // the row in D order, eight entries per lane and 16-byte loads of
            // D and of pos (which names the individual of each entry, -1 for
            // candidates not selected)
#pragma unroll 2
            for (int x0 = lane * 8; x0 < a.m; x0 += 512) {
                const u32x4 dq = gload4(row + x0);
                const u32x4 pa = gload4(a.pos + x0);
                const u32x4 pb = gload4(a.pos + x0 + 4);
                const uint32_t dw[4] = {dq.x, dq.y, dq.z, dq.w};
                const int32_t js[8] = {(int32_t)pa.x, (int32_t)pa.y, (int32_t)pa.z, (int32_t)pa.w,
                                       (int32_t)pb.x, (int32_t)pb.y, (int32_t)pb.z, (int32_t)pb.w};
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int j = js[t];
                    const uint32_t d = (dw[t >> 1] >> (16 * (t & 1))) & 0xFFFFu;
                    const int jc = j < 0 ? 0 : j;
                    const bool ok = j >= 0 && j != i &&
                                    (pass != 0 || !((excl[jc >> 5] >> (jc & 31)) & 1u));
                    const uint64_t key = ok ? (((uint64_t)d << 32) | (uint32_t)j) : ~0ull;
                    lb = key < lb ? key : lb;
                }
            }
        } else if (a.idx) {
            // the row in D order (coalesced); pos names the individual of
            // each entry, -1 for candidates not selected
#pragma unroll 8
            for (int x = lane; x < a.m; x += 64) {
                const int j = *gptr(a.pos + x);
                const uint32_t d = (uint16_t)*gptr(row + x);
                const int jc = j < 0 ? 0 : j;
                const bool ok = j >= 0 && j != i &&
                                (pass != 0 || !((excl[jc >> 5] >> (jc & 31)) & 1u));
                const uint64_t key = ok ? (((uint64_t)d << 32) | (uint32_t)j) : ~0ull;
                lb = key < lb ? key : lb;
            }
        } else {
#pragma unroll 8
            for (int j = lane; j < a.p; j += 64) {
                const uint32_t d = (uint16_t)*gptr(row + j);
                const bool ok = j != i && (pass != 0 || !((excl[j >> 5] >> (j & 31)) & 1u));
                const uint64_t key = ok ? (((uint64_t)d << 32) | (uint32_t)j) : ~0ull;
                lb = key < lb ? key : lb;
            }
        }
        best = wave_min_u64(lb);
    }
    if (lane == 0) {
        const int j = (int)(uint32_t)best;
        a.partner[i] = j;
        a.dpart[i] = (int32_t)(best >> 32);
        if (a.hist_len > 0) {
            const int pos = hcount % a.hist_len;
            a.hist[(size_t)i * kHist + pos] = a.uid[j];
            int nc = hcount + 1;
            if (nc >= 2 * a.hist_len) nc -= a.hist_len;
            a.hc[i] = nc;
        }
    }
}


// ---------------------------------------------------------------------------
// AUX crossover (Alg. 5): vertex v keeps S_i(v) when its XOVER draw is below
// thr = floor((beta*D - |V|) 2^32 / (beta*D)) (p_ij of Eq. 9 in 2^-32
// units; 0 when beta*D <= |V|), else takes S_j(v).  One wave per child, four
// vertices per lane step (one Philox block).
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void aux_kernel(const ArgList L) {
    const AuxArgs a = arg_of<AuxArgs>(L);
    int gen = a.gen_fixed;
    if (gen == 0) {
        if (a.ctl->stop) return;
        gen = a.ctl->gen;
    }
    const int i = (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (i >= a.p) return;
    const int lane = lane_id();
    int j = a.partner[i];
    if (j < 0 || j >= a.p) j = i;  // out-of-range partner: no crossover
    const uint64_t bd = (uint64_t)a.beta_num * (uint64_t)(uint32_t)a.dpart[i];
    const uint64_t bv = (uint64_t)a.beta_den * (uint64_t)a.nv;
    // UX fixes p_ij at 1/2 (Section 3.5.2); without crossover the offspring
    // copies its first parent (Section 5.2)
    const uint64_t thr = a.mode == 1   ? (1ull << 31)
                         : a.mode == 2 ? (1ull << 32)
                                       : ((bd <= bv) ? 0ull : frac_shift32(bd - bv, bd));
    const uint32_t *si = reinterpret_cast<const uint32_t *>(a.S + (size_t)i * a.stride);
    const uint32_t *sj = reinterpret_cast<const uint32_t *>(a.S + (size_t)j * a.stride);
    uint32_t *so = reinterpret_cast<uint32_t *>(a.S_off + (size_t)i * a.stride);
    const int nq = a.stride >> 2;
    for (int q = lane; q < nq; q += 64) {
        uint32_t out = 0u;
        if (4 * q < a.nv) {
            const U4 w = draw(a.seed_lo, a.seed_hi, (uint32_t)i, (uint32_t)gen, TAG_XOVER,
                              (uint32_t)q);
            const uint32_t x = si[q], y = sj[q];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (4 * q + t < a.nv) {
                    const uint32_t b = ((uint64_t)word_of(w, t) < thr) ? x : y;
                    out |= b & (0xFFu << (8 * t));
                }
            }
        }
        so[q] = out;
    }
}






hipError_t launch_ctl_reset(const ArgList &L, int count, hipStream_t stream) {
    hipLaunchKernelGGL(ctl_reset_kernel, dim3(1, count), dim3(64), 0, stream, L);
    return hipGetLastError();
}

hipError_t launch_gen_begin(const ArgList &L, int count, hipStream_t stream) {
    hipLaunchKernelGGL(gen_begin_kernel, dim3(1, count), dim3(64), 0, stream, L);
    return hipGetLastError();
}

hipError_t launch_pop_setup(const ArgList &L, int count, hipStream_t stream) {
    hipLaunchKernelGGL(pop_setup_kernel, dim3(512, count), dim3(256), 0, stream, L);
    return hipGetLastError();
}

hipError_t launch_best(const ArgList &L, int count, hipStream_t stream) {
    hipLaunchKernelGGL(best_kernel, dim3(1, count), dim3(1024), 0, stream, L);
    return hipGetLastError();
}

hipError_t launch_pack(const ArgList &L, int count, size_t max_threads, hipStream_t stream) {
    // at least one block: an instance without vertices packs nothing
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)std::max<size_t>(1, (max_threads + 255) / 256), count), dim3(256),
                       0, stream, L);
    return hipGetLastError();
}

hipError_t launch_dist(const ArgList &L, int count, long tiles, int B, hipStream_t stream) {
    if (tiles <= 0) return hipSuccess;
    const dim3 grid((unsigned)tiles, count);
    switch (B) {
#define PLSE_DIST_CASE(b) \
    case b: hipLaunchKernelGGL(dist_kernel<b>, grid, dim3(256), 0, stream, L); break;
        PLSE_DIST_CASE(1)
        PLSE_DIST_CASE(2)
        PLSE_DIST_CASE(3)
        PLSE_DIST_CASE(4)
        PLSE_DIST_CASE(5)
        PLSE_DIST_CASE(6)
        PLSE_DIST_CASE(7)
#undef PLSE_DIST_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_close(const ArgList &L, int count, int m, hipStream_t stream) {
    hipLaunchKernelGGL(close_kernel, dim3((m + 3) / 4, count), dim3(256), 0, stream, L);
    return hipGetLastError();
}

hipError_t launch_select(const ArgList &L, int count, size_t lds, int pow2, bool keys_in_lds,
                         hipStream_t stream) {
    if (!keys_in_lds) {
        if (pow2 < kSortTile) return hipErrorInvalidValue;
        hipLaunchKernelGGL(select_keys_kernel, dim3((pow2 / 4 + 255) / 256, count), dim3(256), 0,
                           stream, L);
        const int tiles = pow2 / kSortTile;
        hipLaunchKernelGGL(sort_tile_kernel, dim3(tiles, count), dim3(1024), 0, stream, L, 2,
                           kSortTile);
        for (int k = 2 * kSortTile; k <= pow2; k <<= 1) {
            for (int j = k >> 1; j >= kSortTile; j >>= 1)
                hipLaunchKernelGGL(sort_global_kernel, dim3((pow2 / 2 + 255) / 256, count),
                                   dim3(256), 0, stream, L, k, j);
            hipLaunchKernelGGL(sort_tile_kernel, dim3(tiles, count), dim3(1024), 0, stream, L, k,
                               k);
        }
    }
    hipLaunchKernelGGL(select_kernel, dim3(1, count), dim3(1024), lds, stream, L);
    return hipGetLastError();
}

hipError_t launch_gather(const ArgList &L, int count, int p, hipStream_t stream) {
    hipLaunchKernelGGL(gather_kernel, dim3((p + 3) / 4, count), dim3(256), 0, stream, L);
    hipLaunchKernelGGL(copyback_kernel, dim3(256, count), dim3(256), 0, stream, L);
    return hipGetLastError();
}

hipError_t launch_hash(const ArgList &L, int count, int p, int hsize, hipStream_t stream) {
    hipLaunchKernelGGL(hash_clear_kernel, dim3((hsize + 255) / 256, count), dim3(256), 0, stream,
                       L);
    hipLaunchKernelGGL(hash_insert_kernel, dim3((p + 255) / 256, count), dim3(256), 0, stream, L);
    return hipGetLastError();
}

hipError_t launch_match(const ArgList &L, int count, int p, hipStream_t stream) {
    const size_t lds = (size_t)4 * ((p + 31) / 32) * 4;
    hipLaunchKernelGGL(match_kernel, dim3((p + 3) / 4, count), dim3(256), lds, stream, L);
    return hipGetLastError();
}

hipError_t launch_aux(const ArgList &L, int count, int p, hipStream_t stream) {
    hipLaunchKernelGGL(aux_kernel, dim3((p + 3) / 4, count), dim3(256), 0, stream, L);
    return hipGetLastError();
}

hipError_t evo_set_lds_limit(int bytes) {
    hipError_t e = set_dynamic_lds_limit((const void *)select_kernel, bytes);
    if (e != hipSuccess) return e;
    return set_dynamic_lds_limit((const void *)match_kernel, bytes);
}

}  // namespace plse

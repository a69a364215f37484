// k_init.hip -- initial population (Section 3.2: "initialized at random in
// parallel"), one workgroup per individual.  Reading: a randomised greedy legal
// colouring.  Vertices are visited in the order of their INIT_ORDER draws
// (ties by id): the workgroup sorts the (draw, id) keys in LDS with a bitonic
// network, then one lane walks the order, giving each vertex a uniformly drawn
// colour of D*(v) not used in its row or column so far (128-bit masks).
#include "device_common.h"
#include "kernels.h"

namespace plse {


__global__ __launch_bounds__(256) void init_kernel(const ArgList L) {
    extern __shared__ __align__(16) uint8_t lds[];
    const InitArgs a = arg_of<InitArgs>(L);
    const DevInstance &I = a.I;
    const int ind = (int)blockIdx.x;
    const int tid = (int)threadIdx.x, nthr = (int)blockDim.x;
    const int nv = I.nv, n = I.n, P2 = a.pow2;
    uint64_t *key = reinterpret_cast<uint64_t *>(lds);                  // [P2]
    uint64_t *used = key + P2;                                          // [2n][2]
    uint8_t *S = reinterpret_cast<uint8_t *>(used + 4 * n);              // [stride]
    __shared__ int32_t zeros_part[8];

    // keys (INIT_ORDER draw << 32 | v); padding sorts last
    for (int q = tid; q < (P2 >> 2); q += nthr) {
        const int v0 = q * 4;
        U4 w{0, 0, 0, 0};
        if (v0 < nv) w = draw(a.seed_lo, a.seed_hi, (uint32_t)ind, 0u, TAG_INIT_ORDER, (uint32_t)q);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int v = v0 + t;
            key[v] = (v < nv) ? (((uint64_t)word_of(w, t) << 32) | (uint32_t)v) : ~0ull;
        }
    }
    for (int q = tid; q < 4 * n; q += nthr) used[q] = 0ull;
    for (int q = tid; q < (I.stride >> 2); q += nthr) reinterpret_cast<uint32_t *>(S)[q] = 0u;
    __syncthreads();
    // bitonic sort, ascending
    for (int k = 2; k <= P2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < P2; i += nthr) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const uint64_t x = key[i], y = key[ixj];
                    const bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        key[i] = y;
                        key[ixj] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    // replace the sort draw by the INIT_PICK draw of step t
    for (int t = tid; t < nv; t += nthr) {
        const U4 w = draw(a.seed_lo, a.seed_hi, (uint32_t)ind, 0u, TAG_INIT_PICK, (uint32_t)t);
        key[t] = ((uint64_t)w.x << 32) | (key[t] & 0xFFFFFFFFull);
    }
    __syncthreads();
    if (tid == 0) {
        uint64_t *rowu = used;          // row r: rowu[2r], rowu[2r+1]
        uint64_t *colu = used + 2 * n;  // column c
        for (int t = 0; t < nv; ++t) {
            const uint64_t kt = key[t];
            const int v = (int)(uint32_t)kt;
            const uint32_t pw = (uint32_t)(kt >> 32);
            const uint32_t rc = I.vrc[v];
            const int r = (int)(rc & 0xFFu), c = (int)(rc >> 8);
            const uint64_t *dm = reinterpret_cast<const uint64_t *>(I.vrec) + 4 * v;
            const uint64_t l0 = dm[0] & ~(rowu[2 * r] | colu[2 * c]);
            const uint64_t l1 = dm[1] & ~(rowu[2 * r + 1] | colu[2 * c + 1]);
            const uint32_t c0 = (uint32_t)__popcll(l0), cnt = c0 + (uint32_t)__popcll(l1);
            if (cnt == 0) continue;
            uint32_t idx = scale32(pw, cnt);
            uint64_t wsel = l0;
            int basebit = 0;
            if (idx >= c0) {
                idx -= c0;
                wsel = l1;
                basebit = 64;
            }
            for (uint32_t q = 0; q < idx; ++q) wsel &= wsel - 1ull;
            const int colour = basebit + __ffsll((unsigned long long)wsel) - 1;
            S[v] = (uint8_t)colour;
            const int hw = colour >> 6;
            const uint64_t bit = 1ull << (colour & 63);
            rowu[2 * r + hw] |= bit;
            colu[2 * c + hw] |= bit;
        }
    }
    __syncthreads();
    int zeros = 0;
    for (int v = tid; v < nv; v += nthr) zeros += (S[v] == 0);
    uint8_t *dst = a.S + (size_t)ind * I.stride;
    for (int q = tid; q < (I.stride >> 4); q += nthr)
        reinterpret_cast<uint4 *>(dst)[q] = reinterpret_cast<const uint4 *>(S)[q];
    zeros = (int)wave_sum_u32((uint32_t)zeros);
    if ((tid & 63) == 0) zeros_part[tid >> 6] = zeros;
    __syncthreads();
    if (tid == 0) {
        int z = 0;
        for (int w = 0; w < (nthr >> 6); ++w) z += zeros_part[w];
        a.f[ind] = z;
    }
}

size_t init_lds_bytes(const DevInstance &I, int pow2) {
    return (size_t)pow2 * 8 + (size_t)4 * I.n * 8 + (size_t)I.stride;
}

hipError_t launch_init(const ArgList &L, int count, int p, size_t lds, hipStream_t stream) {
    hipLaunchKernelGGL(init_kernel, dim3(p, count), dim3(256), lds, stream, L);
    return hipGetLastError();
}

}  // namespace plse

namespace plse {
hipError_t init_set_lds_limit(int bytes) {
    return set_dynamic_lds_limit((const void *)init_kernel, bytes);
}
}  // namespace plse

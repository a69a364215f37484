// device_common.h -- gfx950 device primitives of libplse: counter-based random
// draws and wave64 collectives.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plse_internal.h"

namespace plse {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64-bit products mixed into the counter, key advanced by the Weyl
// constants between rounds.  The counter is (instance 0, slot, gen<<8|tag,
// index) and the key is the two halves of the 64-bit seed.
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ U4 draw(uint32_t seed_lo, uint32_t seed_hi, uint32_t slot,
                                   uint32_t gen, uint32_t tag, uint32_t idx) {
    return philox(0u, slot, (gen << 8) | tag, idx, seed_lo, seed_hi);
}

__device__ __forceinline__ uint32_t word_of(const U4 &u, int i) {
    return i == 0 ? u.x : (i == 1 ? u.y : (i == 2 ? u.z : u.w));
}

// MurmurHash3 32-bit finaliser (Appleby): a bijection, used to break ties
// between moves of equal value without collisions.
__host__ __device__ inline uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

// floor(x / d) for x < 2^31 and d >= 1, given m = floor((2^32 - 1) / d):
// the high word of x * m is floor(x / d) or one less.
__host__ __device__ inline uint32_t udiv_by(uint32_t x, uint32_t d, uint32_t m) {
    uint32_t q = (uint32_t)(((uint64_t)x * m) >> 32);
    if (x - q * d >= d) ++q;
    return q;
}

// Aspiration bound on the squeezed move scale e = 4 dc + df (|df| <= 1,
// |V| >= 3), which orders moves as delta = |V| dc + df does.  With
// F* - F = dfg + |V| dcg (|dfg| <= |V|) written as |V| q + r, 0 <= r < |V|,
// delta < F* - F holds for every move with dc < q, for dc = q exactly when
// df < r, and never for dc > q; that is e < 4 q + min(r, 2).
__host__ __device__ inline int32_t squeezed_bound(int32_t dfg, int32_t dcg, int32_t nv) {
    const int32_t q = dcg + (dfg < 0 ? -1 : (dfg < nv ? 0 : 1));
    const int32_t r = dfg < 0 ? dfg + nv : (dfg < nv ? dfg : 0);
    return 4 * q + (r < 2 ? r : 2);
}

// floor(x 2^32 / y) for x < y < 2^47 (the Eq. 9 threshold: x = beta_num D -
// beta_den |V|, y = beta_num D, both below 2^35 for the parameter ranges),
// by two 16-bit steps of long division so no product exceeds 64 bits.
__host__ __device__ inline uint64_t frac_shift32(uint64_t x, uint64_t y) {
    const uint64_t a = x << 16;
    const uint64_t q1 = a / y, r1 = a - q1 * y;
    const uint64_t q0 = (r1 << 16) / y;
    return (q1 << 16) | q0;
}

// floor(w * m / 2^32): uniform integer in [0, m).
__device__ __forceinline__ uint32_t scale32(uint32_t w, uint32_t m) { return __umulhi(w, m); }

// Global-memory views of generic pointers.  Accesses through them compile to
// global_* instructions; flat_* accesses (what a pointer read from an argument
// block would give) are also counted with the LDS operations, so that every
// wait for an LDS result would wait for outstanding memory traffic too.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gptr(const T *p) {
    return (const __attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gptr(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}

// 8- and 16-byte global accesses (clang vector types: HIP's uint2/uint4
// classes only bind to generic-address references).
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ u32x4 gload4(const void *p) {
    return *gptr(reinterpret_cast<const u32x4 *>(p));
}
__device__ __forceinline__ u32x2 gload2(const void *p) {
    return *gptr(reinterpret_cast<const u32x2 *>(p));
}
__device__ __forceinline__ void gstore4(void *p, u32x4 v) { *gptr(reinterpret_cast<u32x4 *>(p)) = v; }

// ---------------------------------------------------------------------------
// wave64 collectives.  All lanes of the wave must be active at the call.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

// Orders this wave's memory operations (LDS and global) for the compiler;
// within one wavefront the hardware already performs them in order.
#define PLSE_WAVE_SYNC()                                         \
    do {                                                         \
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");   \
        __builtin_amdgcn_wave_barrier();                         \
    } while (0)

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ uint32_t rank_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t shfl_u32(uint32_t v, int src) {
    return (uint32_t)__shfl((int)v, src, 64);
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
    const uint32_t lo = shfl_u32((uint32_t)v, src), hi = shfl_u32((uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, 64);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, 64);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const uint64_t o = shfl_xor_u64(v, m);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)v, m, 64);
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += shfl_xor_u64(v, m);
    return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += (uint32_t)__shfl_xor((int)v, m, 64);
    return v;
}

// Exclusive prefix sum over the wave; *total receives the wave sum.
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t *total) {
    const int lane = lane_id();
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = (uint32_t)__shfl_up((int)x, d, 64);
        if (lane >= d) x += o;
    }
    *total = shfl_u32(x, 63);
    return x - v;
}

__device__ __forceinline__ int readfirst(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ---------------------------------------------------------------------------
// DPP forms of the collectives: cross-lane moves inside the VALU instead of
// LDS permutes.  Reduction order: quad swaps, half-row and row mirrors, then
// row broadcasts 15 and 31, after which lane 63 holds the wave result.
// ---------------------------------------------------------------------------
enum : int {
    DPP_QUAD_1032 = 0xB1,     // quad_perm [1,0,3,2]
    DPP_QUAD_2301 = 0x4E,     // quad_perm [2,3,0,1]
    DPP_ROW_SHR1 = 0x111,
    DPP_ROW_SHR2 = 0x112,
    DPP_ROW_SHR4 = 0x114,
    DPP_ROW_SHR8 = 0x118,
    DPP_ROW_MIRROR = 0x140,
    DPP_ROW_HALF_MIRROR = 0x141,
    DPP_ROW_BCAST15 = 0x142,
    DPP_ROW_BCAST31 = 0x143,
};

template <int CTRL, int ROW_MASK = 0xF, bool BOUND_ZERO = false>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROW_MASK, 0xF, BOUND_ZERO);
}

__device__ __forceinline__ uint32_t readlane_u32(uint32_t v, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void dpp_min_step(uint32_t &hi, uint32_t &lo) {
    const uint32_t oh = dpp_u32<CTRL, ROW_MASK>(hi, hi);
    const uint32_t ol = dpp_u32<CTRL, ROW_MASK>(lo, lo);
    const bool take = (oh < hi) || (oh == hi && ol < lo);
    hi = take ? oh : hi;
    lo = take ? ol : lo;
}

// Wave minimum of a 64-bit key, returned uniformly to all lanes.
__device__ __forceinline__ uint64_t wave_min_u64_dpp(uint64_t v) {
    uint32_t hi = (uint32_t)(v >> 32), lo = (uint32_t)v;
    dpp_min_step<DPP_QUAD_1032, 0xF>(hi, lo);
    dpp_min_step<DPP_QUAD_2301, 0xF>(hi, lo);
    dpp_min_step<DPP_ROW_HALF_MIRROR, 0xF>(hi, lo);
    dpp_min_step<DPP_ROW_MIRROR, 0xF>(hi, lo);
    dpp_min_step<DPP_ROW_BCAST15, 0xA>(hi, lo);
    dpp_min_step<DPP_ROW_BCAST31, 0xC>(hi, lo);
    return ((uint64_t)readlane_u32(hi, 63) << 32) | readlane_u32(lo, 63);
}

// Wave minimum (u32), returned uniformly.
__device__ __forceinline__ uint32_t wave_min_u32_dpp(uint32_t x) {
    // rows a broadcast does not reach read the identity 0xFFFFFFFF, which
    // lets the compiler fold each move into the min as a DPP operand
    x = min(x, dpp_u32<DPP_QUAD_1032>(0xFFFFFFFFu, x));
    x = min(x, dpp_u32<DPP_QUAD_2301>(0xFFFFFFFFu, x));
    x = min(x, dpp_u32<DPP_ROW_HALF_MIRROR>(0xFFFFFFFFu, x));
    x = min(x, dpp_u32<DPP_ROW_MIRROR>(0xFFFFFFFFu, x));
    x = min(x, dpp_u32<DPP_ROW_BCAST15, 0xA>(0xFFFFFFFFu, x));
    x = min(x, dpp_u32<DPP_ROW_BCAST31, 0xC>(0xFFFFFFFFu, x));
    return readlane_u32(x, 63);
}

// Wave sum (u32), returned uniformly.
__device__ __forceinline__ uint32_t wave_sum_u32_dpp(uint32_t x) {
    x += dpp_u32<DPP_QUAD_1032>(0u, x);
    x += dpp_u32<DPP_QUAD_2301>(0u, x);
    x += dpp_u32<DPP_ROW_HALF_MIRROR>(0u, x);
    x += dpp_u32<DPP_ROW_MIRROR>(0u, x);
    x += dpp_u32<DPP_ROW_BCAST15, 0xA>(0u, x);
    x += dpp_u32<DPP_ROW_BCAST31, 0xC>(0u, x);
    return readlane_u32(x, 63);
}

// Exclusive prefix sum (u32) over the wave; *total receives the wave sum.
__device__ __forceinline__ uint32_t wave_excl_scan_dpp(uint32_t v, uint32_t *total) {
    uint32_t x = v;
    x += dpp_u32<DPP_ROW_SHR1, 0xF, true>(0u, x);
    x += dpp_u32<DPP_ROW_SHR2, 0xF, true>(0u, x);
    x += dpp_u32<DPP_ROW_SHR4, 0xF, true>(0u, x);
    x += dpp_u32<DPP_ROW_SHR8, 0xF, true>(0u, x);
    x += dpp_u32<DPP_ROW_BCAST15, 0xA>(0u, x);
    x += dpp_u32<DPP_ROW_BCAST31, 0xC>(0u, x);
    *total = readlane_u32(x, 63);
    return x - v;
}

// Allow a kernel the device's per-block LDS minus its own static LDS as
// dynamic shared memory.
inline hipError_t set_dynamic_lds_limit(const void *fn, int device_max) {
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(&attr, fn);
    if (e != hipSuccess) return e;
    const int dyn = device_max - (int)attr.sharedSizeBytes;
    if (dyn <= 0) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
}

}  // namespace plse

// k_measure.hip -- device measurement used to state the LDS roofline of the
// tabu search: sustained LDS read bandwidth of the whole GPU (gfx950).
//
// Every lane reads 16-byte words at consecutive addresses (a wave covers
// 1 KiB per read, each bank once per cycle group), XOR-folding them so no
// read can be dropped; the walk's stride and mask come from the arguments so
// the compiler cannot hoist the reads out of the loop.
#include "device_common.h"

namespace plse {

namespace {
constexpr int kLdsWords = 2048;  // 16-byte words: 32 KiB per block
constexpr int kThreads = 256;
}

__global__ __launch_bounds__(kThreads) void lds_read_kernel(uint32_t iters, uint32_t step,
                                                            uint32_t mask, uint32_t *sink) {
    __shared__ u32x4 buf[kLdsWords];
    const uint32_t t = threadIdx.x;
    for (uint32_t i = t; i < (uint32_t)kLdsWords; i += kThreads)
        buf[i] = u32x4{i, i * 3u + 1u, i * 5u + 2u, i * 7u + 3u};
    __syncthreads();
    u32x4 acc{0u, 0u, 0u, 0u};
    uint32_t idx = t;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) acc ^= buf[(idx + j * kThreads) & mask];
        idx = (idx + step) & mask;
    }
    if ((acc.x ^ acc.y ^ acc.z ^ acc.w) == 0x9E3779B9u) sink[blockIdx.x] = acc.x;
}

// Bytes one launch reads: blocks x threads x iters x 8 reads x 16 bytes.
hipError_t launch_lds_read(int blocks, uint32_t iters, uint32_t *sink, hipStream_t stream,
                           double *bytes) {
    hipLaunchKernelGGL(lds_read_kernel, dim3(blocks), dim3(kThreads), 0, stream, iters,
                       (uint32_t)(8 * kThreads), (uint32_t)(kLdsWords - 1), sink);
    *bytes = (double)blocks * kThreads * iters * 8.0 * 16.0;
    return hipGetLastError();
}

}  // namespace plse

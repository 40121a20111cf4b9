// Yardsticks that the scoring kernels are measured against:
//  * k_copy16 - a plain copy with 16-byte vector loads and stores. It moves a
//    known number of bytes each way, so the hardware traffic counters of a
//    profiled run are calibrated against it.
//  * k_lds_atomic - LDS atomic-add throughput for the four accumulator types a
//    doc-tiled scatter-add can use (uint32, uint64, float, double). The
//    scoring kernels scatter-add one product per posting into an LDS copy of a
//    doc tile; which accumulator type they use is decided by these rates.
#include "gs_internal.h"

namespace gs {

namespace {

__global__ __launch_bounds__(256) void k_copy16(uint4* __restrict__ dst, const uint4* __restrict__ src, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// Every lane issues `iters` no-return atomic adds (iters a multiple of 16) into a
// 64 KiB LDS array, the footprint of one scoring tile. pattern 0: addresses from
// a per-lane linear congruential sequence (scattered, like postings of many
// terms landing in one tile; bank conflicts as they fall); pattern 1: lane l of
// wavefront w adds to word (w * 64 + l + 512 * u) of the array (consecutive words
// across a wavefront). One value per workgroup goes to `sink` so that the adds
// are not removed.
template <typename T>
__global__ __launch_bounds__(512) void k_lds_atomic(int iters, int pattern, T* __restrict__ sink) {
    constexpr int kWords = 65536 / (int)sizeof(T);
    static_assert((kWords & (kWords - 1)) == 0, "power-of-two word count");
    __shared__ T acc[kWords];
    for (int i = threadIdx.x; i < kWords; i += 512) acc[i] = T(0);
    __syncthreads();
    uint32_t h = (uint32_t)(blockIdx.x * 512u + threadIdx.x) * 2654435761u + 0x9E3779B9u;
    const T one = T(1);
    for (int it = 0; it < iters; it += 16) {
        uint32_t a[16];
#pragma unroll
        for (int u = 0; u < 16; u++) {
            h = h * 1664525u + 1013904223u;
            a[u] = pattern == 0 ? (h >> 7) & (uint32_t)(kWords - 1)
                                : (uint32_t)(threadIdx.x + 512 * (u + it)) & (uint32_t)(kWords - 1);
        }
#pragma unroll
        for (int u = 0; u < 16; u++) atomicAdd(&acc[a[u]], one);
    }
    __syncthreads();
    if (threadIdx.x == 0) sink[blockIdx.x] = acc[blockIdx.x & (kWords - 1)];
}

}  // namespace

hipError_t launch_copy16(void* dst, const void* src, int64_t n16, hipStream_t s) {
    if (n16 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy16, dim3(4096), dim3(256), 0, s, (uint4*)dst, (const uint4*)src, n16);
    GS_CHECK_LAUNCH("k_copy16");
    return hipSuccess;
}

hipError_t launch_lds_atomic(int op, int pattern, int workgroups, int iters, void* sink, hipStream_t s) {
    const dim3 grid((unsigned)workgroups), block(512);
    switch (op) {
        case 0: hipLaunchKernelGGL(k_lds_atomic<uint32_t>, grid, block, 0, s, iters, pattern, (uint32_t*)sink); break;
        case 1:
            hipLaunchKernelGGL(k_lds_atomic<unsigned long long>, grid, block, 0, s, iters, pattern,
                               (unsigned long long*)sink);
            break;
        case 2: hipLaunchKernelGGL(k_lds_atomic<float>, grid, block, 0, s, iters, pattern, (float*)sink); break;
        case 3: hipLaunchKernelGGL(k_lds_atomic<double>, grid, block, 0, s, iters, pattern, (double*)sink); break;
        default: return hipErrorInvalidValue;
    }
    GS_CHECK_LAUNCH("k_lds_atomic");
    return hipSuccess;
}

}  // namespace gs

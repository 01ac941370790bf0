// LDS atomic throughput of the device: the denominator of the finder's
// vote-rate roofline (every histogram vote is one LDS atomic add).
//
// Each workgroup (1024 threads, 16 row buffers of 1024 words, 64 KiB) adds 1
// to LDS words for a fixed number of rounds, eight atomics per thread per
// round. Mode 0: lane-consecutive addresses, no return value (conflict-free
// peak). Mode 1: pseudo-random addresses inside the wave's 1024-word row,
// returning the old value (the access pattern of the finder's votes).

#include <hip/hip_runtime.h>

#include "hough_internal.h"

namespace hough {

namespace {

constexpr int kProbeThreads = 1024;
constexpr int kProbeWords = 16 * 1024;
constexpr int kProbeUnroll = 8;

template <int MODE>
__global__ __launch_bounds__(kProbeThreads) void k_lds_atomic(int rounds, uint32_t *sink) {
    __shared__ uint32_t buf[kProbeWords];
    for (int i = threadIdx.x; i < kProbeWords; i += kProbeThreads) buf[i] = 0u;
    __syncthreads();
    const uint32_t row = (threadIdx.x >> 6) << 10;
    uint32_t x = threadIdx.x * 2654435761u + blockIdx.x * 97u;
    uint32_t acc = 0u;
    for (int r = 0; r < rounds; ++r) {
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            if (MODE == 0) {
                atomicAdd(&buf[(threadIdx.x + (uint32_t)u * kProbeThreads) & (kProbeWords - 1)], 1u);
            } else {
                x = x * 1664525u + 1013904223u;
                acc += atomicAdd(&buf[row + (x >> 22)], 1u);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) sink[blockIdx.x] = buf[0] + acc;
}

}  // namespace

hipError_t lds_atomic_rate(int mode, hipStream_t s, int n_cu, double *lane_ops_per_s) {
    const int blocks = 2 * n_cu;
    const int rounds = 4096;
    uint32_t *sink = nullptr;
    hipError_t st = hipMalloc(&sink, sizeof(uint32_t) * (size_t)blocks);
    if (st != hipSuccess) return st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best_ms = 0.f;
    for (int rep = 0; rep < 3 && st == hipSuccess; ++rep) {
        (void)hipEventRecord(e0, s);
        if (mode == 0)
            hipLaunchKernelGGL(k_lds_atomic<0>, dim3(blocks), dim3(kProbeThreads), 0, s, rounds, sink);
        else
            hipLaunchKernelGGL(k_lds_atomic<1>, dim3(blocks), dim3(kProbeThreads), 0, s, rounds, sink);
        st = hipGetLastError();
        (void)hipEventRecord(e1, s);
        if (st == hipSuccess) st = hipEventSynchronize(e1);
        float ms = 0.f;
        if (st == hipSuccess) st = hipEventElapsedTime(&ms, e0, e1);
        if (st == hipSuccess && rep > 0 && (best_ms == 0.f || ms < best_ms)) best_ms = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    if (st != hipSuccess) return st;
    const double ops = (double)blocks * kProbeThreads * (double)rounds * kProbeUnroll;
    *lane_ops_per_s = best_ms > 0.f ? ops / (best_ms * 1e-3) : 0.0;
    return hipSuccess;
}

}  // namespace hough

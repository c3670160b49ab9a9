// Measurement probe, not part of the sampler: the rate at which the GPU
// performs device-scope int32 atomic adds at random addresses.  The degree
// sink of the batched sampler issues one such add per sampled edge, so this
// rate is the ceiling its throughput is compared against.
//
// Built into its own library (libmh_probe.so); only the benchmark loads it.

#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kProbeThreads = 256;

// Every lane adds 1 to `iters` counters chosen by a linear congruential
// sequence of its own; the index is masked to the power-of-two table size.
__global__ __launch_bounds__(kProbeThreads) void k_probe_atomic_adds(int32_t* __restrict__ counters, uint32_t mask,
                                                                     int32_t iters) {
    uint32_t h = (blockIdx.x * blockDim.x + threadIdx.x) * 2654435761u + 12345u;
    for (int32_t i = 0; i < iters; ++i) {
        h = h * 1664525u + 1013904223u;
        atomicAdd(&counters[(h >> 3) & mask], 1);
    }
}

}  // namespace

extern "C" {

// Launches blocks x 256 lanes, each adding 1 to `iters` pseudo-random counters
// of `counters` (device memory of `slots` int32, slots a power of two, 1 to
// 2^30).  Asynchronous on `stream`; returns 0, or -1 for invalid arguments
// (nothing launched) and -2 for a failed launch.
int mhp_atomic_adds(int32_t* counters, int64_t slots, int32_t blocks, int32_t iters, hipStream_t stream) {
    if (!counters || slots < 1 || slots > (int64_t{1} << 30) || (slots & (slots - 1)) != 0 || blocks < 1 ||
        iters < 0)
        return -1;
    hipLaunchKernelGGL(k_probe_atomic_adds, dim3(blocks), dim3(kProbeThreads), 0, stream, counters,
                       (uint32_t)(slots - 1), iters);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // extern "C"

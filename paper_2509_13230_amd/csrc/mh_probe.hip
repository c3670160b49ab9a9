// Measurement and test probes, not part of the sampler, built into their own
// library (libmh_probe.so), which only the benchmark and the tests load:
//  - the rate at which the GPU performs device-scope int32 atomic adds at
//    random addresses (the degree sink of the batched sampler issues one such
//    add per sampled edge, so this rate is the ceiling it is compared against);
//  - the sweep's own logarithms (log_fast, log1p_fast of mh_common.hpp)
//    evaluated on the device, so that tests can bound their error against the
//    host's log and log1p.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "mh_common.hpp"

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

// out_log[i] = log_fast(u[i]) and out_log1p[i] = log1p_fast(t[i]), the
// device functions the sweep calls for the skip (U in (0, 1], t > -1 finite).
__global__ __launch_bounds__(kProbeThreads) void k_probe_logs(const double* __restrict__ u,
                                                              const double* __restrict__ t, int64_t n,
                                                              double* __restrict__ out_log,
                                                              double* __restrict__ out_log1p) {
    const int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
    if (i >= n) return;
    out_log[i] = mh::log_fast(u[i]);
    out_log1p[i] = mh::log1p_fast(t[i]);
}

}  // namespace

extern "C" {

// Evaluates the sweep's logarithms on n inputs (device arrays of float64):
// out_log = log_fast(u), u normal and positive; out_log1p = log1p_fast(t),
// t finite and > -1 (1 + t rounded to a normal number).  Asynchronous on `stream`; 0, -1 for invalid arguments,
// -2 for a failed launch.
int mhp_sweep_logs(const double* u, const double* t, int64_t n, double* out_log, double* out_log1p,
                   hipStream_t stream) {
    if (n < 0 || (n > 0 && (!u || !t || !out_log || !out_log1p))) return -1;
    if (n == 0) return 0;
    const int64_t blocks = (n + kProbeThreads - 1) / kProbeThreads;
    if (blocks > 0x7FFFFFFF) return -1;
    hipLaunchKernelGGL(k_probe_logs, dim3((unsigned)blocks), dim3(kProbeThreads), 0, stream, u, t, n, out_log,
                       out_log1p);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

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

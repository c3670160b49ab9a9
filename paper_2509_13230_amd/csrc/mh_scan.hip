// Exclusive prefix sums (unsigned 32/64-bit) over device arrays, in three
// steps per level: per-tile sums, a scan of the tile sums (recursive), and a
// per-tile scan that adds the carried-in sum.  out has n + 1 entries, out[n]
// is the total; in == out is allowed (each tile is read before it is written).
#include "mh_common.hpp"
#include "mh_internal.hpp"
#include "mh_lookback.hpp"

namespace mh {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;  // 2048

template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* lds_waves, T* block_total) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    T inc = wave_inclusive_scan(v);
    if (lane == 63) lds_waves[wave] = inc;
    __syncthreads();
    T before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        T t = lds_waves[w];
        if (w < wave) before += t;
        total += t;
    }
    *block_total = total;
    return before + inc - v;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const T* __restrict__ in, int64_t n, T* __restrict__ sums) {
    __shared__ T lds_waves[kScanThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    T v = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;  // coalesced
        if (i < n) v += in[i];
    }
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) lds_waves[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        T t = 0;
        for (int w = 0; w < kScanThreads / kWave; ++w) t += lds_waves[w];
        sums[blockIdx.x] = t;
    }
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_tile_scan(const T* in, T* out, int64_t n, const T* __restrict__ carry) {
    __shared__ T lds_waves[kScanThreads / kWave];
    __shared__ T lds_items[kScanTile];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    // stage the tile through LDS: coalesced global reads, then per-thread runs
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int idx = k * kScanThreads + threadIdx.x;
        int64_t i = base + idx;
        lds_items[idx] = (i < n) ? in[i] : T(0);
    }
    __syncthreads();
    T vals[kScanItems];
    T run = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        vals[k] = lds_items[threadIdx.x * kScanItems + k];
        run += vals[k];
    }
    T total;
    T before = block_exclusive_scan(run, lds_waves, &total);
    const T c = carry ? carry[blockIdx.x] : T(0);
    before += c;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        lds_items[threadIdx.x * kScanItems + k] = before;
        before += vals[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int idx = k * kScanThreads + threadIdx.x;
        int64_t i = base + idx;
        if (i < n) out[i] = lds_items[idx];
    }
    if (threadIdx.x == 0 && base + kScanTile >= n) out[n] = c + total;
}

template <typename T>
size_t levels_bytes(int64_t n) {
    Sizer s;
    while (n > kScanTile) {
        int64_t nb = (n + kScanTile - 1) / kScanTile;
        s.take<T>(nb + 1);
        n = nb;
    }
    return s.used + 256;
}

template <typename T>
mh_status scan_impl(const T* in, T* out, int64_t n, Arena& ar, hipStream_t stream) {
    if (n <= kScanTile) {
        hipLaunchKernelGGL(k_tile_scan<T>, dim3(1), dim3(kScanThreads), 0, stream, in, out, n, (const T*)nullptr);
        MH_HIP_TRY(hipGetLastError());
        return MH_OK;
    }
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    T* sums = ar.take<T>(nb + 1);
    if (!sums) return MH_EWORKSPACE;
    hipLaunchKernelGGL(k_tile_sums<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, stream, in, n, sums);
    MH_HIP_TRY(hipGetLastError());
    mh_status st = scan_impl<T>(sums, sums, nb, ar, stream);
    if (st != MH_OK) return st;
    hipLaunchKernelGGL(k_tile_scan<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, stream, in, out, n, (const T*)sums);
    MH_HIP_TRY(hipGetLastError());
    return MH_OK;
}

// ---- single pass: one kernel, decoupled look-back over tiles ----
__global__ __launch_bounds__(kLbThreads) void k_scan_onepass(const uint64_t* in, uint64_t* out, int64_t n,
                                                             int64_t tiles, uint64_t* state, uint64_t* samples,
                                                             int32_t* err) {
    __shared__ LbShared sh;
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t base = tile * kLbTile;
#pragma unroll
        for (int k = 0; k < kLbItems; ++k) {
            const int idx = k * kLbThreads + threadIdx.x;
            const int64_t i = base + idx;
            sh.items[lb_at(idx)] = (i < n) ? in[i] : 0ull;
        }
        const uint64_t end = lb_tile_scan(sh, tile, state, err);
#pragma unroll
        for (int k = 0; k < kLbItems; ++k) {
            const int idx = k * kLbThreads + threadIdx.x;
            const int64_t i = base + idx;
            if (i < n) {
                const uint64_t v = sh.items[lb_at(idx)];
                out[i] = v;
                if (samples && (i & ((1 << kSampleShift) - 1)) == 0) samples[i >> kSampleShift] = v;
            }
        }
        if (threadIdx.x == 0 && base + kLbTile >= n) {
            out[n] = end;
            if (samples && (n & ((1 << kSampleShift) - 1)) == 0) samples[n >> kSampleShift] = end;
        }
    }
}

}  // namespace

size_t scan_workspace_bytes(int64_t n) { return levels_bytes<uint64_t>(n); }

mh_status scan_exclusive_u64_onepass(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* state,
                                     uint64_t* samples, int32_t* err, hipStream_t stream) {
    if (n < 0) return MH_EINVAL;
    const int64_t tiles = lb_tiles(n);
    const int64_t resident = resident_blocks(k_scan_onepass, kLbThreads);
    const int64_t grid = tiles < resident ? tiles : resident;
    hipLaunchKernelGGL(k_scan_onepass, dim3((unsigned)grid), dim3(kLbThreads), 0, stream, in, out, n, tiles, state,
                       samples, err);
    MH_HIP_TRY(hipGetLastError());
    return MH_OK;
}

mh_status scan_exclusive_u64(const uint64_t* in, uint64_t* out, int64_t n, void* ws, size_t ws_bytes,
                             hipStream_t stream) {
    if (n < 0) return MH_EINVAL;
    Arena ar(ws, ws_bytes);
    return scan_impl<uint64_t>(in, out, n, ar, stream);
}

mh_status scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, void* ws, size_t ws_bytes,
                             hipStream_t stream) {
    if (n < 0) return MH_EINVAL;
    Arena ar(ws, ws_bytes);
    return scan_impl<uint32_t>(in, out, n, ar, stream);
}

}  // namespace mh

// Exclusive prefix sums (unsigned 32/64-bit) over device arrays, in three
// steps per level: per-tile sums, a scan of the tile sums (recursive), and a
// per-tile scan that adds the carried-in sum.  out has n + 1 entries, out[n]
// is the total; in == out is allowed (each tile is read before it is written).
#include "mh_common.hpp"
#include "mh_internal.hpp"

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
constexpr int kOneItems = 16;
constexpr int kOneTile = kScanThreads * kOneItems;  // 4096
constexpr uint32_t kOneSpinLimit = 1u << 20;
// Look-back word per tile, zero at launch: the flag in the top two bits (1 = the
// tile's own sum, 2 = the inclusive prefix through the tile) and the value in
// the low 62.  Flag and value travel in one relaxed atomic, so no fence is
// needed between them.  Prefix sums must stay below 2^62 (the caller checks).
constexpr uint64_t kOneAgg = 1ull << 62;
constexpr uint64_t kOneInc = 2ull << 62;
constexpr uint64_t kOneValue = kOneAgg - 1;

// Blocks take tiles blockIdx, blockIdx + gridDim, ... with the whole grid
// resident, so a tile waits only on lower tiles that are being processed.
__global__ __launch_bounds__(kScanThreads) void k_scan_onepass(const uint64_t* in, uint64_t* out, int64_t n,
                                                               int64_t tiles, uint64_t* state, int32_t* err) {
    __shared__ uint64_t lds_items[kOneTile];
    __shared__ uint64_t lds_waves[kScanThreads / kWave];
    __shared__ uint64_t s_excl;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t base = tile * kOneTile;
#pragma unroll
        for (int k = 0; k < kOneItems; ++k) {
            const int idx = k * kScanThreads + threadIdx.x;
            const int64_t i = base + idx;
            lds_items[idx] = (i < n) ? in[i] : 0ull;
        }
        __syncthreads();
        uint64_t vals[kOneItems];
        uint64_t run = 0;
#pragma unroll
        for (int k = 0; k < kOneItems; ++k) {
            vals[k] = lds_items[threadIdx.x * kOneItems + k];
            run += vals[k];
        }
        uint64_t total;
        const uint64_t before = block_exclusive_scan(run, lds_waves, &total);
        if (threadIdx.x == 0) {
            __hip_atomic_store(&state[tile], (tile == 0 ? kOneInc : kOneAgg) | total, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            if (tile == 0) s_excl = 0;
        }
        if (wave == 0 && tile > 0) {
            // lane l looks at tile t - l; sum published sums back to the
            // nearest inclusive prefix, re-polling where a tile is not yet out
            uint64_t excl = 0;
            int64_t t = tile - 1;
            uint32_t spins = 0;
            for (;;) {
                const int64_t tt = t - lane;
                const uint64_t w =
                    (tt >= 0) ? __hip_atomic_load(&state[tt], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kOneInc;
                const uint64_t f = w & ~kOneValue;
                const uint64_t none = __ballot(f == 0);
                const uint64_t incl = __ballot(f == kOneInc);
                const int first_none = none ? (int)__ffsll((unsigned long long)none) - 1 : kWave;
                const int first_incl = incl ? (int)__ffsll((unsigned long long)incl) - 1 : kWave;
                const bool finish = first_incl < first_none;
                const int used = finish ? first_incl + 1 : first_none;
                excl += wave_sum(lane < used ? (w & kOneValue) : 0ull);
                if (finish) break;
                t -= used;
                if (used == 0) {
                    if (++spins > kOneSpinLimit) {
                        raise_status(err, MH_EHIP);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            if (lane == 0) {
                __hip_atomic_store(&state[tile], kOneInc | (excl + total), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_excl = excl;
            }
        }
        __syncthreads();
        uint64_t acc = s_excl + before;
#pragma unroll
        for (int k = 0; k < kOneItems; ++k) {
            lds_items[threadIdx.x * kOneItems + k] = acc;
            acc += vals[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kOneItems; ++k) {
            const int idx = k * kScanThreads + threadIdx.x;
            const int64_t i = base + idx;
            if (i < n) out[i] = lds_items[idx];
        }
        if (threadIdx.x == 0 && base + kOneTile >= n) out[n] = s_excl + total;
        __syncthreads();  // the next tile reuses the LDS
    }
}

}  // namespace

size_t scan_workspace_bytes(int64_t n) { return levels_bytes<uint64_t>(n); }

int64_t scan_onepass_state_words(int64_t n) { return n > 0 ? (n + kOneTile - 1) / kOneTile : 1; }

mh_status scan_exclusive_u64_onepass(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* state, int32_t* err,
                                     hipStream_t stream) {
    if (n < 0) return MH_EINVAL;
    const int64_t tiles = scan_onepass_state_words(n);
    const int64_t resident = resident_blocks(k_scan_onepass, kScanThreads);
    const int64_t grid = tiles < resident ? tiles : resident;
    hipLaunchKernelGGL(k_scan_onepass, dim3((unsigned)grid), dim3(kScanThreads), 0, stream, in, out, n, tiles, state,
                       err);
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

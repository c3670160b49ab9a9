// Stable LSD radix sort of 64-bit keys with 32-bit payloads, 8 passes of 8
// bits.  Per pass: a counting kernel (per-tile digit histograms, digit-major),
// an exclusive scan of the histograms, and a scatter kernel.  Inside a wave,
// keys with equal digits are grouped by 8 ballots (one per digit bit), which
// gives each key its rank among equal digits without LDS atomics, so heavy
// ties (many equal keys) cost nothing extra.
#include "mh_common.hpp"
#include "mh_internal.hpp"

namespace mh {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kKeysPerLane = 16;
constexpr int kWaveKeys = kWave * kKeysPerLane;     // 1024, contiguous per wave
constexpr int kTileKeys = kWaveKeys * kSortWaves;  // 4096 per block
constexpr int kRadix = 256;

// Lanes (among `valid`) whose digit equals this lane's.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t vote = __ballot(bit);
        m &= bit ? vote : ~vote;
    }
    return m;
}

__global__ __launch_bounds__(kSortThreads) void k_radix_count(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                              uint32_t* __restrict__ counts, int nblocks) {
    __shared__ uint32_t cnt[kSortWaves][kRadix];
    for (int i = threadIdx.x; i < kSortWaves * kRadix; i += kSortThreads) (&cnt[0][0])[i] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kTileKeys + (int64_t)wave * kWaveKeys;
    const uint64_t lt = lanemask_lt();
    for (int r = 0; r < kKeysPerLane; ++r) {
        const int64_t i = base + (int64_t)r * kWave + lane;
        const bool valid = i < n;
        if (__ballot(valid) == 0) break;
        const uint32_t d = valid ? (uint32_t)(keys[i] >> shift) & (kRadix - 1) : 0u;
        const uint64_t m = match_digit(d, valid);
        if (valid && (m & lt) == 0) cnt[wave][d] += (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    const int d = threadIdx.x;  // kSortThreads == kRadix
    uint32_t total = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) total += cnt[w][d];
    counts[(int64_t)d * nblocks + blockIdx.x] = total;
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint64_t* __restrict__ kin,
                                                                const uint32_t* __restrict__ vin,
                                                                uint64_t* __restrict__ kout,
                                                                uint32_t* __restrict__ vout, int64_t n, int shift,
                                                                const uint32_t* __restrict__ offsets, int nblocks) {
    __shared__ uint32_t cnt[kSortWaves][kRadix];
    __shared__ uint32_t woff[kSortWaves][kRadix];
    for (int i = threadIdx.x; i < kSortWaves * kRadix; i += kSortThreads) (&cnt[0][0])[i] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kTileKeys + (int64_t)wave * kWaveKeys;
    const uint64_t lt = lanemask_lt();
    uint64_t k[kKeysPerLane];
    uint32_t v[kKeysPerLane];
    uint32_t rank[kKeysPerLane];
#pragma unroll
    for (int r = 0; r < kKeysPerLane; ++r) {
        const int64_t i = base + (int64_t)r * kWave + lane;
        const bool valid = i < n;
        k[r] = valid ? kin[i] : 0ull;
        v[r] = valid ? vin[i] : 0u;
        const uint32_t d = (uint32_t)(k[r] >> shift) & (kRadix - 1);
        const uint64_t m = match_digit(d, valid);
        const uint32_t prior = cnt[wave][d];
        rank[r] = prior + (uint32_t)__popcll(m & lt);
        __builtin_amdgcn_wave_barrier();
        if (valid && (m & lt) == 0) cnt[wave][d] = prior + (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    {
        const int d = threadIdx.x;
        uint32_t run = offsets[(int64_t)d * nblocks + blockIdx.x];
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) {
            woff[w][d] = run;
            run += cnt[w][d];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kKeysPerLane; ++r) {
        const int64_t i = base + (int64_t)r * kWave + lane;
        if (i < n) {
            const uint32_t d = (uint32_t)(k[r] >> shift) & (kRadix - 1);
            const uint32_t pos = woff[wave][d] + rank[r];
            kout[pos] = k[r];
            vout[pos] = v[r];
        }
    }
}

}  // namespace

size_t radix_workspace_bytes(int64_t n) {
    const int64_t nblocks = (n + kTileKeys - 1) / kTileKeys;
    Sizer s;
    s.take<uint32_t>((size_t)nblocks * kRadix + 1);
    return s.used + scan_workspace_bytes(nblocks * kRadix + 1) + 256;
}

mh_status radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt, int64_t n,
                         void* ws, size_t ws_bytes, hipStream_t stream) {
    if (n <= 1) return MH_OK;
    if (n > (int64_t)0xFFFFFFFFll) return MH_EINVAL;
    const int64_t nblocks = (n + kTileKeys - 1) / kTileKeys;
    Arena ar(ws, ws_bytes);
    uint32_t* counts = ar.take<uint32_t>((size_t)nblocks * kRadix + 1);
    if (!counts) return MH_EWORKSPACE;
    void* scan_ws = ar.base + ((ar.used + 255) & ~size_t(255));
    size_t scan_bytes = ws_bytes > ((ar.used + 255) & ~size_t(255)) ? ws_bytes - ((ar.used + 255) & ~size_t(255)) : 0;
    uint64_t* kin = keys;
    uint32_t* vin = vals;
    uint64_t* kout = keys_alt;
    uint32_t* vout = vals_alt;
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = pass * 8;
        hipLaunchKernelGGL(k_radix_count, dim3((unsigned)nblocks), dim3(kSortThreads), 0, stream, kin, n, shift, counts,
                           (int)nblocks);
        MH_HIP_TRY(hipGetLastError());
        mh_status st = scan_exclusive_u32(counts, counts, nblocks * kRadix, scan_ws, scan_bytes, stream);
        if (st != MH_OK) return st;
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nblocks), dim3(kSortThreads), 0, stream, kin, vin, kout, vout,
                           n, shift, counts, (int)nblocks);
        MH_HIP_TRY(hipGetLastError());
        uint64_t* tk = kin; kin = kout; kout = tk;
        uint32_t* tv = vin; vin = vout; vout = tv;
    }
    return MH_OK;  // 8 passes: the result is back in keys/vals
}

}  // namespace mh

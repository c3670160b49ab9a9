// Exclusive prefix sums over tiles of 4096 u64 values with decoupled
// look-back, as a block-level step that producer kernels embed: a kernel
// computes a tile's values into LDS, calls lb_tile_scan, and writes the
// prefixes, so a plan array is produced and scanned in one pass.
//
// Each tile publishes one word: a flag in the top two bits (1 = the tile's own
// sum, 2 = the inclusive prefix through the tile, 3 = the same once the
// producer has written the tile's prefixes out) and the value in the low 62.
// Flag and value travel in one relaxed atomic, so no fence is needed between
// them (an agent-scope release would write back the L2 of an XCD).  Prefix sums
// must stay below 2^62.  Blocks take tiles blockIdx, blockIdx + gridDim, ...
// with at most as many blocks as are resident at once, so a tile waits only on
// lower tiles that running blocks hold; a spin limit turns a stall into an
// error (MH_EHIP), never a hang.
#pragma once

#include "mh_common.hpp"

namespace mh {

constexpr int kLbThreads = 1024;
constexpr int kLbItems = 4;
constexpr int kLbTile = kLbThreads * kLbItems;  // 4096
constexpr uint64_t kLbAgg = 1ull << 62;
constexpr uint64_t kLbInc = 2ull << 62;
// A producer may later mark its inclusive word 3: the same prefix, and the
// tile's scanned values written out (see k_finish_plan_scan).
constexpr uint64_t kLbDone = 3ull << 62;
constexpr uint64_t kLbValue = kLbAgg - 1;
constexpr uint32_t kLbSpinLimit = 1u << 20;

// Element i of a tile lives at items[lb_at(i)]: one padding word per 4
// elements, so that threads reading their 4 consecutive elements (a stride of
// 5 words, 10 banks) hit distinct LDS banks.
__host__ __device__ constexpr int lb_at(int i) { return i + (i >> 2); }

struct LbShared {
    uint64_t items[lb_at(kLbTile)];
    uint64_t waves[kLbThreads / kWave];
    uint64_t excl;
};

// Look-back words of an array of n values (zero before the producing kernel).
__host__ __device__ inline int64_t lb_tiles(int64_t n) { return n > 0 ? (n + kLbTile - 1) / kLbTile : 1; }

// Producers can also write every 256th prefix (indices 0, 256, ..., <= n) to a
// compact sample array, which later searches stage in LDS.
constexpr int kSampleShift = 8;
__host__ __device__ inline int64_t lb_samples(int64_t n) { return (n >> kSampleShift) + 1; }

// In: sh.items[lb_at(i)] = value of element i of the tile (0 past the end).
// Out: sh.items[lb_at(i)] = exclusive prefix of element i over the whole
// array.  Returns the inclusive prefix through the tile's end (the array total
// for the last tile).  Called by all kLbThreads threads of the block.
__device__ inline uint64_t lb_tile_scan(LbShared& sh, int64_t tile, uint64_t* state, int32_t* err) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    uint64_t vals[kLbItems];
    uint64_t run = 0;
#pragma unroll
    for (int k = 0; k < kLbItems; ++k) {
        vals[k] = sh.items[lb_at(threadIdx.x * kLbItems + k)];
        run += vals[k];
    }
    // block exclusive scan of the per-thread runs
    const uint64_t inc = wave_inclusive_scan(run);
    if (lane == 63) sh.waves[wave] = inc;
    __syncthreads();
    uint64_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kLbThreads / kWave; ++w) {
        const uint64_t t = sh.waves[w];
        if (w < wave) before += t;
        total += t;
    }
    before += inc - run;
    if (threadIdx.x == 0) {
        __hip_atomic_store(&state[tile], (tile == 0 ? kLbInc : kLbAgg) | total, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        if (tile == 0) sh.excl = 0;
    }
    if (wave == 0 && tile > 0) {
        // lane l looks at tile t - l: sum the published words back to the
        // nearest inclusive prefix, polling again where a tile is not yet out
        uint64_t excl = 0;
        int64_t t = tile - 1;
        uint32_t spins = 0;
        for (;;) {
            const int64_t tt = t - lane;
            const uint64_t w =
                (tt >= 0) ? __hip_atomic_load(&state[tt], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kLbInc;
            const uint64_t f = w & ~kLbValue;
            const uint64_t none = __ballot(f == 0);
            const uint64_t incl = __ballot(f >= kLbInc);  // an inclusive prefix (flag 2 or 3)
            const int first_none = none ? (int)__ffsll((unsigned long long)none) - 1 : kWave;
            const int first_incl = incl ? (int)__ffsll((unsigned long long)incl) - 1 : kWave;
            const bool finish = first_incl < first_none;
            const int used = finish ? first_incl + 1 : first_none;
            excl += wave_sum(lane < used ? (w & kLbValue) : 0ull);
            if (finish) break;
            t -= used;
            if (used == 0) {
                if (++spins > kLbSpinLimit) {
                    raise_status(err, MH_EHIP);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        if (lane == 0) {
            __hip_atomic_store(&state[tile], kLbInc | (excl + total), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            sh.excl = excl;
        }
    }
    __syncthreads();
    const uint64_t excl = sh.excl;
    uint64_t acc = excl + before;
#pragma unroll
    for (int k = 0; k < kLbItems; ++k) {
        sh.items[lb_at(threadIdx.x * kLbItems + k)] = acc;
        acc += vals[k];
    }
    __syncthreads();
    return excl + total;
}

}  // namespace mh

// Stable LSD radix sort of 64-bit keys with 32-bit payloads: 8 passes of 8
// bits, one kernel per pass ("one-sweep" with decoupled look-back).
//
// The digit histograms of all 8 passes come from one counting kernel (fused
// into key preparation by the caller, or k_radix_hist).  In a pass, each block
// takes a tile ticket, ranks its 4096 keys (keys with equal digits are grouped
// by 8 ballots, one per digit bit, so ties cost nothing extra), publishes its
// per-digit counts, and finds the counts of all earlier tiles by looking back
// over their published words (a 64-bit word per tile and digit: a flag in the
// high half -- 1 = this tile's count, 2 = inclusive prefix over tiles 0..t --
// and the value in the low half).  A block waits only on tiles with smaller
// tickets, which have started and publish without waiting, so the look-back
// always ends; a spin limit turns a lost update into an error, never a hang.
// Keys are then reordered by digit in LDS and written in coalesced runs.
#include "mh_common.hpp"
#include "mh_internal.hpp"

namespace mh {

namespace {

// 16 waves share a tile (4 keys per lane): a pass is a chain of dependent
// steps (load, rank, publish, look back, scatter) on ~250 tiles for 1M keys,
// so the waves of a block, not more tiles, are what hide its latencies.
constexpr int kSortThreads = 1024;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kKeysPerLane = 4;
constexpr int kWaveKeys = kWave * kKeysPerLane;     // 256, contiguous per wave
constexpr int kTileKeys = kWaveKeys * kSortWaves;  // 4096 per block
constexpr int kRadix = 256;
constexpr int kPasses = 8;
constexpr uint64_t kFlagAggregate = 1ull << 32;
constexpr uint64_t kFlagPrefix = 2ull << 32;
constexpr uint32_t kSpinLimit = 1u << 20;
constexpr int kLookWindow = 8;
// Column exchange: a column of at most kXchgTiles tiles per 256 threads, so a
// block scans kXchgCols digit columns at once.
constexpr int kXchgTiles = 256;
constexpr int kXchgCols = kSortThreads / kXchgTiles;
// The counting kernel adds its block histograms into kHistCopies copies (block
// b into copy b % kHistCopies); readers sum the copies.
constexpr int kHistCopies = kRadixHistCopies;

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

// Exclusive scan of one value per thread (all kSortThreads) through LDS.
__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t* lds_wave) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = wave_inclusive_scan(v);
    if (lane == 63) lds_wave[wave] = inc;
    __syncthreads();
    uint32_t before = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w)
        if (w < wave) before += lds_wave[w];
    __syncthreads();
    return before + inc - v;
}

// Zeroes two ranges of u64 words (the second may be empty).
__global__ __launch_bounds__(kSortThreads) void k_zero_u64(uint64_t* __restrict__ p, int64_t n,
                                                           uint64_t* __restrict__ q, int64_t m) {
    const int64_t stride = (int64_t)gridDim.x * kSortThreads;
    for (int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x; i < n; i += stride) p[i] = 0;
    for (int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x; i < m; i += stride) q[i] = 0;
}

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t* __restrict__ keys, int64_t n,
                                                             uint32_t* __restrict__ ghist) {
    __shared__ uint32_t h[kPasses * kRadix];
    for (int i = threadIdx.x; i < kPasses * kRadix; i += kSortThreads) h[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTileKeys;
    for (int k = threadIdx.x; k < kTileKeys; k += kSortThreads) {
        const int64_t i = base + k;
        if (i < n) {
            const uint64_t key = keys[i];
#pragma unroll
            for (int p = 0; p < kPasses; ++p) atomicAdd(&h[p * kRadix + ((key >> (8 * p)) & 255)], 1u);
        }
    }
    __syncthreads();
    uint32_t* copy = ghist + (blockIdx.x % kHistCopies) * kPasses * kRadix;
    for (int i = threadIdx.x; i < kPasses * kRadix; i += kSortThreads)
        if (h[i]) atomicAdd(&copy[i], h[i]);
}

template <bool XCHG>
__global__ __launch_bounds__(kSortThreads) void k_onesweep(const uint64_t* __restrict__ kin,
                                                           const uint32_t* __restrict__ vin,
                                                           uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                           int64_t n, int shift, const uint32_t* __restrict__ ghist,
                                                           uint64_t* status, uint32_t* ticket, bool use_ticket,
                                                           int32_t* err) {
    __shared__ uint64_t s_keys[kTileKeys];
    __shared__ uint32_t s_vals[kTileKeys];
    __shared__ uint32_t cnt[kSortWaves][kRadix];
    __shared__ uint32_t s_bstart[kRadix];
    __shared__ uint32_t s_goff[kRadix];
    __shared__ uint32_t s_dstart[kRadix];
    __shared__ uint32_t s_scan[kSortWaves];
    __shared__ uint32_t s_tile;

    // Tiles are taken in ticket order unless the whole grid is resident at once
    // (then every block runs concurrently and its index serves, sparing 1 atomic
    // per block on one address).
    if (threadIdx.x == 0) s_tile = use_ticket ? atomicAdd(ticket, 1u) : blockIdx.x;
    for (int i = threadIdx.x; i < kSortWaves * kRadix; i += kSortThreads) (&cnt[0][0])[i] = 0;
    __syncthreads();
    const int64_t tile = s_tile;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t tbase = tile * kTileKeys;
    const int64_t base = tbase + (int64_t)wave * kWaveKeys;
    const uint64_t lt = lanemask_lt();

    // rank every key among the wave's keys with the same digit
    uint64_t k[kKeysPerLane];
    uint32_t v[kKeysPerLane];
    uint32_t rank[kKeysPerLane];
    // all loads first: the ranking below orders LDS accesses with wave barriers,
    // which the compiler will not move loads across
#pragma unroll
    for (int r = 0; r < kKeysPerLane; ++r) {
        const int64_t i = base + (int64_t)r * kWave + lane;
        const bool valid = i < n;
        k[r] = valid ? kin[i] : 0ull;
        v[r] = valid ? vin[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kKeysPerLane; ++r) {
        const int64_t i = base + (int64_t)r * kWave + lane;
        const bool valid = i < n;
        const uint32_t d = (uint32_t)(k[r] >> shift) & (kRadix - 1);
        const uint64_t m = match_digit(d, valid);
        const uint32_t prior = cnt[wave][d];
        rank[r] = prior + (uint32_t)__popcll(m & lt);
        __builtin_amdgcn_wave_barrier();
        if (valid && (m & lt) == 0) cnt[wave][d] = prior + (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    const int d = threadIdx.x;  // one digit per thread of the first kRadix
    const bool dig = d < kRadix;
    uint32_t total = 0, dtotal = 0;
    uint64_t* st = status + tile * kRadix + d;
    if (dig) {
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) {
            const uint32_t c = cnt[w][d];
            cnt[w][d] = total;  // becomes the wave's offset inside the block's digit run
            total += c;
        }
        __hip_atomic_store(st, (tile == 0 && !XCHG ? kFlagPrefix : kFlagAggregate) | total, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (int c = 0; c < kHistCopies; ++c) dtotal += ghist[c * kPasses * kRadix + d];
    }
    const uint32_t bstart = block_exclusive(total, s_scan);
    const uint32_t dstart = block_exclusive(dtotal, s_scan);
    uint32_t excl = 0;
    if (XCHG) {
        // Every tile is resident (at most kXchgTiles): instead of a chain of
        // look-backs, block b scans the digit columns b, b + G, b + 2G, ...
        // (G blocks; kXchgCols columns at once, 256 threads each, one tile per
        // thread) over all tiles' published counts, and writes each tile its
        // start for that digit (flag 2 over the count word, which only this
        // block reads); then every tile reads its 256 starts back.  Two round
        // trips per pass when G >= 256 / kXchgCols.
        if (dig) s_dstart[d] = dstart;
        const int nt = (int)gridDim.x;
        const int tcol = threadIdx.x & (kXchgTiles - 1);  // this thread's tile in the column
        for (int c0 = blockIdx.x; c0 < kRadix; c0 += kXchgCols * nt) {
            const int col = c0 + (int)(threadIdx.x / kXchgTiles) * nt;
            const bool mine = tcol < nt && col < kRadix;
            uint64_t* cw = status + (int64_t)tcol * kRadix + col;
            uint32_t c = 0;
            if (mine) {
                uint32_t spins = 0;
                for (;;) {
                    const uint64_t w = __hip_atomic_load(cw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (w & ~0xFFFFFFFFull) {
                        c = (uint32_t)w;
                        break;
                    }
                    if (++spins > kSpinLimit) {
                        raise_status(err, MH_EHIP);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            // exclusive scan over each column's 256 threads (4 waves)
            const uint32_t inc = wave_inclusive_scan(c);
            if (lane == 63) s_scan[wave] = inc;
            __syncthreads();  // also orders the s_dstart writes
            uint32_t before = inc - c;
            for (int w = wave & ~(kXchgTiles / kWave - 1); w < wave; ++w) before += s_scan[w];
            if (mine)
                __hip_atomic_store(cw, kFlagPrefix | (s_dstart[col] + before), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
        }
        if (dig) {
            uint32_t spins = 0;
            for (;;) {
                const uint64_t w = __hip_atomic_load(st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((w & ~0xFFFFFFFFull) == kFlagPrefix) {
                    excl = (uint32_t)w - dstart;  // earlier tiles' keys with digit d
                    break;
                }
                if (++spins > kSpinLimit) {
                    raise_status(err, MH_EHIP);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
    } else if (dig && tile > 0) {
        // look back over the preceding tiles, kLookWindow words in flight at a time
        int64_t t = tile - 1;
        uint32_t spins = 0;
        bool done = false;
        while (!done) {
            uint64_t w[kLookWindow];
#pragma unroll
            for (int q = 0; q < kLookWindow; ++q)
                w[q] = (t - q >= 0) ? __hip_atomic_load(status + (t - q) * kRadix + d, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT)
                                    : kFlagPrefix;
            int used = 0;
#pragma unroll
            for (int q = 0; q < kLookWindow; ++q) {
                if (done || used < q) continue;  // stop at the first word still unpublished
                const uint64_t flag = w[q] & ~0xFFFFFFFFull;
                if (flag == 0) continue;
                excl += (uint32_t)w[q];
                used = q + 1;
                if (flag == kFlagPrefix) done = true;
            }
            if (done) break;
            t -= used;
            if (used == 0) {
                if (++spins > kSpinLimit) {
                    raise_status(err, MH_EHIP);  // the scatter below stays in bounds
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __hip_atomic_store(st, kFlagPrefix | (excl + total), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (dig) {
        s_bstart[d] = bstart;
        s_goff[d] = dstart + excl - bstart;
    }
    __syncthreads();

    // reorder the tile by digit in LDS, then write each digit's run contiguously
#pragma unroll
    for (int r = 0; r < kKeysPerLane; ++r) {
        const int64_t i = base + (int64_t)r * kWave + lane;
        if (i < n) {
            const uint32_t dd = (uint32_t)(k[r] >> shift) & (kRadix - 1);
            const uint32_t lp = s_bstart[dd] + cnt[wave][dd] + rank[r];
            s_keys[lp] = k[r];
            s_vals[lp] = v[r];
        }
    }
    __syncthreads();
    const int64_t cnt_tile = (n - tbase) < kTileKeys ? (n - tbase) : kTileKeys;
    for (int i = threadIdx.x; i < cnt_tile; i += kSortThreads) {
        const uint64_t key = s_keys[i];
        const uint32_t dd = (uint32_t)(key >> shift) & (kRadix - 1);
        const uint32_t pos = s_goff[dd] + (uint32_t)i;
        if (pos < (uint64_t)n) {  // always, unless a look-back gave up (then the error is raised)
            kout[pos] = key;
            vout[pos] = s_vals[i];
        }
    }
}

int64_t sort_blocks(int64_t n) { return (n + kTileKeys - 1) / kTileKeys; }

}  // namespace

size_t radix_workspace_bytes(int64_t n) {
    const int64_t nb = sort_blocks(n);
    Sizer s;
    s.take<uint64_t>((size_t)kPasses * nb * kRadix + kHistCopies * kPasses * kRadix / 2 + kPasses);
    s.take<int32_t>(1);
    return s.used + 256;
}

// Zeroes the look-back words, histograms and tickets (one kernel), counts all
// passes' digits (unless the caller already did, hist_ready), then runs the
// 8 passes.  The result ends in keys/vals.
mh_status radix_sort_u64_hist(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt, int64_t n,
                              uint32_t* hist, uint64_t* status, uint32_t* tickets, int32_t* err,
                              bool hist_ready, hipStream_t stream) {
    const int64_t nb = sort_blocks(n);
    if (!hist_ready) {
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kSortThreads), 0, stream, keys, n, hist);
        MH_HIP_TRY(hipGetLastError());
    }
    // One tile per CU at most: the column exchange (all tiles resident, with a
    // CU to spare for each); otherwise the look-back, by ticket unless the
    // whole grid is resident.
    const bool xchg = nb <= kXchgTiles && nb <= device_cus();
    const bool use_ticket = !xchg && nb > resident_blocks(k_onesweep<false>, kSortThreads);
    uint64_t* kin = keys;
    uint32_t* vin = vals;
    uint64_t* kout = keys_alt;
    uint32_t* vout = vals_alt;
    for (int pass = 0; pass < kPasses; ++pass) {
        hipLaunchKernelGGL(xchg ? k_onesweep<true> : k_onesweep<false>, dim3((unsigned)nb), dim3(kSortThreads), 0,
                           stream, kin, vin, kout, vout, n, pass * 8, hist + pass * kRadix,
                           status + (int64_t)pass * nb * kRadix, tickets + pass, use_ticket, err);
        MH_HIP_TRY(hipGetLastError());
        uint64_t* tk = kin; kin = kout; kout = tk;
        uint32_t* tv = vin; vin = vout; vout = tv;
    }
    return MH_OK;
}

// Layout of the sort's scratch: look-back words, then histograms and tickets.
struct SortScratch {
    uint64_t* status;
    uint32_t* hist;
    uint32_t* tickets;
    int32_t* err;
    int64_t words;  // u64 words to zero (status + hist + tickets)
};

static SortScratch sort_scratch(void* ws, size_t ws_bytes, int64_t n, bool* ok) {
    const int64_t nb = sort_blocks(n);
    Arena ar(ws, ws_bytes);
    const int64_t status_words = (int64_t)kPasses * nb * kRadix;
    const int64_t extra_words = kHistCopies * kPasses * kRadix / 2 + kPasses;
    uint64_t* block = ar.take<uint64_t>(status_words + extra_words);
    int32_t* err = ar.take<int32_t>(1);
    *ok = !ar.overflow;
    SortScratch s{};
    if (!*ok) return s;
    s.status = block;
    s.hist = reinterpret_cast<uint32_t*>(block + status_words);
    s.tickets = s.hist + kHistCopies * kPasses * kRadix;
    s.err = err;
    s.words = status_words + extra_words;
    return s;
}

mh_status radix_prepare(void* ws, size_t ws_bytes, int64_t n, uint32_t** hist, hipStream_t stream,
                        uint64_t* extra_zero, int64_t extra_words) {
    bool ok = false;
    SortScratch s = sort_scratch(ws, ws_bytes, n, &ok);
    if (!ok) return MH_EWORKSPACE;
    if (!extra_zero) extra_words = 0;
    const int64_t most = s.words > extra_words ? s.words : extra_words;
    int64_t blocks = (most + kSortThreads - 1) / kSortThreads;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)blocks), dim3(kSortThreads), 0, stream, s.status, s.words,
                       extra_zero, extra_words);
    MH_HIP_TRY(hipGetLastError());
    *hist = s.hist;
    return MH_OK;
}

mh_status radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt, int64_t n,
                         void* ws, size_t ws_bytes, bool hist_ready, int32_t* err, hipStream_t stream) {
    if (n <= 1) return MH_OK;
    if (n > (int64_t)0xFFFFFFFFll) return MH_EINVAL;
    bool ok = false;
    SortScratch s = sort_scratch(ws, ws_bytes, n, &ok);
    if (!ok) return MH_EWORKSPACE;
    return radix_sort_u64_hist(keys, vals, keys_alt, vals_alt, n, s.hist, s.status, s.tickets, err ? err : s.err,
                               hist_ready, stream);
}

}  // namespace mh

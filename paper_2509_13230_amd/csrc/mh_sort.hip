// Stable LSD radix sort of 64-bit keys with 32-bit payloads, done as a sort by
// the keys' high 32 bits (4 passes of 8 bits, one kernel per pass) followed by
// a repair of the runs whose high halves tie but whose low halves are out of
// order.  The caller passes hi = key >> 32 as the sort key and pay = (low half
// << 32) | payload, so sorting a run of equal hi by pay orders it by (key,
// payload); with payloads distinct (node ids) that is the order of a full
// stable sort.  A first pass that makes the keys from node parameters sorts
// them less their least high half, found by the zeroing kernel before it, with
// only the passes their spread needs (fitted degrees within a factor 2^15
// span 24 bits: 3 passes); the passes it does not need return at once.
//
// Passes ("one-sweep"): the digit histograms of all passes come from one
// counting kernel (fused into key preparation by the caller).  In a pass, each
// block ranks its 4096 keys (keys with equal digits are grouped by 8 ballots,
// one per digit bit, so ties cost nothing extra), publishes its per-digit
// counts, and finds the counts of all earlier tiles, by a column exchange when
// every tile has a CU of its own, else by looking back over their published
// words (a 64-bit word per tile and digit: a flag in the high half -- 1 = this
// tile's count, 2 = inclusive prefix over tiles 0..t -- and the value in the
// low half).  A block waits only on tiles that have started and publish
// without waiting, so the look-back always ends; a spin limit turns a lost
// update into an error, never a hang.  Keys are then reordered by digit in LDS
// and written in coalesced runs.
//
// Repair: one kernel finds every run of equal hi that holds a descent of pay,
// claims it for one block (a bit at the run's start), and sorts it by pay --
// a wave per run of up to 64, a block and LDS up to 512, and a block-level LSD
// through scratch beyond.  Inputs whose keys differ within their high halves
// (fitted parameters: ties by degree class) have no such runs.
#include "mh_common.hpp"
#include "mh_internal.hpp"
#include "mh_keys.hpp"

namespace mh {

namespace {

// 16 waves share a tile (4 keys per lane): a pass is a chain of dependent
// steps (load, rank, publish, exchange, scatter) on ~250 tiles for 1M keys,
// so the waves of a block, not more tiles, are what hide its latencies.
constexpr int kSortThreads = 1024;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kKeysPerLane = 4;
constexpr int kWaveKeys = kWave * kKeysPerLane;     // 256, contiguous per wave
constexpr int kTileKeys = kWaveKeys * kSortWaves;  // 4096 per block
constexpr int kRadix = 256;
constexpr int kPasses = kRadixPasses;  // 4 passes over the 32-bit sort key
constexpr uint64_t kFlagAggregate = 1ull << 32;
constexpr uint64_t kFlagPrefix = 2ull << 32;
constexpr uint32_t kSpinLimit = 1u << 20;
constexpr int kLookWindow = 8;
// Column exchange: at most kXchgTiles tiles; above 64 tiles a digit column of
// the tiles' counts is scanned by 256 threads, kXchgCols columns a block at once.
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

// A tile's published count of one digit (flag and value in one word),
// waited for with a bounded spin: a stall raises MH_EHIP and reads 0.
__device__ __forceinline__ uint32_t xchg_wait_count(uint64_t* cw, int32_t* err) {
    uint32_t spins = 0;
    for (;;) {
        const uint64_t w = __hip_atomic_load(cw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (w & ~0xFFFFFFFFull) return (uint32_t)w;
        if (++spins > kSpinLimit) {
            raise_status(err, MH_EHIP);
            return 0u;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Node parameters whose sort keys a first pass will make (x null: none), and
// where the least and largest key (high halves) of each tile go.
struct KeySpan {
    const double* x = nullptr;
    const double* y = nullptr;
    int64_t n = 0;
    uint64_t* part = nullptr;  // tile t: largest << 32 | least; part[tiles + t]: the tile's column mass
    int64_t tiles = 0;
};

// Zeroes three ranges of u64 words (any may be empty); with a key span, block
// t < tiles also writes the range of tile t's keys and the sum of their column
// masses floor(z 2^32) (the total over all tiles does not depend on the
// order; the grid covers both jobs).
__global__ __launch_bounds__(kSortThreads) void k_zero_u64(ZeroRange a, ZeroRange b, ZeroRange c, KeySpan ks) {
    const int64_t stride = (int64_t)gridDim.x * kSortThreads;
    const int64_t t = (int64_t)blockIdx.x * kSortThreads + threadIdx.x;
    for (int64_t i = t; i < a.n; i += stride) a.p[i] = 0;
    for (int64_t i = t; i < b.n; i += stride) b.p[i] = 0;
    for (int64_t i = t; i < c.n; i += stride) c.p[i] = 0;
    const int64_t base = (int64_t)blockIdx.x * kTileKeys;
    if (!ks.x || base >= ks.n) return;  // uniform over the block
    __shared__ uint32_t s_mn[kSortWaves], s_mx[kSortWaves];
    __shared__ uint64_t s_ms[kSortWaves];
    uint32_t mn = ~0u, mx = 0u;
    uint64_t ms = 0;
#pragma unroll
    for (int q = 0; q < kKeysPerLane; ++q) {
        const int64_t i = base + (int64_t)q * kSortThreads + threadIdx.x;
        if (i < ks.n) {
            bool ok;  // an invalid node sorts as z = 0, as in the first pass
            const double z = node_z(ks.x[i], ks.y != nullptr, ks.y ? ks.y[i] : 0.0, &ok);
            const uint32_t h = (uint32_t)(desc_key(z) >> 32);
            mn = h < mn ? h : mn;
            mx = h > mx ? h : mx;
            ms += mass_q(z);
        }
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t on = __shfl_xor(mn, d, kWave), ox = __shfl_xor(mx, d, kWave);
        mn = on < mn ? on : mn;
        mx = ox > mx ? ox : mx;
        ms += __shfl_xor(ms, d, kWave);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        s_mn[wave] = mn;
        s_mx[wave] = mx;
        s_ms[wave] = ms;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kSortWaves; ++w) {
            mn = s_mn[w] < mn ? s_mn[w] : mn;
            mx = s_mx[w] > mx ? s_mx[w] : mx;
            ms += s_ms[w];
        }
        ks.part[blockIdx.x] = ((uint64_t)mx << 32) | mn;
        ks.part[ks.tiles + blockIdx.x] = ms;
    }
}

// Radix passes that keys spanning [0, spread] need (8 bits each; one at least).
__device__ __forceinline__ uint32_t passes_for(uint32_t spread) {
    return spread < (1u << 8) ? 1u : spread < (1u << 16) ? 2u : spread < (1u << 24) ? 3u : 4u;
}

// FROMX (first pass, column exchange only): the pass prepares its own keys from
// the parameters x (and y) as the key-preparation kernel would, adds the digit
// histograms of the later passes to hist_all, and takes its own digit totals
// from the exchange (column owners publish them in dtot) instead of ghist.
// It also reduces the tiles' key ranges (part) to the least key and the
// spread, sorts every key less the least (so keys spanning 24 bits need 3
// passes, not 4), and writes meta = {least key, passes}.  With meta (passes
// after such a first pass), a pass beyond the count returns at once, and with
// an odd count every pass swaps its input and output arrays, so that the last
// pass still writes the arrays the caller passed as the sort's input.
template <bool XCHG, bool FROMX>
__global__ __launch_bounds__(kSortThreads) void k_onesweep(const uint32_t* kin, const uint64_t* vin, uint32_t* kout,
                                                           uint64_t* vout,
                                                           int64_t n, int shift, const uint32_t* __restrict__ ghist,
                                                           uint64_t* status, uint32_t* ticket, bool use_ticket,
                                                           int32_t* err, const double* __restrict__ x,
                                                           const double* __restrict__ y,
                                                           uint32_t* __restrict__ hist_all, uint64_t* dtot,
                                                           uint32_t* meta, const uint64_t* __restrict__ part) {
    static_assert(!FROMX || XCHG, "a pass preparing its keys takes its digit totals from the exchange");
    if (!FROMX && meta) {
        const uint32_t npass = meta[1];
        if ((uint32_t)(shift >> 3) >= npass) return;  // the whole grid: nothing left to sort
        if (npass & 1u) {
            const uint32_t* kt = kin;
            kin = kout;
            kout = const_cast<uint32_t*>(kt);
            const uint64_t* vt = vin;
            vin = vout;
            vout = const_cast<uint64_t*>(vt);
        }
    }
    __shared__ uint32_t s_keys[kTileKeys];
    __shared__ uint64_t s_vals[kTileKeys];
    __shared__ uint32_t cnt[kSortWaves][kRadix];
    __shared__ uint32_t s_bstart[kRadix];
    __shared__ uint32_t s_goff[kRadix];
    __shared__ uint32_t s_scan[kSortWaves];
    __shared__ uint32_t s_later[FROMX ? (kPasses - 1) * kRadix : 1];
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_kmin[FROMX ? kSortWaves : 1], s_kmax[FROMX ? kSortWaves : 1];

    // Tiles are taken in ticket order unless the whole grid is resident at once
    // (then every block runs concurrently and its index serves, sparing 1 atomic
    // per block on one address).
    if (threadIdx.x == 0) s_tile = use_ticket ? atomicAdd(ticket, 1u) : blockIdx.x;
    for (int i = threadIdx.x; i < kSortWaves * kRadix; i += kSortThreads) (&cnt[0][0])[i] = 0;
    if (FROMX)
        for (int i = threadIdx.x; i < (kPasses - 1) * kRadix; i += kSortThreads) s_later[i] = 0;
    __syncthreads();
    const int64_t tile = s_tile;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t tbase = tile * kTileKeys;
    const int64_t base = tbase + (int64_t)wave * kWaveKeys;
    const uint64_t lt = lanemask_lt();

    // rank every key among the wave's keys with the same digit
    uint32_t k[kKeysPerLane];
    uint64_t v[kKeysPerLane];
    uint32_t rank[kKeysPerLane];
    // all loads first: the ranking below orders LDS accesses with wave barriers,
    // which the compiler will not move loads across.  With them, this digit's
    // count over all keys (the histogram copies): its latency hides under the
    // keys' instead of stalling the digit step after the ranking.
    uint32_t hc[kHistCopies];
#pragma unroll
    for (int c = 0; c < kHistCopies; ++c)
        hc[c] = (!FROMX && threadIdx.x < kRadix) ? ghist[c * kPasses * kRadix + threadIdx.x] : 0u;
    if (FROMX) {
        double xv[kKeysPerLane], yv[kKeysPerLane];
#pragma unroll
        for (int r = 0; r < kKeysPerLane; ++r) {
            const int64_t i = base + (int64_t)r * kWave + lane;
            xv[r] = i < n ? x[i] : 0.0;
            yv[r] = (y && i < n) ? y[i] : 0.0;
        }
        // least and largest key over all tiles (the zeroing kernel's ranges)
        {
            const uint64_t pw = threadIdx.x < gridDim.x ? part[threadIdx.x] : 0x00000000FFFFFFFFull;
            uint32_t mn = (uint32_t)pw, mx = (uint32_t)(pw >> 32);
#pragma unroll
            for (int dd = 1; dd < kWave; dd <<= 1) {
                const uint32_t on = __shfl_xor(mn, dd, kWave), ox = __shfl_xor(mx, dd, kWave);
                mn = on < mn ? on : mn;
                mx = ox > mx ? ox : mx;
            }
            if (lane == 0) {
                s_kmin[wave] = mn;
                s_kmax[wave] = mx;
            }
        }
        __syncthreads();
        uint32_t kmin = s_kmin[0], kmax = s_kmax[0];
#pragma unroll
        for (int w = 1; w < kSortWaves; ++w) {
            kmin = s_kmin[w] < kmin ? s_kmin[w] : kmin;
            kmax = s_kmax[w] > kmax ? s_kmax[w] : kmax;
        }
        const uint32_t npass = passes_for(kmax - kmin);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            meta[0] = kmin;
            meta[1] = npass;
        }
        if (npass & 1u) {  // the last pass writes the input arrays
            kout = const_cast<uint32_t*>(kin);
            vout = const_cast<uint64_t*>(vin);
        }
        bool bad = false;
#pragma unroll
        for (int r = 0; r < kKeysPerLane; ++r) {
            const int64_t i = base + (int64_t)r * kWave + lane;
            const bool valid = i < n;
            k[r] = 0u;
            v[r] = 0ull;
            if (valid) {
                bool ok;
                const double z = node_z(xv[r], y != nullptr, yv[r], &ok);
                bad = bad || !ok;
                split_key(z, i, &k[r], &v[r]);
                k[r] -= kmin;
            }
            count_key_digits(s_later, k[r], valid, 1, kPasses);
        }
        if (bad) raise_status(err, MH_EINVAL);
    } else {
#pragma unroll
        for (int r = 0; r < kKeysPerLane; ++r) {
            const int64_t i = base + (int64_t)r * kWave + lane;
            const bool valid = i < n;
            k[r] = valid ? kin[i] : 0u;
            v[r] = valid ? vin[i] : 0ull;
        }
    }
#pragma unroll
    for (int r = 0; r < kKeysPerLane; ++r) {
        const int64_t i = base + (int64_t)r * kWave + lane;
        const bool valid = i < n;
        const uint32_t d = (k[r] >> shift) & (kRadix - 1);
        const uint64_t m = match_digit(d, valid);
        const uint32_t prior = cnt[wave][d];
        rank[r] = prior + (uint32_t)__popcll(m & lt);
        __builtin_amdgcn_wave_barrier();
        if (valid && (m & lt) == 0) cnt[wave][d] = prior + (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    if (FROMX) {
        // the later passes' histograms, into this block's copy
        uint32_t* copy = hist_all + ((blockIdx.x % kHistCopies) * kPasses + 1) * kRadix;
        for (int i = threadIdx.x; i < (kPasses - 1) * kRadix; i += kSortThreads)
            if (s_later[i]) atomicAdd(&copy[i], s_later[i]);
    }

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
        for (int c = 0; c < kHistCopies; ++c) dtotal += hc[c];
    }
    const uint32_t bstart = block_exclusive(total, s_scan);
    uint32_t dstart = FROMX ? 0u : block_exclusive(dtotal, s_scan);
    uint32_t excl = 0;
    if (XCHG) {
        // Every tile is resident (at most kXchgTiles): instead of a chain of
        // look-backs, the blocks scan the digit columns over all tiles'
        // published counts, one thread per tile of a column: block b takes
        // columns b, b + G, b + 2G, ... (G blocks), several at once.  Each
        // column's scan writes every tile the count of that digit in the
        // tiles before it (flag 2 over the count word, which only this block
        // reads) and, when the pass has no digit totals of its own, the
        // column's total to dtot; then every tile reads its 256 words back.
        // Two round trips per pass, however few the tiles.
        const int nt = (int)gridDim.x;
        if (nt > kWave) {
            // a column by 256 threads (4 waves), 4 columns at once
            const int tcol = threadIdx.x & (kXchgTiles - 1);  // this thread's tile in the column
            for (int c0 = blockIdx.x; c0 < kRadix; c0 += kXchgCols * nt) {
                const int col = c0 + (int)(threadIdx.x / kXchgTiles) * nt;
                const bool mine = tcol < nt && col < kRadix;
                uint64_t* cw = status + (int64_t)tcol * kRadix + col;
                const uint32_t c = mine ? xchg_wait_count(cw, err) : 0u;
                // exclusive scan over each column's 256 threads (4 waves)
                const uint32_t inc = wave_inclusive_scan(c);
                if (lane == 63) s_scan[wave] = inc;
                __syncthreads();
                const int w0 = wave & ~(kXchgTiles / kWave - 1);
                uint32_t before = inc - c;
                for (int w = w0; w < wave; ++w) before += s_scan[w];
                if (mine) __hip_atomic_store(cw, kFlagPrefix | before, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (FROMX && tcol == 0 && col < kRadix) {
                    uint32_t coltotal = 0;
                    for (int w = w0; w < w0 + kXchgTiles / kWave; ++w) coltotal += s_scan[w];
                    __hip_atomic_store(dtot + col, kFlagPrefix | coltotal, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                }
                __syncthreads();
            }
        } else {
            // at most 64 tiles: a column by tpc lanes of a wave (the tile count
            // rounded up to a power of two), kSortThreads / tpc columns at once
            int lg = 0;
            while ((1 << lg) < nt) ++lg;
            const int tpc = 1 << lg;
            const int tcol = threadIdx.x & (tpc - 1);
            for (int c0 = blockIdx.x; c0 < kRadix; c0 += (kSortThreads >> lg) * nt) {
                const int col = c0 + (int)(threadIdx.x >> lg) * nt;
                const bool mine = tcol < nt && col < kRadix;
                uint64_t* cw = status + (int64_t)tcol * kRadix + col;
                const uint32_t c = mine ? xchg_wait_count(cw, err) : 0u;
                uint32_t inc = c;  // inclusive scan within each group of tpc lanes
                for (int dd = 1; dd < tpc; dd <<= 1) {
                    const uint32_t u = __shfl_up(inc, (unsigned)dd, tpc);
                    if (tcol >= dd) inc += u;
                }
                if (mine) __hip_atomic_store(cw, kFlagPrefix | (inc - c), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (FROMX) {
                    const uint32_t coltotal = __shfl(inc, lane | (tpc - 1), kWave);
                    if (tcol == 0 && col < kRadix)
                        __hip_atomic_store(dtot + col, kFlagPrefix | coltotal, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        if (dig) {
            uint32_t spins = 0;
            bool need_excl = true, need_total = FROMX;
            while (need_excl || need_total) {
                if (need_excl) {
                    const uint64_t w = __hip_atomic_load(st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if ((w & ~0xFFFFFFFFull) == kFlagPrefix) {
                        excl = (uint32_t)w;  // earlier tiles' keys with digit d
                        need_excl = false;
                    }
                }
                if (FROMX && need_total) {
                    const uint64_t w = __hip_atomic_load(dtot + d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if ((w & ~0xFFFFFFFFull) == kFlagPrefix) {
                        dtotal = (uint32_t)w;  // keys with digit d over all tiles
                        need_total = false;
                    }
                }
                if (!(need_excl || need_total)) break;
                if (++spins > kSpinLimit) {
                    raise_status(err, MH_EHIP);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        if (FROMX) dstart = block_exclusive(dtotal, s_scan);
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
            const uint32_t dd = (k[r] >> shift) & (kRadix - 1);
            const uint32_t lp = s_bstart[dd] + cnt[wave][dd] + rank[r];
            s_keys[lp] = k[r];
            s_vals[lp] = v[r];
        }
    }
    __syncthreads();
    const int64_t cnt_tile = (n - tbase) < kTileKeys ? (n - tbase) : kTileKeys;
    for (int i = threadIdx.x; i < cnt_tile; i += kSortThreads) {
        const uint32_t key = s_keys[i];
        const uint32_t dd = (key >> shift) & (kRadix - 1);
        const uint32_t pos = s_goff[dd] + (uint32_t)i;
        if (pos < (uint64_t)n) {  // always, unless a look-back gave up (then the error is raised)
            // device-scope stores: written through to the device's coherence
            // point, so the kernel's end has no dirty L2 lines to write back
            // (the next pass starts ~1.5 us sooner after 12 MB)
            __hip_atomic_store(&kout[pos], key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&vout[pos], s_vals[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ------------------------------------------------------------------ tie runs
// First index in [0, r] whose key equals hi[r] (hi ascending), found by the
// whole wave (r the same in every lane): lane l first probes r - 64 * 2^l,
// which brackets the start within a factor of two of its distance; then each
// round's 63 evenly spaced probes narrow the bracket 64-fold.  A start 3,000
// ranks back costs 3 rounds of loads where a one-lane search takes ~18.
__device__ int64_t wave_run_start(const uint32_t* __restrict__ hi, int64_t r) {
    const int lane = threadIdx.x & 63;
    const uint32_t h = hi[r];
    int64_t lo, up;  // the start is in (lo, up]: hi[lo] < h (or lo = -1), hi[up] == h
    {
        const int sh = lane < 40 ? lane : 40;
        const int64_t p = r - ((int64_t)64 << sh);
        const bool before = p < 0 || hi[p] < h;  // true from some lane on (lane 40 at the latest)
        const int l = __ffsll((unsigned long long)__ballot(before)) - 1;
        lo = r - ((int64_t)64 << l);
        if (lo < 0) lo = -1;
        up = l == 0 ? r : r - ((int64_t)64 << (l - 1));
    }
    while (up - lo > 1) {
        const int64_t step = (up - lo + 63) / 64;
        const int64_t p = lo + step * (lane + 1);
        const bool before = p < up && hi[p] < h;  // a prefix of the lanes
        const int cnt = __popcll(__ballot(before));
        const int64_t nup = lo + step * (cnt + 1);
        lo += step * cnt;
        up = nup < up ? nup : up;
    }
    return up;
}

// ------------------------------------------------------------------ run repair
constexpr int kFixThreads = 1024;
constexpr int kFixWaves = kFixThreads / kWave;
constexpr int kFixLds = 4096;  // runs up to this long are sorted in LDS (block_lds_run), longer ones by block_lsd_run
constexpr int kFixWaveRun = 256;  // runs up to this long are sorted by one wave (wave_sort_run)
// A block of k_fix_runs takes chunks of ranks: small chunks spread the runs
// longer than a wave (each sorted by the whole block) over many blocks.  Chunks
// are 1024 ranks where every chunk then has a block of its own, else 2048
// (fewer chunks a block: each costs its barriers).
constexpr int kFixChunk = 2048;  // the largest chunk
constexpr int kFixClaims = kFixChunk / 2;  // runs with a descent among 2048 ranks: at most 1024
constexpr int kFixList = 64;  // runs of more than kFixWaveRun ranks claimed by a chunk of 2048: at most 9

// Sorts up to 64 values held one per lane (absent lanes hold ~0).
__device__ __forceinline__ uint64_t wave_bitonic(uint64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint64_t u = __shfl_xor(v, j, kWave);
            const bool up = (lane & k) == 0;
            const bool low = (lane & j) == 0;
            v = (low == up) ? (u < v ? u : v) : (u > v ? u : v);
        }
    }
    return v;
}

// First index >= a + 1 whose hi differs from hi[a] (n if none), searched by
// the whole block: 1024 probes per round, each round narrowing the step.
__device__ int64_t block_run_end(const uint32_t* __restrict__ hi, int64_t n, int64_t a, int64_t* s_pos) {
    const uint32_t h = hi[a];
    int64_t lo = a;  // hi[lo] == h
    int64_t up = n;  // first index known to differ (or n)
    while (up - lo > 1) {
        const int64_t span = up - lo;
        const int64_t step = (span + kFixThreads - 1) / kFixThreads;
        const int64_t p = lo + (int64_t)(threadIdx.x + 1) * step;
        const bool differs = p < up && hi[p] != h;
        if (threadIdx.x == 0) *s_pos = up;
        __syncthreads();
        if (differs) atomicMin((unsigned long long*)s_pos, (unsigned long long)p);
        __syncthreads();
        const int64_t first = *s_pos;  // first probe that differs, else up
        __syncthreads();
        if (step == 1) return first;
        up = first;
        lo = first - step > lo ? first - step : lo;
    }
    return up;
}

// Stable LSD sort of pay[a, b) by its high 32 bits through alt[a, b), by one
// block; the result ends in pay.  The digits are those of the high word minus
// its least value in the run, 8 bits a pass, as many passes as the spread needs
// (values of a run of near-equal keys lie a few units apart, so one pass, even
// where they straddle a byte boundary).  One read counts the digits of every
// pass, and a pass whose digit is the same for every value moves nothing.
__device__ void block_lsd_run(uint64_t* __restrict__ pay, uint64_t* __restrict__ alt, int64_t a, int64_t b,
                              uint32_t* s_cnt /* kFixWaves * 256 */, uint32_t* s_hist /* 4 * 256 */,
                              uint32_t* s_off /* 256 */, uint32_t* s_scan /* kFixWaves */,
                              uint32_t* s_flag /* 4 */) {
    __shared__ uint32_t s_mm[2];  // least and largest high word of the run
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t lt = lanemask_lt();
    const uint32_t len = (uint32_t)(b - a);
    for (int i = threadIdx.x; i < 4 * 256; i += kFixThreads) s_hist[i] = 0;
    if (threadIdx.x < 4) s_flag[threadIdx.x] = 0;  // one flag per pass: no reset races a late reader
    if (threadIdx.x == 0) {
        s_mm[0] = ~0u;
        s_mm[1] = 0u;
    }
    __syncthreads();
    uint32_t mn = ~0u, mx = 0u;
    for (int64_t i = a + threadIdx.x; i < b; i += kFixThreads) {
        const uint32_t h = (uint32_t)(pay[i] >> 32);
        mn = h < mn ? h : mn;
        mx = h > mx ? h : mx;
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t on = __shfl_xor(mn, d, kWave), ox = __shfl_xor(mx, d, kWave);
        mn = on < mn ? on : mn;
        mx = ox > mx ? ox : mx;
    }
    if (lane == 0) {
        atomicMin(&s_mm[0], mn);
        atomicMax(&s_mm[1], mx);
    }
    __syncthreads();
    const uint32_t base = s_mm[0];
    const uint32_t spread = s_mm[1] - base;
    const int npass = spread == 0 ? 0 : (spread >> 8) == 0 ? 1 : (spread >> 16) == 0 ? 2 : (spread >> 24) == 0 ? 3 : 4;
    for (int64_t i = a + threadIdx.x; i < b; i += kFixThreads) {
        const uint32_t d = (uint32_t)(pay[i] >> 32) - base;
        for (int pass = 0; pass < npass; ++pass) atomicAdd(&s_hist[pass * 256 + ((d >> (8 * pass)) & 255u)], 1u);
    }
    __syncthreads();
    uint64_t* src = pay;
    uint64_t* dst = alt;
    for (int pass = 0; pass < npass; ++pass) {
        const int shift = 8 * pass;
        // a pass with one digit for all values keeps the order as it is
        if (threadIdx.x < 256 && s_hist[pass * 256 + threadIdx.x] == len) s_flag[pass] = 1;
        __syncthreads();
        if (s_flag[pass]) continue;  // the same for every thread of the block
        const uint32_t c = threadIdx.x < 256 ? s_hist[pass * 256 + threadIdx.x] : 0u;
        const uint32_t ex = block_exclusive(c, s_scan);
        if (threadIdx.x < 256) s_off[threadIdx.x] = ex;
        __syncthreads();
        // chunks of 4096 in order; each wave ranks 256 consecutive values stably
        for (int64_t cb = a; cb < b; cb += kTileKeys) {
            for (int i = threadIdx.x; i < kFixWaves * 256; i += kFixThreads) s_cnt[i] = 0;
            __syncthreads();
            const int64_t wb = cb + (int64_t)wave * kWaveKeys;
            uint64_t v[kKeysPerLane];
            uint32_t rk[kKeysPerLane];
#pragma unroll
            for (int r = 0; r < kKeysPerLane; ++r) {
                const int64_t i = wb + (int64_t)r * kWave + lane;
                v[r] = i < b ? src[i] : 0ull;
            }
#pragma unroll
            for (int r = 0; r < kKeysPerLane; ++r) {
                const int64_t i = wb + (int64_t)r * kWave + lane;
                const bool valid = i < b;
                const uint32_t dg = (((uint32_t)(v[r] >> 32) - base) >> shift) & 255u;
                const uint64_t m = match_digit(dg, valid);
                const uint32_t prior = s_cnt[wave * 256 + dg];
                rk[r] = prior + (uint32_t)__popcll(m & lt);
                __builtin_amdgcn_wave_barrier();
                if (valid && (m & lt) == 0) s_cnt[wave * 256 + dg] = prior + (uint32_t)__popcll(m);
                __builtin_amdgcn_wave_barrier();
            }
            __syncthreads();
            // per digit: waves' offsets inside the chunk, then advance the run offset
            if (threadIdx.x < 256) {
                uint32_t run = 0;
                for (int w = 0; w < kFixWaves; ++w) {
                    const uint32_t t = s_cnt[w * 256 + threadIdx.x];
                    s_cnt[w * 256 + threadIdx.x] = run + s_off[threadIdx.x];
                    run += t;
                }
                s_off[threadIdx.x] += run;
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < kKeysPerLane; ++r) {
                const int64_t i = wb + (int64_t)r * kWave + lane;
                if (i < b) {
                    const uint32_t dg = (((uint32_t)(v[r] >> 32) - base) >> shift) & 255u;
                    dst[a + s_cnt[wave * 256 + dg] + rk[r]] = v[r];
                }
            }
            __syncthreads();
        }
        uint64_t* t = src;
        src = dst;
        dst = t;
    }
    if (src != pay) {  // an odd number of passes moved the values: back to pay
        for (int64_t i = a + threadIdx.x; i < b; i += kFixThreads) pay[i] = src[i];
        __syncthreads();
    }
}

// Sorts up to 64 K values held K a lane (element k * 64 + lane in v[k]; absent
// ones hold ~0) ascending: a bitonic network over 64 K elements, partners 64 or
// more apart in two registers of the same lane, nearer ones in the same
// register of two lanes (shuffles).  Registers only: no LDS.
template <int K>
__device__ __forceinline__ void wave_bitonic_regs(uint64_t (&v)[K]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int s = 2; s <= K * kWave; s <<= 1) {
#pragma unroll
        for (int j = s >> 1; j > 0; j >>= 1) {
            if (j >= kWave) {
                const int kj = j / kWave;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    if (k & kj) continue;  // the pair (k, k + kj)
                    const bool up = ((k * kWave + lane) & s) == 0;
                    const uint64_t lo = v[k], hi2 = v[k + kj];
                    const bool swap = up ? lo > hi2 : lo < hi2;
                    v[k] = swap ? hi2 : lo;
                    v[k + kj] = swap ? lo : hi2;
                }
            } else {
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const uint64_t u = __shfl_xor(v[k], j, kWave);
                    const bool up = ((k * kWave + lane) & s) == 0;
                    const bool low = (lane & j) == 0;
                    v[k] = (low == up) ? (u < v[k] ? u : v[k]) : (u > v[k] ? u : v[k]);
                }
            }
        }
    }
}

// Loads the len values pay[a, a + len) K a lane, sorts them by the whole
// 64-bit payload (in a run of equal high halves the payload's low word rises
// with the input order, so this is the stable order by its high word) and
// writes them back.
template <int K>
__device__ __forceinline__ void wave_sort_run(uint64_t* __restrict__ pay, int64_t a, int len) {
    const int lane = threadIdx.x & 63;
    uint64_t v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = k * kWave + lane;
        v[k] = i < len ? pay[a + i] : ~0ull;
    }
    wave_bitonic_regs<K>(v);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = k * kWave + lane;
        if (i < len) pay[a + i] = v[k];
    }
}

// Length of the run of equal hi (= h) that starts at a, if it ends within
// kFixWaveRun ranks of a (its first 64 ranks are known to be in it), else -1;
// the same in every lane of the wave.
__device__ int wave_run_length(const uint32_t* __restrict__ hi, int64_t n, int64_t a, uint32_t h) {
    const int lane = threadIdx.x & 63;
    for (int k = 1; k <= kFixWaveRun / kWave; ++k) {
        const int i = k * kWave + lane;
        const bool past = i <= kFixWaveRun && (a + i >= n || hi[a + i] != h);
        const uint64_t m = __ballot(past);
        if (m) return k * kWave + __ffsll((unsigned long long)m) - 1;
    }
    return -1;
}

// Stable sort by the high 32 bits of the run of equal hi that starts at a, in
// LDS, if the run ends within kFixLds ranks of a; returns false (nothing
// written) if it is longer.  The window is read 1024 ranks a round until a
// round finds the run's end, loading the values on the way; the digits are
// those of the high word minus its least value
// in the run, 8 bits a pass, as many passes as the spread needs (one for a run
// of near-equal keys); each pass ranks values stably as the block LSD does,
// from s_a into s_b; one write returns the result.
__device__ bool block_lds_run(const uint32_t* __restrict__ hi, uint64_t* __restrict__ pay, int64_t n, int64_t a,
                              uint64_t* s_a /* kFixLds */, uint64_t* s_b /* kFixLds */,
                              uint32_t* s_cnt /* kFixWaves * 256 */, uint32_t* s_scan /* kFixWaves */,
                              uint32_t* s_misc /* 3 */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t lt = lanemask_lt();
    const int win = n - a < kFixLds ? (int)(n - a) : kFixLds;
    const uint32_t h0 = hi[a];
    if (threadIdx.x == 0) {
        s_misc[0] = (uint32_t)win;  // first rank of the window (from a) whose hi differs
        s_misc[1] = ~0u;
        s_misc[2] = 0u;
    }
    __syncthreads();
    // the window in rounds of one rank per thread, until a round sees the run end
    for (int i0 = 0; i0 < win; i0 += kFixThreads) {
        const int i = i0 + threadIdx.x;
        const bool in = i < win;
        const uint64_t m = __ballot(in && hi[a + i] != h0);
        // one atomic per wave: its first rank past the run
        if (m && lane == __ffsll((unsigned long long)m) - 1) atomicMin(&s_misc[0], (uint32_t)i);
        if (in) s_a[i] = pay[a + i];
        __syncthreads();
        const bool found = s_misc[0] < (uint32_t)win;
        __syncthreads();  // every thread has read s_misc[0] before the next round may lower it
        if (found) break;
    }
    // a run that fills the window may go on past it
    const bool longer = a + win < n && hi[a + win] == h0;
    const int len = (int)s_misc[0];
    if (len == win && longer) return false;  // the same for every thread of the block
    uint32_t mn = ~0u, mx = 0u;
    for (int i = threadIdx.x; i < len; i += kFixThreads) {
        const uint32_t h = (uint32_t)(s_a[i] >> 32);
        mn = h < mn ? h : mn;
        mx = h > mx ? h : mx;
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t on = __shfl_xor(mn, d, kWave), ox = __shfl_xor(mx, d, kWave);
        mn = on < mn ? on : mn;
        mx = ox > mx ? ox : mx;
    }
    if (lane == 0) {
        atomicMin(&s_misc[1], mn);
        atomicMax(&s_misc[2], mx);
    }
    __syncthreads();
    const uint32_t base = s_misc[1];
    const uint32_t spread = s_misc[2] - base;
    const int npass = spread == 0 ? 0 : (spread >> 8) == 0 ? 1 : (spread >> 16) == 0 ? 2 : (spread >> 24) == 0 ? 3 : 4;
    static_assert(kFixLds <= kFixWaves * kWaveKeys, "one round of the block ranks the whole window");
    const int wb = wave * kWaveKeys;
    const int nw = (len + kWaveKeys - 1) / kWaveKeys;  // waves that hold values
    for (int pass = 0; pass < npass; ++pass) {
        const int shift = 8 * pass;
        for (int i = threadIdx.x; i < nw * 256; i += kFixThreads) s_cnt[i] = 0;
        __syncthreads();
        uint64_t v[kKeysPerLane];
        uint32_t dg[kKeysPerLane], rk[kKeysPerLane];
#pragma unroll
        for (int r = 0; r < kKeysPerLane; ++r) {
            const int i = wb + r * kWave + lane;
            const bool valid = i < len;
            v[r] = valid ? s_a[i] : 0ull;
            dg[r] = ((((uint32_t)(v[r] >> 32)) - base) >> shift) & 255u;
            const uint64_t m = match_digit(dg[r], valid);
            const uint32_t prior = s_cnt[wave * 256 + dg[r]];
            rk[r] = prior + (uint32_t)__popcll(m & lt);
            __builtin_amdgcn_wave_barrier();
            if (valid && (m & lt) == 0) s_cnt[wave * 256 + dg[r]] = prior + (uint32_t)__popcll(m);
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        // per digit: the waves' counts become running offsets, then the digit's start is added
        uint32_t tot = 0;
        if (threadIdx.x < 256) {
            for (int w = 0; w < nw; ++w) {
                const uint32_t t = s_cnt[w * 256 + threadIdx.x];
                s_cnt[w * 256 + threadIdx.x] = tot;
                tot += t;
            }
        }
        const uint32_t start = block_exclusive(tot, s_scan);
        if (threadIdx.x < 256)
            for (int w = 0; w < nw; ++w) s_cnt[w * 256 + threadIdx.x] += start;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kKeysPerLane; ++r) {
            const int i = wb + r * kWave + lane;
            if (i < len) s_b[s_cnt[wave * 256 + dg[r]] + rk[r]] = v[r];
        }
        __syncthreads();
        uint64_t* t = s_a;
        s_a = s_b;
        s_b = t;
    }
    for (int i = threadIdx.x; i < len; i += kFixThreads) pay[a + i] = s_a[i];
    __syncthreads();
    return true;
}

// Finds and sorts by pay every run of equal hi whose pay descends somewhere.
// Blocks take chunks of 2048 ranks; each wave looks at 64 ranks at a time, and
// the first descent it sees in a run claims the run by setting the run's
// start bit in `claims` (zero at launch) with an atomic OR: the one block that
// sets it sorts the whole run, wherever it lies.  A run without a descent is
// never claimed, however long; while its owner sorts a run, other blocks may
// read that run's values mid-sort, which can only make them try the claim
// again, and fail.  The block's claimed runs are sorted by single waves at
// once up to kFixWaveRun ranks (bitonic over the lanes below 64, else
// wave_sort_run: a bitonic network in registers), longer ones by the whole
// block: in LDS up to kFixLds
// (block_lds_run), else by block_lsd_run through alt.
__global__ __launch_bounds__(kFixThreads) void k_fix_runs(const uint32_t* __restrict__ hi,
                                                          uint64_t* __restrict__ pay, uint64_t* __restrict__ alt,
                                                          int64_t n, uint32_t* __restrict__ claims, int32_t chunk) {
    __shared__ uint64_t s_run[kFixLds];
    __shared__ uint64_t s_run2[kFixLds];
    __shared__ uint32_t s_wcnt[kFixWaves * 256];
    __shared__ uint32_t s_misc[3];
    __shared__ int64_t s_claim[kFixClaims];
    __shared__ int64_t s_list[kFixList];
    __shared__ int64_t s_pos;
    __shared__ uint32_t s_nclaim, s_nlist;
    __shared__ uint32_t s_off[256];
    __shared__ uint32_t s_scan[kFixWaves];
    __shared__ uint32_t s_flag[4];
    static_assert(kFixWaves * 256 + 4 * 256 <= 2 * kFixLds, "digit counts fit in the run buffer");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t c0 = (int64_t)blockIdx.x * chunk; c0 < n; c0 += (int64_t)gridDim.x * chunk) {
        const int64_t c1 = c0 + chunk < n ? c0 + chunk : n;
        if (threadIdx.x == 0) {
            s_nclaim = 0;
            s_nlist = 0;
        }
        __syncthreads();
        // 1. descents, and the claims of their runs
        for (int64_t wbase = c0 + (int64_t)wave * kWave; wbase < c1; wbase += (int64_t)kFixWaves * kWave) {
            const int64_t r = wbase + lane;
            bool eq = false, desc = false;
            if (r > 0 && r < c1) {
                eq = hi[r - 1] == hi[r];
                if (eq) desc = pay[r - 1] > pay[r];
            }
            const uint64_t dm = __ballot(desc);
            if (dm == 0) continue;
            const uint64_t eqm = __ballot(eq);
            const uint64_t starts = ~eqm & ~1ull;  // run starts inside the wave (lane 0 aside)
            // the wave's first segment (lanes before the first start) continues a
            // run from before the wave: if it holds a descent, the wave finds that
            // run's start together
            const bool cont = (eqm & 1ull) != 0;
            const uint64_t first_seg = starts ? (1ull << (__ffsll((unsigned long long)starts) - 1)) - 1 : ~0ull;
            int64_t a_cont = wbase;
            if (cont && (dm & first_seg)) a_cont = wave_run_start(hi, wbase);
            if (desc) {
                const uint64_t le = lanemask_lt();
                const uint64_t before = starts & le;
                const int st = before ? 63 - __clzll((long long)before) : 0;  // segment's first lane in the wave
                const uint64_t seg_desc = dm & le & ~((1ull << st) - 1);   // earlier descents in the segment
                if (seg_desc == 0) {
                    const int64_t a = before ? wbase + st : a_cont;
                    const uint32_t mask = 1u << (a & 31);
                    if ((atomicOr(&claims[a >> 5], mask) & mask) == 0) s_claim[atomicAdd(&s_nclaim, 1u)] = a;
                }
            }
        }
        __syncthreads();
        // 2. the claimed runs: up to kFixWaveRun ranks by a wave each, longer ones listed
        const uint32_t ncl = s_nclaim;
        for (uint32_t q = (uint32_t)wave; q < ncl; q += kFixWaves) {
            const int64_t a = s_claim[q];
            const uint32_t h = hi[a];
            const int64_t r = a + lane;
            const bool in = r < n && hi[r] == h;
            const uint64_t inm = __ballot(in);
            if (inm == ~0ull) {
                const int len = wave_run_length(hi, n, a, h);
                if (len < 0) {
                    if (lane == 0) {
                        const uint32_t slot = atomicAdd(&s_nlist, 1u);
                        if (slot < kFixList) s_list[slot] = a;
                    }
                } else if (len <= 2 * kWave) {
                    wave_sort_run<2>(pay, a, len);
                } else {
                    wave_sort_run<4>(pay, a, len);
                }
            } else {
                // run of length < 64: lanes below the first differing lane
                const int len = __ffsll((unsigned long long)~inm) - 1;
                const bool mine = lane < len;
                uint64_t v = mine ? pay[r] : ~0ull;
                v = wave_bitonic(v);
                if (mine) pay[r] = v;
            }
        }
        __syncthreads();
        const uint32_t nl = s_nlist < kFixList ? s_nlist : kFixList;
        for (uint32_t q = 0; q < nl; ++q) {
            const int64_t a = s_list[q];
            if (block_lds_run(hi, pay, n, a, s_run, s_run2, s_wcnt, s_scan, s_misc)) continue;
            const int64_t b = block_run_end(hi, n, a, &s_pos);
            block_lsd_run(pay, alt, a, b, reinterpret_cast<uint32_t*>(s_run),
                          reinterpret_cast<uint32_t*>(s_run) + kFixWaves * 256, s_off, s_scan, s_flag);
        }
        __syncthreads();
    }
}

int64_t sort_blocks(int64_t n) { return (n + kTileKeys - 1) / kTileKeys; }
int64_t tie_words(int64_t n) { return ((n + 31) >> 5) + 2; }  // u32 bitmap words (even)

// Layout of the sort's scratch: look-back words, histograms and tickets, then
// the tie-run bitmap (all zeroed by radix_prepare).
struct SortScratch {
    uint64_t* status;
    uint32_t* hist;
    uint32_t* tickets;
    uint32_t* bits;
    uint64_t* dtot;  // the first pass's digit totals when it prepares its own keys
    int32_t* err;
    uint64_t* part;  // per tile: the range of the keys a first pass will make
    uint32_t* meta;  // {least key, passes} of a first pass that made its keys
    int64_t words;  // u64 words to zero
};

SortScratch sort_scratch(void* ws, size_t ws_bytes, int64_t n, bool* ok) {
    const int64_t nb = sort_blocks(n);
    Arena ar(ws, ws_bytes);
    const int64_t status_words = (int64_t)kPasses * nb * kRadix;
    const int64_t hist_words = kHistCopies * kPasses * kRadix / 2 + kPasses;
    const int64_t bit_words = tie_words(n) / 2;
    uint64_t* block = ar.take<uint64_t>(status_words + hist_words + bit_words + kRadix);
    int32_t* err = ar.take<int32_t>(1);
    uint64_t* part = ar.take<uint64_t>(2 * nb);
    uint32_t* meta = ar.take<uint32_t>(2);
    *ok = !ar.overflow;
    SortScratch s{};
    if (!*ok) return s;
    s.status = block;
    s.hist = reinterpret_cast<uint32_t*>(block + status_words);
    s.tickets = s.hist + kHistCopies * kPasses * kRadix;
    s.bits = reinterpret_cast<uint32_t*>(block + status_words + hist_words);
    s.dtot = block + status_words + hist_words + bit_words;
    s.err = err;
    s.part = part;
    s.meta = meta;
    s.words = status_words + hist_words + bit_words + kRadix;
    return s;
}

// One tile per CU at most: the column exchange (all tiles resident, with a CU
// to spare for each).
bool use_exchange(int64_t n) {
    const int64_t nb = sort_blocks(n);
    return nb <= kXchgTiles && nb <= device_cus();
}

}  // namespace

size_t radix_workspace_bytes(int64_t n) {
    Sizer s;
    s.take<uint64_t>((size_t)kPasses * sort_blocks(n) * kRadix + kHistCopies * kPasses * kRadix / 2 + kPasses +
                     tie_words(n) / 2 + kRadix);
    s.take<int32_t>(1);
    s.take<uint64_t>(2 * sort_blocks(n));
    s.take<uint32_t>(2);
    return s.used + 256;
}

mh_status radix_prepare(void* ws, size_t ws_bytes, int64_t n, uint32_t** hist, hipStream_t stream,
                        ZeroRange e1, ZeroRange e2, const double* x, const double* y) {
    bool ok = false;
    SortScratch s = sort_scratch(ws, ws_bytes, n, &ok);
    if (!ok) return MH_EWORKSPACE;
    if (!e1.p) e1.n = 0;
    if (!e2.p) e2.n = 0;
    int64_t most = s.words > e1.n ? s.words : e1.n;
    most = most > e2.n ? most : e2.n;
    int64_t blocks = (most + kSortThreads - 1) / kSortThreads;
    if (blocks > 1024) blocks = 1024;
    KeySpan ks{};
    if (x && radix_prepares_keys(n)) {
        ks = KeySpan{x, y, n, s.part, sort_blocks(n)};
        if (blocks < sort_blocks(n)) blocks = sort_blocks(n);
    }
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)blocks), dim3(kSortThreads), 0, stream,
                       ZeroRange{s.status, s.words}, e1, e2, ks);
    MH_HIP_TRY(hipGetLastError());
    *hist = s.hist;
    return MH_OK;
}

bool radix_prepares_keys(int64_t n) { return n > 1 && n <= (int64_t)0xFFFFFFFFll && use_exchange(n); }

mh_status radix_sort_split64(uint32_t* hi, uint64_t* pay, uint32_t* hi_alt, uint64_t* pay_alt, int64_t n,
                             void* ws, size_t ws_bytes, int32_t* err, hipStream_t stream, const double* x,
                             const double* y, const uint32_t** kbase, const uint64_t** tile_mass) {
    if (kbase) *kbase = nullptr;
    if (tile_mass) *tile_mass = nullptr;
    if (n <= 1) return MH_OK;
    if (n > (int64_t)0xFFFFFFFFll) return MH_EINVAL;
    bool ok = false;
    SortScratch s = sort_scratch(ws, ws_bytes, n, &ok);
    if (!ok) return MH_EWORKSPACE;
    if (!err) err = s.err;
    const int64_t nb = sort_blocks(n);
    // the column exchange when every tile has a CU; otherwise the look-back, by
    // ticket unless the whole grid is resident
    const bool xchg = use_exchange(n);
    if (x && !xchg) return MH_EINVAL;  // keys from x need the exchange (radix_prepares_keys)
    // a first pass making its keys sets the pass count, which the later passes read
    uint32_t* meta = x ? s.meta : nullptr;
    if (kbase) *kbase = meta;
    if (tile_mass && x) *tile_mass = s.part + nb;
    const bool use_ticket = !xchg && nb > resident_blocks(k_onesweep<false, false>, kSortThreads);
    uint32_t* kin = hi;
    uint64_t* vin = pay;
    uint32_t* kout = hi_alt;
    uint64_t* vout = pay_alt;
    for (int pass = 0; pass < kPasses; ++pass) {
        auto kern = xchg ? (pass == 0 && x ? k_onesweep<true, true> : k_onesweep<true, false>)
                         : k_onesweep<false, false>;
        hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(kSortThreads), 0, stream, kin, vin, kout, vout, n, pass * 8,
                           s.hist + pass * kRadix, s.status + (int64_t)pass * nb * kRadix, s.tickets + pass,
                           use_ticket, err, x, y, s.hist, s.dtot, meta, (const uint64_t*)s.part);
        MH_HIP_TRY(hipGetLastError());
        uint32_t* tk = kin; kin = kout; kout = tk;
        uint64_t* tv = vin; vin = vout; vout = tv;
    }
    // 4 passes end in the input arrays; a first pass that sets an odd count
    // swaps the arrays of every pass, with the same result
    static_assert(kPasses % 2 == 0, "the passes end in the input arrays");
    // runs of equal high halves out of order by the low halves
    const int64_t cus = device_cus();
    const int32_t chunk = n <= (kFixChunk / 2) * cus ? kFixChunk / 2 : kFixChunk;
    const int64_t chunks = (n + chunk - 1) / chunk;
    const int64_t fix_grid = chunks < cus ? chunks : cus;
    hipLaunchKernelGGL(k_fix_runs, dim3((unsigned)fix_grid), dim3(kFixThreads), 0, stream, (const uint32_t*)hi, pay,
                       pay_alt, n, s.bits, chunk);
    MH_HIP_TRY(hipGetLastError());
    return MH_OK;
}

}  // namespace mh

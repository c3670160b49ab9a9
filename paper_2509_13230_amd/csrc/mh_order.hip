// Node order (ascending alpha, or alpha + beta, i.e. descending x or x*y:
// Sec. 2.4 step (i), first line of Alg. 1) and the bound of Sec. 2.5
// (product of the two largest y among the ranks not yet processed).
#include "mh_common.hpp"
#include "mh_internal.hpp"
#include "mh_keys.hpp"
#include "mh_lookback.hpp"
#include "mh_sweep_core.hpp"

namespace mh {

namespace {

constexpr int kThreads = 256;

constexpr int kPrepTile = 4096;
// 16 waves per tile of keys: the kernel is a chain of loads, histogram atomics
// and stores with little arithmetic, which only more waves per CU overlap.
constexpr int kPrepThreads = 1024;

// Sort keys (complemented bits of z = x or x*y, split: high half as the radix
// key, low half above the id as payload), checks of the parameters, and the
// digit histograms of all radix passes.
__global__ __launch_bounds__(kPrepThreads) void k_prep_keys(const double* __restrict__ x, const double* __restrict__ y,
                                                        int64_t n, uint32_t* __restrict__ keys,
                                                        uint64_t* __restrict__ vals, uint32_t* __restrict__ hist,
                                                        int32_t* status) {
    constexpr int kHist = kRadixPasses * 256;
    __shared__ uint32_t h[kHist];
    for (int i = threadIdx.x; i < kHist; i += kPrepThreads) h[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kPrepTile;
    constexpr int kPer = kPrepTile / kPrepThreads;
    // all loads first, then the keys and their counts
    double xv[kPer], yv[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int64_t i = base + (int64_t)q * kPrepThreads + threadIdx.x;
        xv[q] = 0.0;
        yv[q] = 0.0;
        if (i < n) {
            xv[q] = x[i];
            if (y) yv[q] = y[i];
        }
    }
    bool bad = false;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int64_t i = base + (int64_t)q * kPrepThreads + threadIdx.x;
        const bool valid = i < n;
        uint32_t key = 0;
        if (valid) {
            bool ok;
            const double z = node_z(xv[q], y != nullptr, yv[q], &ok);
            bad = bad || !ok;
            uint64_t pay;
            split_key(z, i, &key, &pay);
            keys[i] = key;
            vals[i] = pay;
        }
        count_key_digits(h, key, valid, 0, kRadixPasses);
    }
    if (bad) raise_status(status, MH_EINVAL);
    __syncthreads();
    // one of the histogram copies per block (the sort sums them)
    uint32_t* copy = hist + (blockIdx.x % kRadixHistCopies) * kHist;
    for (int i = threadIdx.x; i < kHist; i += kPrepThreads)
        if (h[i]) atomicAdd(&copy[i], h[i]);
}

// The sorted key and id at a rank, from the split sort's arrays (whose high
// halves are the keys' less kb).
__device__ __forceinline__ double sorted_z(const uint32_t* __restrict__ keys, const uint64_t* __restrict__ vals,
                                           int64_t r, uint32_t kb, uint32_t* id) {
    const uint64_t v = vals[r];
    *id = (uint32_t)v;
    return key_value(((uint64_t)(keys[r] + kb) << 32) | (v >> 32));
}

__global__ __launch_bounds__(kThreads) void k_finish_order(const uint32_t* __restrict__ keys,
                                                           const uint64_t* __restrict__ vals, int64_t n,
                                                           int32_t* __restrict__ perm, double* __restrict__ zs,
                                                           NodeRec* __restrict__ node,
                                                           const double* __restrict__ y, double* __restrict__ ys,
                                                           uint64_t* __restrict__ mass, int32_t check_square,
                                                           const uint32_t* kbase, int32_t* status) {
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r >= n) return;
    uint32_t id;
    const double z = sorted_z(keys, vals, r, kbase ? *kbase : 0u, &id);
    if (node) {
        node[r].z = z;
        node[r].id = (int32_t)id;
    } else {
        perm[r] = (int32_t)id;
        zs[r] = z;
    }
    if (ys) ys[r] = y[id];
    if (mass) mass[r] = mass_q(z);
    if (check_square && r == 0 && !isfinite(z * z)) raise_status(status, MH_EINVAL);
}

// The same, into node records, with the column masses scanned on the way:
// P[r] = sum of floor(z 2^32) over ranks < r, P[n] = total (tiles of 4096
// ranks, look-back state zero at launch); every 256th P and z to the sample
// arrays.
__global__ __launch_bounds__(kLbThreads) void k_finish_order_scan(const uint32_t* __restrict__ keys,
                                                                  const uint64_t* __restrict__ vals, int64_t n,
                                                                  NodeRec* __restrict__ node,
                                                                  const double* __restrict__ y,
                                                                  double* __restrict__ ys, uint64_t* __restrict__ P,
                                                                  int64_t tiles, uint64_t* state,
                                                                  uint64_t* samples, double* zsamples,
                                                                  int32_t check_square, const uint32_t* kbase,
                                                                  int32_t* status) {
    __shared__ LbShared sh;
    const uint32_t kb = kbase ? *kbase : 0u;
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t base = tile * kLbTile;
#pragma unroll 4
        for (int k = 0; k < kLbItems; ++k) {
            const int idx = k * kLbThreads + threadIdx.x;
            const int64_t r = base + idx;
            uint64_t m = 0;
            if (r < n) {
                uint32_t id;
                const double z = sorted_z(keys, vals, r, kb, &id);
                node[r].z = z;
                node[r].id = (int32_t)id;
                if (ys) ys[r] = y[id];
                if (zsamples && (r & ((1 << kSampleShift) - 1)) == 0) zsamples[r >> kSampleShift] = z;
                m = mass_q(z);
                if (check_square && r == 0 && !isfinite(z * z)) raise_status(status, MH_EINVAL);
            }
            sh.items[lb_at(idx)] = m;
        }
        const uint64_t end = lb_tile_scan(sh, tile, state, status);
#pragma unroll
        for (int k = 0; k < kLbItems; ++k) {
            const int idx = k * kLbThreads + threadIdx.x;
            const int64_t r = base + idx;
            if (r < n) {
                const uint64_t v = sh.items[lb_at(idx)];
                P[r] = v;
                if (samples && (r & ((1 << kSampleShift) - 1)) == 0) samples[r >> kSampleShift] = v;
            }
        }
        if (threadIdx.x == 0 && base + kLbTile >= n) {
            P[n] = end;
            if (samples && (n & ((1 << kSampleShift) - 1)) == 0) samples[n >> kSampleShift] = end;
        }
    }
}

// ---- suffix top-2 of ys: the monoid keeps the two largest values (multiset) ----
struct Top2 {
    double a, b;  // a >= b; -1 marks "none" (inputs are >= 0)
};

__device__ __forceinline__ Top2 top2_combine(Top2 p, Top2 q) {
    Top2 r;
    if (p.a >= q.a) {
        r.a = p.a;
        r.b = fmax(p.b, q.a);
    } else {
        r.a = q.a;
        r.b = fmax(q.b, p.a);
    }
    return r;
}

__device__ __forceinline__ Top2 top2_shfl_down(Top2 v, int off) {
    Top2 r;
    r.a = __shfl_down(v.a, off, kWave);
    r.b = __shfl_down(v.b, off, kWave);
    return r;
}

constexpr int kBoundItems = 8;
constexpr int kBoundTile = kThreads * kBoundItems;

// Suffix (towards higher ranks) inclusive scan of per-thread values over the block.
__device__ __forceinline__ Top2 block_suffix_exclusive(Top2 v, Top2* lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    Top2 inc = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        Top2 u = top2_shfl_down(inc, off);
        if (lane + off < kWave) inc = top2_combine(inc, u);
    }
    if (lane == 0) lds[wave] = inc;  // wave's total
    __syncthreads();
    Top2 after = {-1.0, -1.0};
    for (int w = kThreads / kWave - 1; w > wave; --w) after = top2_combine(after, lds[w]);
    // exclusive within the wave: the value of the next lane's inclusive
    Top2 nxt = top2_shfl_down(inc, 1);
    Top2 excl = (lane + 1 < kWave) ? top2_combine(nxt, after) : after;
    __syncthreads();
    return excl;
}

__global__ __launch_bounds__(kThreads) void k_bound_tile_aggr(const double* __restrict__ ys, int64_t n,
                                                              Top2* __restrict__ aggr) {
    __shared__ Top2 lds[kThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kBoundTile;
    Top2 v = {-1.0, -1.0};
    for (int k = 0; k < kBoundItems; ++k) {
        const int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
        if (i < n) v = top2_combine(v, Top2{ys[i], -1.0});
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        Top2 u;
        u.a = __shfl_xor(v.a, off, kWave);
        u.b = __shfl_xor(v.b, off, kWave);
        v = top2_combine(v, u);
    }
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        Top2 t = lds[0];
        for (int w = 1; w < kThreads / kWave; ++w) t = top2_combine(t, lds[w]);
        aggr[blockIdx.x] = t;
    }
}

// One block: exclusive suffix combine of the tile aggregates, in place.
__global__ __launch_bounds__(kThreads) void k_bound_aggr_scan(Top2* aggr, int64_t nb) {
    __shared__ Top2 lds[kThreads / kWave];
    Top2 carry = {-1.0, -1.0};
    const int64_t nchunks = (nb + kThreads - 1) / kThreads;
    for (int64_t ch = nchunks - 1; ch >= 0; --ch) {
        const int64_t i = ch * kThreads + threadIdx.x;
        Top2 v = (i < nb) ? aggr[i] : Top2{-1.0, -1.0};
        Top2 excl = block_suffix_exclusive(v, lds);
        Top2 out = top2_combine(excl, carry);
        // chunk total = combine of everything in the chunk (thread 0's inclusive)
        Top2 tot0 = top2_combine(v, excl);
        __shared__ Top2 chunk_total;
        if (threadIdx.x == 0) chunk_total = tot0;
        __syncthreads();
        if (i < nb) aggr[i] = out;
        carry = top2_combine(carry, chunk_total);
        __syncthreads();
    }
}

__global__ __launch_bounds__(kThreads) void k_bound_tile_scan(const double* __restrict__ ys, int64_t n,
                                                              const Top2* __restrict__ aggr_excl,
                                                              double* __restrict__ c, int32_t* status) {
    __shared__ Top2 lds[kThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kBoundTile + (int64_t)threadIdx.x * kBoundItems;
    double vals[kBoundItems];
    Top2 v = {-1.0, -1.0};
#pragma unroll
    for (int k = 0; k < kBoundItems; ++k) {
        const int64_t i = base + k;
        vals[k] = (i < n) ? ys[i] : -1.0;
        v = top2_combine(v, Top2{vals[k], -1.0});
    }
    Top2 after = block_suffix_exclusive(v, lds);
    after = top2_combine(after, aggr_excl[blockIdx.x]);
    bool bad = false;
#pragma unroll
    for (int k = kBoundItems - 1; k >= 0; --k) {
        const int64_t r = base + k;
        after = top2_combine(Top2{vals[k], -1.0}, after);
        if (r < n) {
            const double Y = (after.b < 0.0) ? 0.0 : after.a * after.b;
            c[r] = 1.0 - Y;
            if (r < n - 1 && !(Y < 1.0)) bad = true;
        }
    }
    if (bad) raise_status(status, MH_EINVAL);
}

}  // namespace

size_t order_workspace_bytes(int64_t n) {
    Sizer s;
    s.take<uint32_t>(n);  // keys
    s.take<uint32_t>(n);  // keys alt
    s.take<uint64_t>(n);  // vals
    s.take<uint64_t>(n);  // vals alt
    return s.used + radix_workspace_bytes(n) + 256;
}

mh_status order_nodes(const double* x, const double* y, int64_t n, int32_t* perm, double* zs, double* ys,
                      NodeRec* node, int32_t* status, uint64_t* mass_prefix, uint64_t* mass_state,
                      uint64_t* mass_samples, double* z_samples, void* ws, size_t ws_bytes, hipStream_t stream,
                      bool check_square,
                      ZeroRange e1, ZeroRange e2, SortedKeys* sorted) {
    if (sorted) *sorted = SortedKeys{};
    if (n <= 0) return MH_OK;
    Arena ar(ws, ws_bytes);
    uint32_t* keys = ar.take<uint32_t>(n);
    uint32_t* keys_alt = ar.take<uint32_t>(n);
    uint64_t* vals = ar.take<uint64_t>(n);
    uint64_t* vals_alt = ar.take<uint64_t>(n);
    if (ar.overflow) return MH_EWORKSPACE;
    const size_t off = (ar.used + 255) & ~size_t(255);
    void* sort_ws = ar.base + off;
    const size_t sort_bytes = ws_bytes > off ? ws_bytes - off : 0;
    uint32_t* hist = nullptr;
    // keys and histograms: made by the first radix pass itself when the sort
    // exchanges digit counts between resident tiles, else by k_prep_keys
    const bool fused = radix_prepares_keys(n);
    mh_status st = radix_prepare(sort_ws, sort_bytes, n, &hist, stream, e1, e2, fused ? x : nullptr, y);
    if (st != MH_OK) return st;
    if (!fused) {
        const unsigned tiles = (unsigned)((n + kPrepTile - 1) / kPrepTile);
        hipLaunchKernelGGL(k_prep_keys, dim3(tiles), dim3(kPrepThreads), 0, stream, x, y, n, keys, vals, hist,
                           status);
        MH_HIP_TRY(hipGetLastError());
    }
    const uint32_t* kbase = nullptr;  // the keys' least high half, when the sort subtracted it
    const uint64_t* tile_mass = nullptr;
    st = radix_sort_split64(keys, vals, keys_alt, vals_alt, n, sort_ws, sort_bytes, status, stream,
                            fused ? x : nullptr, y, &kbase, &tile_mass);
    if (st != MH_OK) return st;
    if (sorted && kbase && tile_mass) {
        *sorted = SortedKeys{keys, vals, kbase, tile_mass, (n + kPrepTile - 1) / kPrepTile};
        return MH_OK;
    }
    if (mass_prefix && node && n <= (int64_t)1 << 30) {
        // records and the masses' prefix sums in one pass (sums stay below 2^62)
        const int64_t tiles = lb_tiles(n);
        const int64_t resident = resident_blocks(k_finish_order_scan, kLbThreads);
        const int64_t grid = tiles < resident ? tiles : resident;
        hipLaunchKernelGGL(k_finish_order_scan, dim3((unsigned)grid), dim3(kLbThreads), 0, stream,
                           (const uint32_t*)keys, (const uint64_t*)vals, n, node, y, y ? ys : nullptr, mass_prefix,
                           tiles, mass_state, mass_samples, z_samples, (int32_t)check_square, kbase, status);
        MH_HIP_TRY(hipGetLastError());
        return MH_OK;
    }
    const unsigned grid = (unsigned)((n + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_finish_order, dim3(grid), dim3(kThreads), 0, stream, keys, vals, n, perm, zs, node, y,
                       y ? ys : nullptr, mass_prefix, (int32_t)check_square, kbase, status);
    MH_HIP_TRY(hipGetLastError());
    if (mass_prefix) return scan_exclusive_u64(mass_prefix, mass_prefix, n, ws, ws_bytes, stream);
    return MH_OK;
}

size_t bound_workspace_bytes(int64_t n) {
    const int64_t nb = (n + kBoundTile - 1) / kBoundTile;
    Sizer s;
    s.take<Top2>(nb + 1);
    return s.used + 256;
}

mh_status bound_suffix_top2(const double* ys, int64_t n, double* c, int32_t* status, void* ws, size_t ws_bytes,
                            hipStream_t stream) {
    if (n <= 0) return MH_OK;
    const int64_t nb = (n + kBoundTile - 1) / kBoundTile;
    Arena ar(ws, ws_bytes);
    Top2* aggr = ar.take<Top2>(nb + 1);
    if (!aggr) return MH_EWORKSPACE;
    hipLaunchKernelGGL(k_bound_tile_aggr, dim3((unsigned)nb), dim3(kThreads), 0, stream, ys, n, aggr);
    MH_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_bound_aggr_scan, dim3(1), dim3(kThreads), 0, stream, aggr, nb);
    MH_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_bound_tile_scan, dim3((unsigned)nb), dim3(kThreads), 0, stream, ys, n, aggr, c, status);
    MH_HIP_TRY(hipGetLastError());
    return MH_OK;
}

}  // namespace mh

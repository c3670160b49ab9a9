// Triangle count of a sampled network (the motif statistic of Sec. 2.1 and
// Fig. 1B, on which the Chung-Lu model and the unbiased configuration model
// lead to opposite conclusions).
//
// Every edge is oriented from its smaller to its larger id, so that each
// triangle a < b < c is found exactly once: at the edge (a, b), as the common
// out-neighbour c of a and b.  The oriented edges are sorted by (a, b) with the
// node order's split radix sort, which makes every out-neighbour list a sorted
// slice of the edge array; row offsets come from a binary search per node.
// The intersections are balanced by work item, not by edge: edge e costs
// w_e = min(outdeg a, outdeg b) membership tests, each test (one element of
// the shorter list searched in the longer) is one thread's work, and a prefix
// sum over w_e maps threads to edges.  One 64-bit atomic per block adds the
// block's count.
#include "mh_common.hpp"
#include "mh_internal.hpp"
#include "mh_keys.hpp"

namespace mh {

namespace {

constexpr int kTriThreads = 256;
constexpr int kTriKeyThreads = 1024;
constexpr int kTriTile = 4096;

// Oriented keys (hi = smaller id, pay = larger id above zero) and their digit
// histograms; an invalid edge (an id outside [0, n) or a loop) raises
// MH_EINVAL.
__global__ __launch_bounds__(kTriKeyThreads) void k_tri_keys(const int32_t* __restrict__ src,
                                                             const int32_t* __restrict__ dst, int64_t m, int64_t n,
                                                             uint32_t* __restrict__ hi, uint64_t* __restrict__ pay,
                                                             uint32_t* __restrict__ hist, int32_t* err) {
    constexpr int kHist = kRadixPasses * 256;
    __shared__ uint32_t h[kHist];
    for (int i = threadIdx.x; i < kHist; i += kTriKeyThreads) h[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTriTile;
    bool bad = false;
#pragma unroll
    for (int q = 0; q < kTriTile / kTriKeyThreads; ++q) {
        const int64_t e = base + (int64_t)q * kTriKeyThreads + threadIdx.x;
        const bool valid = e < m;
        uint32_t key = 0;
        if (valid) {
            int32_t a = src[e], b = dst[e];
            if (a < 0 || b < 0 || a >= n || b >= n || a == b) {
                bad = true;  // reported; the edge becomes (0, 0) so that every later index stays in range
                a = 0;
                b = 0;
            }
            const uint32_t lo = (uint32_t)(a < b ? a : b), up = (uint32_t)(a < b ? b : a);
            key = lo;
            hi[e] = lo;
            pay[e] = (uint64_t)up << 32;
        }
        count_key_digits(h, key, valid, 0, kRadixPasses);
    }
    if (bad) raise_status(err, MH_EINVAL);
    __syncthreads();
    uint32_t* copy = hist + (blockIdx.x % kRadixHistCopies) * kHist;
    for (int i = threadIdx.x; i < kHist; i += kTriKeyThreads)
        if (h[i]) atomicAdd(&copy[i], h[i]);
}

// off[v] = first edge whose smaller end is v (v = 0..n; off[n] = m).
__global__ __launch_bounds__(kTriThreads) void k_tri_offsets(const uint32_t* __restrict__ hi, int64_t m, int64_t n,
                                                             int64_t* __restrict__ off) {
    const int64_t v = (int64_t)blockIdx.x * kTriThreads + threadIdx.x;
    if (v > n) return;
    int64_t lo = 0, up = m;
    while (lo < up) {
        const int64_t mid = lo + (up - lo) / 2;
        if ((int64_t)hi[mid] < v) lo = mid + 1; else up = mid;
    }
    off[v] = lo;
}

// w[e] = min(outdeg(a), outdeg(b)) for the sorted edge e = (a, b).
__global__ __launch_bounds__(kTriThreads) void k_tri_work(const uint32_t* __restrict__ hi,
                                                          const uint64_t* __restrict__ pay, int64_t m,
                                                          const int64_t* __restrict__ off, uint64_t* __restrict__ w) {
    const int64_t e = (int64_t)blockIdx.x * kTriThreads + threadIdx.x;
    if (e >= m) return;
    const uint32_t a = hi[e], b = (uint32_t)(pay[e] >> 32);
    const int64_t da = off[a + 1] - off[a], db = off[b + 1] - off[b];
    w[e] = (uint64_t)(da < db ? da : db);
}

// Membership tests t = 0..W-1 (W = wo[m]): test t belongs to the edge e with
// wo[e] <= t < wo[e + 1] and checks element t - wo[e] of the shorter
// out-neighbour list of e's ends against the longer one.
__global__ __launch_bounds__(kTriThreads) void k_tri_count(const uint32_t* __restrict__ hi,
                                                           const uint64_t* __restrict__ pay, int64_t m,
                                                           const int64_t* __restrict__ off,
                                                           const uint64_t* __restrict__ wo,
                                                           unsigned long long* __restrict__ total) {
    __shared__ unsigned long long s_sum[kTriThreads / kWave];
    const uint64_t W = wo[m];
    unsigned long long found = 0;
    for (uint64_t t = (uint64_t)blockIdx.x * kTriThreads + threadIdx.x; t < W;
         t += (uint64_t)gridDim.x * kTriThreads) {
        int64_t lo = 0, up = m;  // last e with wo[e] <= t
        while (up - lo > 1) {
            const int64_t mid = lo + (up - lo) / 2;
            if (wo[mid] <= t) lo = mid; else up = mid;
        }
        const int64_t e = lo;
        const uint32_t a = hi[e], b = (uint32_t)(pay[e] >> 32);
        const int64_t a0 = off[a], a1 = off[a + 1], b0 = off[b], b1 = off[b + 1];
        const bool a_short = (a1 - a0) <= (b1 - b0);
        const int64_t s0 = a_short ? a0 : b0;
        int64_t l0 = a_short ? b0 : a0, l1 = a_short ? b1 : a1;
        const uint32_t c = (uint32_t)(pay[s0 + (int64_t)(t - wo[e])] >> 32);
        while (l0 < l1) {  // c in the longer list?
            const int64_t mid = l0 + (l1 - l0) / 2;
            const uint32_t v = (uint32_t)(pay[mid] >> 32);
            if (v < c) l0 = mid + 1; else l1 = mid;
        }
        const int64_t L1 = a_short ? b1 : a1;
        found += (l0 < L1 && (uint32_t)(pay[l0] >> 32) == c) ? 1ull : 0ull;
    }
    found = wave_sum(found);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = found;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = 0;
        for (int i = 0; i < kTriThreads / kWave; ++i) b += s_sum[i];
        if (b) atomicAdd(total, b);
    }
}

struct TriScratch {
    uint32_t* hi;
    uint32_t* hi_alt;
    uint64_t* pay;
    uint64_t* pay_alt;
    int64_t* off;
    uint64_t* wo;     // m + 1
    uint64_t* words;  // [0]: total; [1]: status (int32)
};

template <typename A>
TriScratch carve_tri(A& ar, int64_t n, int64_t m) {
    TriScratch s{};
    s.hi = ar.template take<uint32_t>(m);
    s.hi_alt = ar.template take<uint32_t>(m);
    s.pay = ar.template take<uint64_t>(m);
    s.pay_alt = ar.template take<uint64_t>(m);
    s.off = ar.template take<int64_t>(n + 1);
    s.wo = ar.template take<uint64_t>(m + 1);
    s.words = ar.template take<uint64_t>(2);
    return s;
}

size_t tri_scratch_bytes(int64_t m) {
    const size_t a = radix_workspace_bytes(m);
    const size_t b = scan_workspace_bytes(m);
    return (a > b ? a : b) + 256;
}

}  // namespace

}  // namespace mh

extern "C" {

size_t mh_triangles_workspace_bytes(int64_t n, int64_t n_edges) {
    if (n < 0 || n_edges < 0) return 0;
    mh::Sizer sz;
    mh::carve_tri(sz, n, n_edges);
    return ((sz.used + 255) & ~size_t(255)) + mh::tri_scratch_bytes(n_edges) + 256;
}

mh_status mh_count_triangles(const int32_t* src, const int32_t* dst, int64_t n_edges, int64_t n,
                             uint64_t* triangles_host, void* workspace, size_t ws_bytes, hipStream_t stream) {
    using namespace mh;
    if (!triangles_host) return MH_EINVAL;
    *triangles_host = 0;
    if (n < 0 || n > 0x7FFFFFFFll || n_edges < 0 || n_edges > 0x7FFFFFFFll) return MH_EINVAL;
    if (n_edges == 0) return MH_OK;
    if (!src || !dst || n == 0) return MH_EINVAL;
    if (!workspace || ws_bytes < mh_triangles_workspace_bytes(n, n_edges)) return MH_EWORKSPACE;
    Arena ar(workspace, ws_bytes);
    TriScratch s = carve_tri(ar, n, n_edges);
    if (ar.overflow) return MH_EWORKSPACE;
    const size_t off = (ar.used + 255) & ~size_t(255);
    void* scratch = ar.base + off;
    const size_t scratch_bytes = ws_bytes - off;
    int32_t* err = reinterpret_cast<int32_t*>(s.words + 1);
    uint32_t* hist = nullptr;
    mh_status st = radix_prepare(scratch, scratch_bytes, n_edges, &hist, stream, ZeroRange{s.words, 2});
    if (st != MH_OK) return st;
    const unsigned tiles = (unsigned)((n_edges + kTriTile - 1) / kTriTile);
    hipLaunchKernelGGL(k_tri_keys, dim3(tiles), dim3(kTriKeyThreads), 0, stream, src, dst, n_edges, n, s.hi, s.pay,
                       hist, err);
    MH_HIP_TRY(hipGetLastError());
    st = radix_sort_split64(s.hi, s.pay, s.hi_alt, s.pay_alt, n_edges, scratch, scratch_bytes, err, stream);
    if (st != MH_OK) return st;
    hipLaunchKernelGGL(k_tri_offsets, dim3((unsigned)((n + kTriThreads) / kTriThreads)), dim3(kTriThreads), 0, stream,
                       (const uint32_t*)s.hi, n_edges, n, s.off);
    MH_HIP_TRY(hipGetLastError());
    const unsigned eg = (unsigned)((n_edges + kTriThreads - 1) / kTriThreads);
    hipLaunchKernelGGL(k_tri_work, dim3(eg), dim3(kTriThreads), 0, stream, (const uint32_t*)s.hi,
                       (const uint64_t*)s.pay, n_edges, (const int64_t*)s.off, s.wo);
    MH_HIP_TRY(hipGetLastError());
    st = scan_exclusive_u64(s.wo, s.wo, n_edges, scratch, scratch_bytes, stream);
    if (st != MH_OK) return st;
    const int64_t grid = resident_blocks(k_tri_count, kTriThreads);
    hipLaunchKernelGGL(k_tri_count, dim3((unsigned)grid), dim3(kTriThreads), 0, stream, (const uint32_t*)s.hi,
                       (const uint64_t*)s.pay, n_edges, (const int64_t*)s.off, (const uint64_t*)s.wo,
                       reinterpret_cast<unsigned long long*>(s.words));
    MH_HIP_TRY(hipGetLastError());
    uint64_t hw[2] = {0, 0};
    MH_HIP_TRY(hipMemcpyAsync(hw, s.words, sizeof(hw), hipMemcpyDeviceToHost, stream));
    MH_HIP_TRY(hipStreamSynchronize(stream));
    const int32_t status = (int32_t)(uint32_t)hw[1];
    if (status != 0) return (mh_status)status;
    *triangles_host = hw[0];
    return MH_OK;
}

}  // extern "C"

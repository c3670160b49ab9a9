// Canonical order of an edge list: (src, dst[, w]) sorted by (src, dst).  The
// method's output is a set of edges (Alg. 1 returns E as a set); a sample's
// edges leave the sweep in an order that depends on the schedule, and a
// canonical order makes two samples comparable element by element.  Every pair
// appears once, so (src, dst) orders the list totally.  The keys go through
// the node order's split radix sort: src as the radix key, dst above the
// weight as payload, runs of equal src repaired by dst.
#include "mh_common.hpp"
#include "mh_internal.hpp"
#include "mh_keys.hpp"

namespace mh {

namespace {

constexpr int kEdgeThreads = 1024;
constexpr int kEdgeTile = 4096;

__global__ __launch_bounds__(kEdgeThreads) void k_edge_keys(const int32_t* __restrict__ src,
                                                            const int32_t* __restrict__ dst,
                                                            const int32_t* __restrict__ w, int64_t m,
                                                            uint32_t* __restrict__ hi, uint64_t* __restrict__ pay,
                                                            uint32_t* __restrict__ hist) {
    constexpr int kHist = kRadixPasses * 256;
    __shared__ uint32_t h[kHist];
    for (int i = threadIdx.x; i < kHist; i += kEdgeThreads) h[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kEdgeTile;
#pragma unroll
    for (int q = 0; q < kEdgeTile / kEdgeThreads; ++q) {
        const int64_t e = base + (int64_t)q * kEdgeThreads + threadIdx.x;
        const bool valid = e < m;
        uint32_t key = 0;
        if (valid) {
            key = (uint32_t)src[e];
            hi[e] = key;
            pay[e] = ((uint64_t)(uint32_t)dst[e] << 32) | (uint64_t)(uint32_t)(w ? w[e] : 0);
        }
        count_key_digits(h, key, valid, 0, kRadixPasses);
    }
    __syncthreads();
    uint32_t* copy = hist + (blockIdx.x % kRadixHistCopies) * kHist;
    for (int i = threadIdx.x; i < kHist; i += kEdgeThreads)
        if (h[i]) atomicAdd(&copy[i], h[i]);
}

__global__ __launch_bounds__(kEdgeThreads) void k_edge_unpack(const uint32_t* __restrict__ hi,
                                                              const uint64_t* __restrict__ pay, int64_t m,
                                                              int32_t* __restrict__ src, int32_t* __restrict__ dst,
                                                              int32_t* __restrict__ w) {
    const int64_t e = (int64_t)blockIdx.x * kEdgeThreads + threadIdx.x;
    if (e >= m) return;
    const uint64_t p = pay[e];
    src[e] = (int32_t)hi[e];
    dst[e] = (int32_t)(p >> 32);
    if (w) w[e] = (int32_t)(uint32_t)p;
}

struct EdgeScratch {
    uint32_t* hi;
    uint32_t* hi_alt;
    uint64_t* pay;
    uint64_t* pay_alt;
    uint64_t* err;  // one word: the sort's device status
    void* sort_ws;
    size_t sort_bytes;
};

template <typename A>
EdgeScratch carve_edges(A& ar, int64_t m) {
    EdgeScratch s{};
    s.hi = ar.template take<uint32_t>(m);
    s.hi_alt = ar.template take<uint32_t>(m);
    s.pay = ar.template take<uint64_t>(m);
    s.pay_alt = ar.template take<uint64_t>(m);
    s.err = ar.template take<uint64_t>(1);
    return s;
}

}  // namespace

}  // namespace mh

extern "C" {

size_t mh_sort_edges_workspace_bytes(int64_t n_edges) {
    if (n_edges < 0) return 0;
    mh::Sizer sz;
    mh::carve_edges(sz, n_edges);
    return ((sz.used + 255) & ~size_t(255)) + mh::radix_workspace_bytes(n_edges) + 256;
}

mh_status mh_sort_edges(int32_t* src, int32_t* dst, int32_t* w, int64_t n_edges, void* workspace, size_t ws_bytes,
                        hipStream_t stream) {
    using namespace mh;
    if (n_edges < 0 || n_edges > (int64_t)0x7FFFFFFFll) return MH_EINVAL;
    if (n_edges <= 1) return MH_OK;
    if (!src || !dst) return MH_EINVAL;
    if (!workspace || ws_bytes < mh_sort_edges_workspace_bytes(n_edges)) return MH_EWORKSPACE;
    Arena ar(workspace, ws_bytes);
    EdgeScratch s = carve_edges(ar, n_edges);
    if (ar.overflow) return MH_EWORKSPACE;
    const size_t off = (ar.used + 255) & ~size_t(255);
    void* sort_ws = ar.base + off;
    const size_t sort_bytes = ws_bytes - off;
    uint32_t* hist = nullptr;
    mh_status st = radix_prepare(sort_ws, sort_bytes, n_edges, &hist, stream, ZeroRange{s.err, 1});
    if (st != MH_OK) return st;
    const unsigned tiles = (unsigned)((n_edges + kEdgeTile - 1) / kEdgeTile);
    hipLaunchKernelGGL(k_edge_keys, dim3(tiles), dim3(kEdgeThreads), 0, stream, (const int32_t*)src,
                       (const int32_t*)dst, (const int32_t*)w, n_edges, s.hi, s.pay, hist);
    MH_HIP_TRY(hipGetLastError());
    int32_t* err = reinterpret_cast<int32_t*>(s.err);
    st = radix_sort_split64(s.hi, s.pay, s.hi_alt, s.pay_alt, n_edges, sort_ws, sort_bytes, err, stream);
    if (st != MH_OK) return st;
    const unsigned grid = (unsigned)((n_edges + kEdgeThreads - 1) / kEdgeThreads);
    hipLaunchKernelGGL(k_edge_unpack, dim3(grid), dim3(kEdgeThreads), 0, stream, (const uint32_t*)s.hi,
                       (const uint64_t*)s.pay, n_edges, src, dst, w);
    MH_HIP_TRY(hipGetLastError());
    int32_t herr = 0;
    MH_HIP_TRY(hipMemcpyAsync(&herr, err, sizeof(herr), hipMemcpyDeviceToHost, stream));
    MH_HIP_TRY(hipStreamSynchronize(stream));
    return herr != 0 ? (mh_status)herr : MH_OK;
}

}  // extern "C"

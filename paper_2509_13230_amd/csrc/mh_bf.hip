// Brute-force sampler (Sec. 2.2): every pair i < j, i in [row_begin, row_end),
// is an edge with probability p_ij, decided by its own Philox block with
// counter (j, i, replica, 0xFFFFFFFF).  One wave per (row, 1024-column chunk);
// accepted pairs are compacted per wave and written in coalesced runs.
#include "mh_common.hpp"
#include "mh_internal.hpp"
#include "mh_stage.hpp"

namespace mh {

namespace {

constexpr int kThreads = 256;
constexpr int kWavesPerBlock = kThreads / kWave;
constexpr int kChunkCols = 1024;
constexpr int kValThreads = 256;

struct BfCounters {
    unsigned long long n_edges;
    int32_t status;
    int32_t pad;
};

struct ValAggr {
    double zmax, y1, y2;
};

__global__ void k_bf_init(BfCounters* c) {
    if (threadIdx.x == 0) {
        c->n_edges = 0;
        c->status = 0;
        c->pad = 0;
    }
}

__device__ __forceinline__ void top2_push(double v, double& y1, double& y2) {
    if (v > y1) {
        y2 = y1;
        y1 = v;
    } else if (v > y2) {
        y2 = v;
    }
}

// Per-element checks plus per-block max z and two largest y.
__global__ __launch_bounds__(kValThreads) void k_validate(const double* __restrict__ x, const double* __restrict__ y,
                                                          int64_t n, ValAggr* __restrict__ aggr, int32_t* status) {
    __shared__ ValAggr lds[kValThreads];
    double zmax = 0.0, y1 = -1.0, y2 = -1.0;
    bool ok = true;
    for (int64_t i = (int64_t)blockIdx.x * kValThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kValThreads) {
        const double xi = x[i];
        bool good = (xi >= 0.0) && isfinite(xi);
        double z = xi;
        if (y) {
            const double yi = y[i];
            good = good && (yi >= 0.0) && isfinite(yi);
            z = xi * yi;
            good = good && isfinite(z);
            if (good) top2_push(yi, y1, y2);
        }
        ok = ok && good;
        if (good && z > zmax) zmax = z;
    }
    if (!ok) raise_status(status, MH_EINVAL);
    lds[threadIdx.x] = ValAggr{zmax, y1, y2};
    __syncthreads();
    if (threadIdx.x == 0) {
        ValAggr a = lds[0];
        for (int t = 1; t < kValThreads; ++t) {
            if (lds[t].zmax > a.zmax) a.zmax = lds[t].zmax;
            top2_push(lds[t].y1, a.y1, a.y2);
            top2_push(lds[t].y2, a.y1, a.y2);
        }
        aggr[blockIdx.x] = a;
    }
}

__global__ void k_validate_final(const ValAggr* __restrict__ aggr, int nb, bool weighted, int32_t* status) {
    if (threadIdx.x != 0) return;
    ValAggr a = aggr[0];
    for (int b = 1; b < nb; ++b) {
        if (aggr[b].zmax > a.zmax) a.zmax = aggr[b].zmax;
        top2_push(aggr[b].y1, a.y1, a.y2);
        top2_push(aggr[b].y2, a.y1, a.y2);
    }
    if (!isfinite(a.zmax * a.zmax)) raise_status(status, MH_EINVAL);
    if (weighted && a.y2 >= 0.0 && !(a.y1 * a.y2 < 1.0)) raise_status(status, MH_EINVAL);
}

template <bool WEIGHTED>
__global__ __launch_bounds__(kThreads) void k_bruteforce(const double* __restrict__ x, const double* __restrict__ y,
                                                         int64_t n, int64_t row_begin, int64_t row_end, uint32_t key0,
                                                         uint32_t key1, uint32_t replica, EdgeOut out,
                                                         const int32_t* status) {
    __shared__ int32_t s_src[kWavesPerBlock][kStageEdges];
    __shared__ int32_t s_dst[kWavesPerBlock][kStageEdges];
    __shared__ int32_t s_w[WEIGHTED ? kWavesPerBlock : 1][WEIGHTED ? kStageEdges : 1];
    if (*status != 0) return;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t i = row_begin + (int64_t)blockIdx.x * kWavesPerBlock + wave;
    if (i >= row_end) return;
    const int64_t c0 = (int64_t)blockIdx.y * kChunkCols;
    const int64_t jb = (c0 > i + 1) ? c0 : i + 1;
    const int64_t je = (c0 + kChunkCols < n) ? c0 + kChunkCols : n;
    if (jb >= je) return;

    WaveStage<WEIGHTED> stage{s_src[wave], s_dst[wave], WEIGHTED ? s_w[wave] : nullptr, 0u};
    const double yi = WEIGHTED ? y[i] : 0.0;
    const double zi = WEIGHTED ? x[i] * yi : x[i];
    for (int64_t j0 = jb; j0 < je; j0 += kWave) {
        const int64_t j = j0 + lane;
        bool acc = false;
        int32_t wt = 0;
        if (j < je) {
            const double yj = WEIGHTED ? y[j] : 0.0;
            const double zj = WEIGHTED ? x[j] * yj : x[j];
            const double t = zi * zj;
            const u32x4 R = philox4x32_10((uint32_t)j, (uint32_t)i, replica, 0xFFFFFFFFu, key0, key1);
            const double U = uniform53(R.v0, R.v1);
            const double e = WEIGHTED ? 1.0 - yi * yj : 1.0;
            acc = (U * (e + t)) < t;
            if (WEIGHTED && acc) {
                const double bb = yi * yj;
                if (bb == 0.0) {
                    wt = 1;
                } else {
                    const double ratio = log(uniform53(R.v2, R.v3)) / log(bb);
                    wt = (ratio >= 2147483646.0) ? 0x7FFFFFFF : 1 + (int32_t)ratio;
                }
            }
        }
        stage.push(acc, (int32_t)i, (int32_t)j, wt, out);
    }
    stage.flush(out);
}

int val_blocks(int64_t n) {
    int64_t b = (n + kValThreads * 8 - 1) / (kValThreads * 8);
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    return (int)b;
}

}  // namespace

}  // namespace mh

extern "C" {

size_t mh_bruteforce_workspace_bytes(int64_t n) {
    mh::Sizer s;
    s.take<mh::BfCounters>(1);
    s.take<mh::ValAggr>(mh::val_blocks(n));
    return s.used + 512;
}

mh_status mh_sample_bruteforce(const double* x, const double* y, int64_t n, uint64_t seed, uint32_t replica,
                               int64_t row_begin, int64_t row_end, int32_t* src, int32_t* dst, int32_t* w,
                               int64_t capacity, int64_t* n_edges_host, void* workspace, size_t ws_bytes,
                               hipStream_t stream) {
    using namespace mh;
    const bool weighted = (y != nullptr);
    if (!n_edges_host || n < 0 || n > 0x7FFFFFFFll || capacity < 0) return MH_EINVAL;
    if (!x && n > 0) return MH_EINVAL;
    if (capacity > 0 && (!src || !dst || (weighted && !w))) return MH_EINVAL;
    *n_edges_host = 0;
    if (row_begin < 0) row_begin = 0;
    if (row_end > n) row_end = n;
    if (n == 0) return MH_OK;
    if (!workspace || ws_bytes < mh_bruteforce_workspace_bytes(n)) return MH_EWORKSPACE;
    Arena ar(workspace, ws_bytes);
    BfCounters* ctr = ar.take<BfCounters>(1);
    const int vb = val_blocks(n);
    ValAggr* aggr = ar.take<ValAggr>(vb);
    if (ar.overflow) return MH_EWORKSPACE;
    hipLaunchKernelGGL(k_bf_init, dim3(1), dim3(64), 0, stream, ctr);
    MH_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_validate, dim3(vb), dim3(kValThreads), 0, stream, x, y, n, aggr, &ctr->status);
    MH_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_validate_final, dim3(1), dim3(64), 0, stream, aggr, vb, weighted, &ctr->status);
    MH_HIP_TRY(hipGetLastError());
    if (row_begin < row_end) {
        const int64_t rows = row_end - row_begin;
        if ((n + kChunkCols - 1) / kChunkCols > 65535) return MH_EINVAL;  // grid.y limit
        const dim3 grid((unsigned)((rows + kWavesPerBlock - 1) / kWavesPerBlock),
                        (unsigned)((n + kChunkCols - 1) / kChunkCols));
        const EdgeOut out{src, dst, w, capacity, &ctr->n_edges};
        const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
        if (weighted)
            hipLaunchKernelGGL(k_bruteforce<true>, grid, dim3(kThreads), 0, stream, x, y, n, row_begin, row_end, k0, k1,
                               replica, out, &ctr->status);
        else
            hipLaunchKernelGGL(k_bruteforce<false>, grid, dim3(kThreads), 0, stream, x, y, n, row_begin, row_end, k0, k1,
                               replica, out, &ctr->status);
        MH_HIP_TRY(hipGetLastError());
    }
    BfCounters hc;
    MH_HIP_TRY(hipMemcpyAsync(&hc, ctr, sizeof(hc), hipMemcpyDeviceToHost, stream));
    MH_HIP_TRY(hipStreamSynchronize(stream));
    if (hc.status != 0) return (mh_status)hc.status;
    *n_edges_host = (int64_t)hc.n_edges;
    if ((int64_t)hc.n_edges > capacity) return MH_ECAPACITY;
    return MH_OK;
}

}  // extern "C"

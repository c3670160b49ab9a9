// Batched ensembles: many networks x many replicas in one persistent launch.
//
// mh_batch_prepare orders, bounds and plans every network once (A1-A3); each
// mh_batch_sample_async call then lays the items of all requested (network,
// replica) samples end to end and runs one resident grid over them: a wave's
// lanes take items strided over the whole batch, so small and large networks,
// hub segments and tail rows are mixed on every wave.  The call is
// asynchronous and launches kernels only (no memset or host copies), so it can
// be captured in a hipGraph (mh_batch_capture) and replayed.
// mh_batch_autotune times the sweep over candidate segment targets and grid
// sizes on a probe batch and keeps the fastest.
#include <vector>

#include "mh_common.hpp"
#include "mh_internal.hpp"
#include "mh_prepare.hpp"
#include "mh_stage.hpp"
#include "mh_sweep_core.hpp"

namespace mh {

namespace {

constexpr int kThreads = kSweepThreads;

// Items per sample; a network index outside [0, n_networks) makes the call fail
// (MH_EINVAL through the status word, which stops the sweep before it reads).
__global__ __launch_bounds__(kThreads) void k_batch_items(const NetDesc* __restrict__ nets, int32_t n_networks,
                                                          const int32_t* __restrict__ sample_net, int32_t n_samples,
                                                          uint64_t* __restrict__ items, int32_t* status) {
    const int32_t s = blockIdx.x * kThreads + threadIdx.x;
    if (s >= n_samples) return;
    const int32_t k = sample_net[s];
    if (k < 0 || k >= n_networks) {
        raise_status(status, MH_EINVAL);
        items[s] = 0;
        return;
    }
    items[s] = (uint64_t)total_items(nets[k]);
}

__global__ __launch_bounds__(kThreads) void k_batch_zero_degrees(const NetDesc* __restrict__ nets, int32_t n_networks,
                                                                 const int32_t* __restrict__ sample_net,
                                                                 const int64_t* __restrict__ deg_off, int32_t n_samples,
                                                                 int32_t* __restrict__ degrees) {
    for (int32_t s = blockIdx.y; s < n_samples; s += gridDim.y) {
        const int32_t k = sample_net[s];
        if (k < 0 || k >= n_networks) continue;
        const int64_t n = nets[k].n;
        int32_t* d = degrees + deg_off[s];
        for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
            d[i] = 0;
    }
}

// Start of a sampling call: clears the edge count and statistics, and the
// status of any earlier call; a preparation error (invalid networks) stays.
__global__ void k_batch_init(Counters* c) {
    if (threadIdx.x == 0) {
        c->n_edges = 0;
        for (int i = 0; i < ST_COUNT; ++i) c->stats[i].v = 0;
        c->status = c->prep_status;
    }
}

// End of a preparation: its status becomes the batch's preparation status.
__global__ void k_batch_seal(Counters* c) {
    if (threadIdx.x == 0) c->prep_status = c->status;
}

struct BatchLayout {
    Counters* ctr;
    NetDesc* nets;
    uint64_t* item_off;
    std::vector<NetBuffers> bufs;
    void* scratch;
    size_t scratch_bytes;
};

bool layout(const mh_network* nets, int32_t n_networks, int32_t max_samples, void* ws, size_t ws_bytes,
            BatchLayout* L, size_t* bytes_out) {
    size_t bytes = 0;
    int64_t max_n = 0;
    {
        Sizer s;
        s.take<Counters>(1);
        s.take<NetDesc>(n_networks);
        s.take<uint64_t>((size_t)max_samples + 1);
        bytes = s.used;
        for (int32_t i = 0; i < n_networks; ++i) {
            bytes = ((bytes + 255) & ~size_t(255)) + network_bytes(nets[i].n, nets[i].y != nullptr, nets[i].seg_work);
            if (nets[i].n > max_n) max_n = nets[i].n;
        }
        size_t scratch = prepare_scratch_bytes(max_n);
        const size_t s2 = scan_workspace_bytes((int64_t)max_samples + 1);
        if (s2 > scratch) scratch = s2;
        bytes = ((bytes + 255) & ~size_t(255)) + scratch + 512;
    }
    if (bytes_out) *bytes_out = bytes;
    if (!L) return true;
    if (!ws || ws_bytes < bytes) return false;
    Arena ar(ws, ws_bytes);
    L->ctr = ar.take<Counters>(1);
    L->nets = ar.take<NetDesc>(n_networks);
    L->item_off = ar.take<uint64_t>((size_t)max_samples + 1);
    L->bufs.resize(n_networks);
    for (int32_t i = 0; i < n_networks; ++i) {
        Arena sub(ar.base + ((ar.used + 255) & ~size_t(255)), ws_bytes - ((ar.used + 255) & ~size_t(255)));
        L->bufs[i] = carve_network(sub, nets[i].n, nets[i].y != nullptr, nets[i].seg_work);
        ar.used = ((ar.used + 255) & ~size_t(255)) + network_bytes(nets[i].n, nets[i].y != nullptr, nets[i].seg_work);
    }
    const size_t off = (ar.used + 255) & ~size_t(255);
    L->scratch = ar.base + off;
    L->scratch_bytes = ws_bytes - off;
    return !ar.overflow;
}

bool check_networks(const mh_network* nets, int32_t n_networks, bool* weighted) {
    if (!nets || n_networks <= 0) return false;
    const bool w = nets[0].y != nullptr;
    for (int32_t i = 0; i < n_networks; ++i) {
        if (nets[i].n < 0 || nets[i].n > 0x7FFFFFFFll || nets[i].seg_work < 0) return false;
        if (nets[i].n > 0 && !nets[i].x) return false;
        if ((nets[i].y != nullptr) != w) return false;
    }
    *weighted = w;
    return true;
}

template <bool W, int OUT>
mh_status launch_batch(const SweepLaunch& A, int32_t grid_blocks, hipStream_t stream) {
    auto kern = k_sweep<W, false, true, OUT>;
    const int64_t cap = resident_blocks(kern, kThreads);
    const int64_t g = (grid_blocks > 0 && grid_blocks < cap) ? grid_blocks : cap;
    hipLaunchKernelGGL(kern, dim3((unsigned)g), dim3(kThreads), 0, stream, A);
    MH_HIP_TRY(hipGetLastError());
    return MH_OK;
}

}  // namespace

}  // namespace mh

extern "C" {

size_t mh_batch_workspace_bytes(const mh_network* nets, int32_t n_networks, int32_t max_samples) {
    bool weighted;
    if (!mh::check_networks(nets, n_networks, &weighted) || max_samples < 0) return 0;
    size_t bytes = 0;
    mh::layout(nets, n_networks, max_samples, nullptr, 0, nullptr, &bytes);
    return bytes;
}

mh_status mh_batch_prepare(const mh_network* nets, int32_t n_networks, int32_t max_samples, void* workspace,
                           size_t ws_bytes, hipStream_t stream) {
    using namespace mh;
    bool weighted;
    if (!check_networks(nets, n_networks, &weighted) || max_samples < 0) return MH_EINVAL;
    BatchLayout L;
    if (!layout(nets, n_networks, max_samples, workspace, ws_bytes, &L, nullptr)) return MH_EWORKSPACE;
    mh_status st = init_counters(L.ctr, stream);
    if (st != MH_OK) return st;
    std::vector<NetDesc> descs(n_networks);
    for (int32_t i = 0; i < n_networks; ++i) {
        st = prepare_network(nets[i].x, nets[i].y, L.bufs[i], &L.ctr->status, L.scratch, L.scratch_bytes, stream,
                             nullptr);
        if (st != MH_OK) return st;
        descs[i] = net_desc(L.bufs[i]);
    }
    MH_HIP_TRY(hipMemcpyAsync(L.nets, descs.data(), sizeof(NetDesc) * n_networks, hipMemcpyHostToDevice, stream));
    hipLaunchKernelGGL(k_batch_seal, dim3(1), dim3(64), 0, stream, L.ctr);
    MH_HIP_TRY(hipGetLastError());
    Counters hc;
    MH_HIP_TRY(hipMemcpyAsync(&hc, L.ctr, sizeof(hc), hipMemcpyDeviceToHost, stream));
    MH_HIP_TRY(hipStreamSynchronize(stream));
    return hc.status != 0 ? (mh_status)hc.status : MH_OK;
}

mh_status mh_batch_sample_async(const mh_network* nets, int32_t n_networks, int32_t max_samples, void* workspace,
                                size_t ws_bytes, const int32_t* sample_net, const uint32_t* sample_rep,
                                int32_t n_samples, uint64_t seed, int32_t mode, int32_t* src, int32_t* dst, int32_t* w,
                                int32_t* sid, int64_t capacity, int32_t* degrees, const int64_t* deg_off,
                                int32_t grid_blocks, hipStream_t stream) {
    using namespace mh;
    bool weighted;
    if (!check_networks(nets, n_networks, &weighted)) return MH_EINVAL;
    if (n_samples < 0 || n_samples > max_samples || (n_samples > 0 && (!sample_net || !sample_rep))) return MH_EINVAL;
    if (mode == MH_BATCH_EDGES) {
        if (capacity < 0 || (capacity > 0 && (!src || !dst || (weighted && !w)))) return MH_EINVAL;
    } else if (mode == MH_BATCH_DEGREES) {
        if (n_samples > 0 && (!degrees || !deg_off)) return MH_EINVAL;
    } else {
        return MH_EINVAL;
    }
    BatchLayout L;
    if (!layout(nets, n_networks, max_samples, workspace, ws_bytes, &L, nullptr)) return MH_EWORKSPACE;
    hipLaunchKernelGGL(k_batch_init, dim3(1), dim3(64), 0, stream, L.ctr);
    MH_HIP_TRY(hipGetLastError());
    if (n_samples == 0) return MH_OK;
    hipLaunchKernelGGL(k_batch_items, dim3((unsigned)((n_samples + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                       stream, L.nets, n_networks, sample_net, n_samples, L.item_off, &L.ctr->status);
    MH_HIP_TRY(hipGetLastError());
    mh_status st = scan_exclusive_u64(L.item_off, L.item_off, n_samples, L.scratch, L.scratch_bytes, stream);
    if (st != MH_OK) return st;
    if (mode == MH_BATCH_DEGREES) {
        const dim3 zg(64, (unsigned)(n_samples < 4096 ? n_samples : 4096));
        hipLaunchKernelGGL(k_batch_zero_degrees, zg, dim3(kThreads), 0, stream, L.nets, n_networks, sample_net, deg_off,
                           n_samples, degrees);
        MH_HIP_TRY(hipGetLastError());
    }
    SweepLaunch A{};
    A.batch.nets = L.nets;
    A.batch.sample_net = sample_net;
    A.batch.sample_rep = sample_rep;
    A.batch.item_off = L.item_off;
    A.batch.n_samples = n_samples;
    A.batch.degrees = degrees;
    A.batch.deg_off = deg_off;
    A.key0 = (uint32_t)seed;
    A.key1 = (uint32_t)(seed >> 32);
    A.out = EdgeOut{src, dst, w, mode == MH_BATCH_EDGES ? capacity : 0, &L.ctr->n_edges};
    A.sid = sid;
    A.ctr = L.ctr;
    if (mode == MH_BATCH_EDGES)
        return weighted ? launch_batch<true, OUT_EDGES>(A, grid_blocks, stream)
                        : launch_batch<false, OUT_EDGES>(A, grid_blocks, stream);
    return weighted ? launch_batch<true, OUT_DEGREES>(A, grid_blocks, stream)
                    : launch_batch<false, OUT_DEGREES>(A, grid_blocks, stream);
}

mh_status mh_batch_result(const mh_network* nets, int32_t n_networks, int32_t max_samples, void* workspace,
                          size_t ws_bytes, int64_t* n_edges_host, int64_t capacity, hipStream_t stream) {
    using namespace mh;
    bool weighted;
    if (!check_networks(nets, n_networks, &weighted) || !n_edges_host) return MH_EINVAL;
    BatchLayout L;
    if (!layout(nets, n_networks, max_samples, workspace, ws_bytes, &L, nullptr)) return MH_EWORKSPACE;
    Counters hc;
    MH_HIP_TRY(hipMemcpyAsync(&hc, L.ctr, sizeof(hc), hipMemcpyDeviceToHost, stream));
    MH_HIP_TRY(hipStreamSynchronize(stream));
    *n_edges_host = (int64_t)hc.n_edges;
    if (hc.status != 0) return (mh_status)hc.status;
    if (capacity >= 0 && (int64_t)hc.n_edges > capacity) return MH_ECAPACITY;
    return MH_OK;
}

mh_status mh_batch_capture(const mh_network* nets, int32_t n_networks, int32_t max_samples, void* workspace,
                           size_t ws_bytes, const int32_t* sample_net, const uint32_t* sample_rep, int32_t n_samples,
                           uint64_t seed, int32_t mode, int32_t* src, int32_t* dst, int32_t* w, int32_t* sid,
                           int64_t capacity, int32_t* degrees, const int64_t* deg_off, int32_t grid_blocks,
                           hipStream_t stream, hipGraphExec_t* exec_out) {
    if (!exec_out) return MH_EINVAL;
    *exec_out = nullptr;
    // The legacy default stream cannot be captured: capture on a stream of our
    // own (default priority) ordered after the caller's work, then drop it.
    hipStream_t cap = stream;
    if (stream == nullptr) {
        MH_HIP_TRY(hipStreamSynchronize(nullptr));
        MH_HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    }
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        if (cap != stream) (void)hipStreamDestroy(cap);
        return MH_EHIP;
    }
    mh_status st = mh_batch_sample_async(nets, n_networks, max_samples, workspace, ws_bytes, sample_net, sample_rep,
                                         n_samples, seed, mode, src, dst, w, sid, capacity, degrees, deg_off,
                                         grid_blocks, cap);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cap, &graph);
    if (cap != stream) (void)hipStreamDestroy(cap);
    if (st != MH_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return MH_EHIP;
    e = hipGraphInstantiate(exec_out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    return e == hipSuccess ? MH_OK : MH_EHIP;
}

mh_status mh_graph_launch(hipGraphExec_t exec, hipStream_t stream) {
    if (!exec) return MH_EINVAL;
    return hipGraphLaunch(exec, stream) == hipSuccess ? MH_OK : MH_EHIP;
}

mh_status mh_graph_destroy(hipGraphExec_t exec) {
    if (!exec) return MH_OK;
    return hipGraphExecDestroy(exec) == hipSuccess ? MH_OK : MH_EHIP;
}

mh_status mh_batch_autotune(mh_network* nets, int32_t n_networks, int32_t max_samples, void* workspace,
                            size_t ws_bytes, const int32_t* sample_net, const uint32_t* sample_rep, int32_t n_samples,
                            int32_t* degrees, const int64_t* deg_off, const int32_t* seg_candidates, int32_t n_seg,
                            const int32_t* grid_candidates, int32_t n_grid, mh_tuning* best, hipStream_t stream) {
    using namespace mh;
    if (!nets || !seg_candidates || n_seg <= 0 || !best) return MH_EINVAL;
    const int32_t default_grid[1] = {0};
    if (!grid_candidates || n_grid <= 0) {
        grid_candidates = default_grid;
        n_grid = 1;
    }
    std::vector<int32_t> saved(n_networks);
    for (int32_t i = 0; i < n_networks; ++i) saved[i] = nets[i].seg_work;
    hipEvent_t e0, e1;
    MH_HIP_TRY(hipEventCreate(&e0));
    MH_HIP_TRY(hipEventCreate(&e1));
    best->seg_work = -1;
    best->grid_blocks = 0;
    best->ms = 3.0e38f;
    mh_status result = MH_OK;
    for (int32_t a = 0; a < n_seg && result == MH_OK; ++a) {
        if (seg_candidates[a] < 0) continue;
        for (int32_t i = 0; i < n_networks; ++i) nets[i].seg_work = seg_candidates[a];
        if (mh_batch_workspace_bytes(nets, n_networks, max_samples) > ws_bytes) continue;
        result = mh_batch_prepare(nets, n_networks, max_samples, workspace, ws_bytes, stream);
        if (result != MH_OK) break;
        for (int32_t b = 0; b < n_grid && result == MH_OK; ++b) {
            float times[3];
            for (int rep = 0; rep < 3 && result == MH_OK; ++rep) {
                if (hipEventRecord(e0, stream) != hipSuccess) { result = MH_EHIP; break; }
                result = mh_batch_sample_async(nets, n_networks, max_samples, workspace, ws_bytes, sample_net,
                                               sample_rep, n_samples, 1, MH_BATCH_DEGREES, nullptr, nullptr, nullptr,
                                               nullptr, 0, degrees, deg_off, grid_candidates[b], stream);
                if (result != MH_OK) break;
                if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&times[rep], e0, e1) != hipSuccess) {
                    result = MH_EHIP;
                    break;
                }
            }
            if (result != MH_OK) break;
            float t = times[0];  // median of three
            if ((times[1] <= times[0] && times[0] <= times[2]) || (times[2] <= times[0] && times[0] <= times[1]))
                t = times[0];
            else if ((times[0] <= times[1] && times[1] <= times[2]) || (times[2] <= times[1] && times[1] <= times[0]))
                t = times[1];
            else
                t = times[2];
            if (t < best->ms) {
                best->ms = t;
                best->seg_work = seg_candidates[a];
                best->grid_blocks = grid_candidates[b];
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result != MH_OK) {
        for (int32_t i = 0; i < n_networks; ++i) nets[i].seg_work = saved[i];
        return result;
    }
    if (best->seg_work < 0) {
        for (int32_t i = 0; i < n_networks; ++i) nets[i].seg_work = saved[i];
        return MH_EWORKSPACE;
    }
    for (int32_t i = 0; i < n_networks; ++i) nets[i].seg_work = best->seg_work;
    return mh_batch_prepare(nets, n_networks, max_samples, workspace, ws_bytes, stream);
}

}  // extern "C"

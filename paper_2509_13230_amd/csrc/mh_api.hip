// C-ABI entry points for the individual steps (order, bound) and status text.
// The samplers live in mh_sweep.hip and mh_bf.hip, the expected-degree calls
// in mh_degree.hip.
#include <mutex>

#include "mh_common.hpp"
#include "mh_internal.hpp"

namespace mh {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_facts_mu;
int g_cus[kMaxDevices];
struct Occupancy {
    int dev;
    const void* kernel;
    int threads;
    int per_cu;
};
constexpr int kMaxOccupancy = 256;
Occupancy g_occ[kMaxOccupancy];
int g_occ_used = 0;
}  // namespace

int device_cus() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 256;
    {
        std::lock_guard<std::mutex> lk(g_facts_mu);
        if (g_cus[dev] > 0) return g_cus[dev];
    }
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) return 256;
    std::lock_guard<std::mutex> lk(g_facts_mu);
    g_cus[dev] = v;
    return v;
}

int blocks_per_cu(const void* kernel, int threads) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    {
        std::lock_guard<std::mutex> lk(g_facts_mu);
        for (int i = 0; i < g_occ_used; ++i)
            if (g_occ[i].dev == dev && g_occ[i].kernel == kernel && g_occ[i].threads == threads) return g_occ[i].per_cu;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
        return 1;
    std::lock_guard<std::mutex> lk(g_facts_mu);
    if (g_occ_used < kMaxOccupancy) g_occ[g_occ_used++] = Occupancy{dev, kernel, threads, per_cu};
    return per_cu;
}

}  // namespace mh

extern "C" {

mh_status mh_order(const double* x, const double* y, int64_t n, int32_t* perm, double* zs, double* ys,
                   int32_t* status_dev, void* workspace, size_t ws_bytes, hipStream_t stream) {
    if (n < 0 || n > 0x7FFFFFFFll) return MH_EINVAL;
    if (n == 0) return MH_OK;
    if (!x || !perm || !zs || (y && !ys)) return MH_EINVAL;
    if (!workspace || ws_bytes < mh::order_workspace_bytes(n)) return MH_EWORKSPACE;
    return mh::order_nodes(x, y, n, perm, zs, ys, nullptr, status_dev, nullptr, nullptr, nullptr, nullptr, workspace,
                           ws_bytes, stream);
}

size_t mh_bound_workspace_bytes(int64_t n) { return mh::bound_workspace_bytes(n); }

mh_status mh_bound(const double* ys, int64_t n, double* c, void* workspace, size_t ws_bytes, hipStream_t stream) {
    if (n < 0) return MH_EINVAL;
    if (n == 0) return MH_OK;
    if (!ys || !c) return MH_EINVAL;
    if (!workspace || ws_bytes < mh::bound_workspace_bytes(n)) return MH_EWORKSPACE;
    return mh::bound_suffix_top2(ys, n, c, nullptr, workspace, ws_bytes, stream);
}

const char* mh_status_string(mh_status s) {
    switch (s) {
        case MH_OK: return "ok";
        case MH_EINVAL: return "invalid argument or parameters";
        case MH_ECAPACITY: return "output capacity too small";
        case MH_EHIP: return "HIP runtime error";
        case MH_EWORKSPACE: return "workspace missing or too small";
    }
    return "unknown status";
}

}  // extern "C"

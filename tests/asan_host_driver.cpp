// Host-side checks of libmh's argument handling and workspace arithmetic,
// built with AddressSanitizer on the host code (tests/test_host_asan.py).
// Every call here returns before any HIP call: sizes, and the argument and
// workspace checks that precede the first kernel.  Host arrays that the
// library reads (network descriptors) are heap blocks of exactly the stated
// length, so a read past their end is reported.  Device pointers are stand-ins
// that the library must never dereference on the host.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "mh.h"

static int g_fail = 0;
#define EXPECT(cond)                                                   \
    do {                                                               \
        if (!(cond)) {                                                 \
            std::fprintf(stderr, "FAILED line %d: %s\n", __LINE__, #cond); \
            ++g_fail;                                                  \
        }                                                              \
    } while (0)

int main() {
    // stand-ins for device buffers (never read on the host)
    std::vector<double> dev_d(16);
    std::vector<int32_t> dev_i(16);
    double* X = dev_d.data();
    int32_t* I = dev_i.data();
    void* WS = dev_d.data();
    int64_t ne = -7;
    mh_stats st;

    // workspace sizes: positive, growing with n, zero-node cases handled
    mh_plan_params plan{};
    for (int32_t sw : {0, 1, 8, 32, 1024}) {
        plan.seg_work = sw;
        size_t prev = 0;
        for (int64_t n : {0ll, 1ll, 2ll, 4095ll, 4096ll, 4097ll, 1000000ll, 1048576ll, 1048577ll, 2147483647ll}) {
            for (int wgt : {0, 1}) {
                const size_t b = mh_workspace_bytes(n, wgt, &plan);
                EXPECT(b > 0);
                if (wgt == 0) {
                    EXPECT(b >= prev);
                    prev = b;
                }
            }
            EXPECT(mh_bipartite_workspace_bytes(n, n / 2 + 1, 0, &plan) > 0);
        }
    }
    EXPECT(mh_workspace_bytes(1000, 0, nullptr) > 0);
    EXPECT(mh_bruteforce_workspace_bytes(1000) > 0);
    EXPECT(mh_bound_workspace_bytes(1000) > 0);
    EXPECT(mh_plan_workspace_bytes(1000) > 0);
    EXPECT(mh_sort_edges_workspace_bytes(1000) > 0);
    EXPECT(mh_triangles_workspace_bytes(1000, 5000) > 0);

    // status strings, known and unknown codes
    for (int s = -8; s <= 1; ++s) EXPECT(mh_status_string((mh_status)s) != nullptr);

    // single-sample samplers: argument and workspace errors come first
    plan.seg_work = 8;
    EXPECT(mh_sample_unweighted(X, 10, 1, 0, &plan, I, I, 16, nullptr, WS, 1 << 20, nullptr, nullptr) == MH_EINVAL);
    EXPECT(mh_sample_unweighted(nullptr, 10, 1, 0, &plan, I, I, 16, &ne, WS, 1 << 20, &st, nullptr) == MH_EINVAL);
    EXPECT(ne == 0);
    EXPECT(mh_sample_unweighted(X, -1, 1, 0, &plan, I, I, 16, &ne, WS, 1 << 20, nullptr, nullptr) == MH_EINVAL);
    EXPECT(mh_sample_unweighted(X, 10, 1, 0, &plan, I, I, -1, &ne, WS, 1 << 20, nullptr, nullptr) == MH_EINVAL);
    EXPECT(mh_sample_unweighted(X, 10, 1, 0, &plan, nullptr, I, 16, &ne, WS, 1 << 20, nullptr, nullptr) == MH_EINVAL);
    EXPECT(mh_sample_unweighted(X, 10, 1, 0, &plan, I, I, 16, &ne, WS, 64, nullptr, nullptr) == MH_EWORKSPACE);
    EXPECT(mh_sample_unweighted(X, 10, 1, 0, &plan, I, I, 16, &ne, nullptr, 1 << 20, nullptr, nullptr) == MH_EWORKSPACE);
    mh_plan_params bad = plan;
    bad.flags = 1;
    EXPECT(mh_sample_unweighted(X, 10, 1, 0, &bad, I, I, 16, &ne, WS, 1 << 20, nullptr, nullptr) == MH_EINVAL);
    bad = plan;
    bad.seg_work = -1;
    EXPECT(mh_sample_unweighted(X, 10, 1, 0, &bad, I, I, 16, &ne, WS, 1 << 20, nullptr, nullptr) == MH_EINVAL);
    EXPECT(mh_sample_unweighted(X, 0, 1, 0, &plan, nullptr, nullptr, 0, &ne, nullptr, 0, &st, nullptr) == MH_OK);
    EXPECT(ne == 0 && st.n_edges == 0);
    EXPECT(mh_sample_weighted(X, X, 10, 1, 0, &plan, I, I, nullptr, 16, &ne, WS, 1 << 20, nullptr, nullptr) ==
           MH_EINVAL);
    EXPECT(mh_sample_unweighted_async(X, 10, 1, 0, &plan, I, I, 16, WS, 64, nullptr) == MH_EWORKSPACE);
    EXPECT(mh_sample_result(WS, 1 << 20, 16, nullptr, nullptr) == MH_EINVAL);
    EXPECT(mh_sample_result(nullptr, 0, 16, &ne, nullptr) == MH_EWORKSPACE);
    EXPECT(mh_sample_chung_lu(nullptr, 10, 1, 0, &plan, I, I, 16, &ne, WS, 1 << 20, nullptr, nullptr) == MH_EINVAL);
    EXPECT(mh_sample_rank_counts(X, 10, 7, 1, 0, &plan, I, &ne, WS, 1 << 20, nullptr, nullptr) == MH_EINVAL);
    EXPECT(mh_sample_unweighted_noalloc(X, (int64_t)MH_NOALLOC_MAX_NODES + 1, 1, 0, &plan, I, I, 16, &ne, nullptr,
                                        nullptr) == MH_EINVAL);
    EXPECT(mh_sample_bruteforce(X, nullptr, -3, 1, 0, 0, 10, I, I, nullptr, 16, &ne, WS, 1 << 20, nullptr) ==
           MH_EINVAL);
    EXPECT(mh_sample_bruteforce(X, nullptr, 10, 1, 0, 0, 10, I, I, nullptr, 16, &ne, WS, 8, nullptr) ==
           MH_EWORKSPACE);

    // step-level calls
    EXPECT(mh_order(X, nullptr, -1, I, X, nullptr, nullptr, WS, 1 << 20, nullptr) == MH_EINVAL);
    EXPECT(mh_order(X, nullptr, 10, nullptr, X, nullptr, nullptr, WS, 1 << 20, nullptr) == MH_EINVAL);
    EXPECT(mh_order(X, nullptr, 10, I, X, nullptr, nullptr, WS, 8, nullptr) == MH_EWORKSPACE);
    EXPECT(mh_bound(X, -1, X, WS, 1 << 20, nullptr) == MH_EINVAL);
    EXPECT(mh_bound(X, 10, nullptr, WS, 1 << 20, nullptr) == MH_EINVAL);
    EXPECT(mh_expected_degree_fwd(X, nullptr, nullptr, -1, X, nullptr, nullptr) == MH_EINVAL);
    EXPECT(mh_sort_edges(I, I, nullptr, -1, WS, 1 << 20, nullptr) == MH_EINVAL);
    EXPECT(mh_sort_edges(nullptr, I, nullptr, 10, WS, 1 << 20, nullptr) == MH_EINVAL);
    EXPECT(mh_sort_edges(I, I, nullptr, 10, WS, 8, nullptr) == MH_EWORKSPACE);
    uint64_t tri = 0;
    EXPECT(mh_count_triangles(I, I, 10, 5, nullptr, WS, 1 << 20, nullptr) == MH_EINVAL);
    EXPECT(mh_count_triangles(I, I, -1, 5, &tri, WS, 1 << 20, nullptr) == MH_EINVAL);
    EXPECT(mh_count_triangles(I, I, 10, 5, &tri, WS, 8, nullptr) == MH_EWORKSPACE);
    EXPECT(mh_graph_launch(nullptr, nullptr) == MH_EINVAL);
    EXPECT(mh_graph_destroy(nullptr) == MH_OK);

    // batches: descriptors in heap blocks of exactly n_networks entries
    for (int32_t k : {1, 2, 7, 300}) {
        mh_network* nets = static_cast<mh_network*>(std::malloc(sizeof(mh_network) * (size_t)k));
        for (int32_t i = 0; i < k; ++i) {
            nets[i].n = 1 + (int64_t)i * 997 % 200000;
            nets[i].x = X;
            nets[i].y = nullptr;
            nets[i].seg_work = (i % 3) * 8;
        }
        for (int32_t ms : {0, 1, 16, 4096}) {
            const size_t b = mh_batch_workspace_bytes(nets, k, ms);
            EXPECT(b > 0);
            EXPECT(mh_batch_prepare(nets, k, ms, WS, 64, nullptr) == MH_EWORKSPACE);
        }
        EXPECT(mh_batch_workspace_bytes(nets, k, -1) == 0);
        // a bad mode, too many samples, a staged call with a negative capacity
        EXPECT(mh_batch_sample_async(nets, k, 4, WS, 1 << 20, I, reinterpret_cast<const uint32_t*>(I), 2, 1, 9,
                                     I, I, nullptr, nullptr, 16, nullptr, nullptr, 0, nullptr) == MH_EINVAL);
        EXPECT(mh_batch_sample_async(nets, k, 4, WS, 1 << 20, I, reinterpret_cast<const uint32_t*>(I), 5, 1,
                                     MH_BATCH_EDGES, I, I, nullptr, nullptr, 16, nullptr, nullptr, 0,
                                     nullptr) == MH_EINVAL);
        EXPECT(mh_batch_sample_async(nets, k, 4, WS, 1 << 20, I, reinterpret_cast<const uint32_t*>(I), 2, 1,
                                     MH_BATCH_DEGREES_STAGED, I, nullptr, nullptr, nullptr, -1, I,
                                     reinterpret_cast<const int64_t*>(X), 0, nullptr) == MH_EINVAL);
        EXPECT(mh_batch_result(nets, k, 4, WS, 1 << 20, nullptr, 16, nullptr) == MH_EINVAL);
        // invalid descriptors: negative size, missing x, mixed models
        nets[k - 1].n = -1;
        EXPECT(mh_batch_workspace_bytes(nets, k, 16) == 0);
        EXPECT(mh_batch_prepare(nets, k, 16, WS, 1 << 20, nullptr) == MH_EINVAL);
        nets[k - 1].n = 10;
        nets[k - 1].x = nullptr;
        EXPECT(mh_batch_prepare(nets, k, 16, WS, 1 << 20, nullptr) == MH_EINVAL);
        nets[k - 1].x = X;
        if (k > 1) {
            nets[k - 1].y = X;
            EXPECT(mh_batch_prepare(nets, k, 16, WS, 1 << 20, nullptr) == MH_EINVAL);
        }
        std::free(nets);
    }
    EXPECT(mh_batch_workspace_bytes(nullptr, 3, 16) == 0);

    std::printf("asan host driver: %d failed\n", g_fail);
    return g_fail == 0 ? 0 : 1;
}

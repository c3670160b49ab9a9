// The sampler: plan of row segments and the per-segment rejection sweep
// (Sec. 2.3-2.5, Alg. 1), plus the two sampling entry points of the C-ABI.
//
// Work items are (row, segment) pairs.  Rows cut into two or more segments
// ("heavy" rows, the large-z hubs) come first in the item space, one item per
// segment in row order; then every row r < n-1 in rank order, which is an item
// only if the row has exactly one segment.  Each lane runs one item's chain;
// a lane whose chain ends takes the wave's next item, so the 64 lanes stay
// busy whatever the spread of chain lengths.  Waves take items strided by the
// number of waves, which mixes hub segments and tail rows on every wave.
#include "mh_common.hpp"
#include "mh_internal.hpp"
#include "mh_stage.hpp"

namespace mh {

namespace {

constexpr int kThreads = 256;
constexpr int kWavesPerBlock = kThreads / kWave;

enum { ST_STEPS = 0, ST_PROPOSALS, ST_ACCEPTS, ST_SEGMENTS, ST_SATURATED, ST_COUNT };

struct Counters {
    unsigned long long n_edges;
    unsigned long long stats[ST_COUNT];
    int32_t status;
    int32_t pad;
};

__global__ __launch_bounds__(kThreads) void k_mass_of_sorted(const double* __restrict__ zs, int64_t n,
                                                             uint64_t* __restrict__ mass) {
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r < n) mass[r] = mass_q(zs[r]);
}

__global__ void k_init_counters(Counters* c) {
    if (threadIdx.x == 0) {
        c->n_edges = 0;
        for (int i = 0; i < ST_COUNT; ++i) c->stats[i] = 0;
        c->status = 0;
        c->pad = 0;
    }
}

// ---- plan: per row, the number of segments and the data to locate them ----
__global__ __launch_bounds__(kThreads) void k_row_plan(const double* __restrict__ zs, const double* __restrict__ c,
                                                       int64_t n, int32_t T, const uint64_t* __restrict__ P,
                                                       int32_t* __restrict__ nseg, int32_t* __restrict__ jend,
                                                       uint64_t* __restrict__ mq, uint64_t* __restrict__ hn) {
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r >= n) return;
    int64_t total = 0;
    const double s = zs[r];
    if (r < n - 1 && s != 0.0) {
        if (T <= 0) {
            total = 1;
        } else {
            const double cr = c ? c[r] : 1.0;
            int64_t J = r + 1;
            if (s * zs[r + 1] >= cr) {
                int64_t lo = r + 2, hi = n;  // first j in [lo, n] with s*zs[j] < cr (n if none)
                while (lo < hi) {
                    const int64_t mid = lo + (hi - lo) / 2;
                    if (s * zs[mid] < cr) hi = mid; else lo = mid + 1;
                }
                J = lo;
            }
            const int64_t nd = (J - r - 1 + T - 1) / T;
            int64_t ns = 0;
            uint64_t m = 0;
            if (J < n) {
                const double md = ((double)T * cr / s) * 4294967296.0;
                if (!(md < 4611686018427387904.0)) m = (uint64_t)1 << 62;
                else if (md < 1.0) m = 1;
                else m = (uint64_t)md;
                const uint64_t mass = P[n] - P[J];
                ns = (mass == 0) ? 1 : (int64_t)((mass + m - 1) / m);
            }
            total = nd + ns;
            jend[r] = (int32_t)J;
            mq[r] = m;
        }
    }
    nseg[r] = total > 0x7FFFFFFF ? 0x7FFFFFFF : (int32_t)total;
    if (hn) hn[r] = total >= 2 ? (uint64_t)total : 0ull;
}

struct SweepArgs {
    const double* zs;
    const double* ys;
    const double* c;
    const int32_t* perm;
    const int32_t* nseg;
    const int32_t* jend;
    const uint64_t* mq;
    const uint64_t* P;
    const uint64_t* hoff;  // null when unsegmented
    int64_t n;
    int32_t T;
    uint32_t key0, key1;
    uint32_t replica;
    EdgeOut out;
    Counters* ctr;
};

__device__ __forceinline__ int64_t lower_bound_u64(const uint64_t* __restrict__ a, int64_t lo, int64_t hi, uint64_t v) {
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] >= v) hi = mid; else lo = mid + 1;
    }
    return lo;
}

struct Chain {
    int64_t pos, end;
    double s, cr, ysr, tq;
    uint32_t id, step, tag;
};

// Locate item `it` and set up its chain.  Returns false for items that draw nothing.
template <bool WEIGHTED>
__device__ __forceinline__ bool setup_item(const SweepArgs& A, int64_t it, int64_t H, Chain& ch, uint32_t& segs) {
    int64_t r, g, a, b;
    const int64_t n = A.n;
    if (it < H) {
        int64_t lo = 0, hi = n;  // first row index with hoff > it, minus one
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (A.hoff[mid] > (uint64_t)it) hi = mid; else lo = mid + 1;
        }
        r = lo - 1;
        g = it - (int64_t)A.hoff[r];
        const int64_t nsg = (int64_t)(A.hoff[r + 1] - A.hoff[r]);
        const int64_t J = A.jend[r];
        const int64_t T = A.T;
        const int64_t nd = (J - r - 1 + T - 1) / T;
        if (g < nd) {
            a = r + 1 + g * T;
            b = a + T < J ? a + T : J;
        } else {
            const int64_t kk = g - nd;
            const int64_t ns = nsg - nd;
            const uint64_t base = A.P[J];
            const uint64_t m = A.mq[r];
            a = (kk == 0) ? J : lower_bound_u64(A.P, J, n, base + (uint64_t)kk * m);
            b = (kk == ns - 1) ? n : lower_bound_u64(A.P, J, n, base + (uint64_t)(kk + 1) * m);
        }
    } else {
        r = it - H;
        if (A.nseg[r] != 1) return false;
        g = 0;
        a = r + 1;
        b = n;
    }
    if (a >= b) return false;
    ++segs;
    ch.s = A.zs[r];
    ch.id = (uint32_t)A.perm[r];
    ch.cr = WEIGHTED ? A.c[r] : 1.0;
    ch.ysr = WEIGHTED ? A.ys[r] : 0.0;
    ch.pos = a - 1;
    ch.end = b;
    ch.tq = ch.s * A.zs[a - 1];
    ch.step = 0;
    ch.tag = (uint32_t)(g << 1);
    return ch.tq != 0.0;
}

template <bool WEIGHTED, bool STATS>
__global__ __launch_bounds__(kThreads) void k_sweep(SweepArgs A) {
    __shared__ int32_t s_src[kWavesPerBlock][kStageEdges];
    __shared__ int32_t s_dst[kWavesPerBlock][kStageEdges];
    __shared__ int32_t s_w[WEIGHTED ? kWavesPerBlock : 1][WEIGHTED ? kStageEdges : 1];
    if (A.ctr->status != 0) return;

    const int wave = threadIdx.x >> 6;
    const int64_t gwave = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    const int64_t H = A.hoff ? (int64_t)A.hoff[A.n] : 0;
    const int64_t total = H + (A.n > 1 ? A.n - 1 : 0);
    const uint64_t lt = lanemask_lt();

    WaveStage<WEIGHTED> stage{s_src[wave], s_dst[wave], WEIGHTED ? s_w[wave] : nullptr, 0u};

    uint32_t st_steps = 0, st_props = 0, st_acc = 0, st_segs = 0, st_sat = 0;
    Chain ch;
    ch.pos = ch.end = 0;
    ch.s = ch.cr = ch.ysr = ch.tq = 0.0;
    ch.id = ch.step = ch.tag = 0;
    bool active = false;
    int64_t kbase = 0;

    for (;;) {
        const uint64_t idle = __ballot(!active);
        if (idle) {
            if (!active) {
                const int64_t it = gwave + (kbase + __popcll(idle & lt)) * nwaves;
                if (it < total) active = setup_item<WEIGHTED>(A, it, H, ch, st_segs);
            }
            kbase += __popcll(idle);
        }
        if (__ballot(active) == 0) {
            if (gwave + kbase * nwaves >= total) break;
            continue;
        }
        bool acc = false;
        int32_t dst_id = 0, wt = 0;
        if (active) {
            const u32x4 R = philox4x32_10(ch.step, ch.id, A.replica, ch.tag, A.key0, A.key1);
            ++st_steps;
            const double U1 = uniform53(R.v0, R.v1);
            const double U2 = uniform53(R.v2, R.v3);
            const double lq = WEIGHTED ? log1p(ch.tq / ch.cr) : log1p(ch.tq);
            const double d = -log(U1) / lq;
            const double room = (double)(ch.end - 1 - ch.pos);
            if (d >= room) {
                active = false;
            } else {
                const int64_t j = ch.pos + 1 + (int64_t)d;
                const double t = ch.s * A.zs[j];
                double lhs, rhs, ysj = 0.0;
                if (WEIGHTED) {
                    ysj = A.ys[j];
                    const double e = 1.0 - ch.ysr * ysj;
                    lhs = (U2 * ch.tq) * (e + t);
                    rhs = t * (ch.cr + ch.tq);
                } else {
                    lhs = (U2 * ch.tq) * (1.0 + t);
                    rhs = t * (1.0 + ch.tq);
                }
                ++st_props;
                if (lhs < rhs) {
                    acc = true;
                    ++st_acc;
                    dst_id = A.perm[j];
                    if (WEIGHTED) {
                        const u32x4 V = philox4x32_10(ch.step, ch.id, A.replica, ch.tag | 1u, A.key0, A.key1);
                        const double U3 = uniform53(V.v0, V.v1);
                        const double bb = ch.ysr * ysj;
                        if (bb == 0.0) {
                            wt = 1;
                        } else {
                            const double ratio = log(U3) / log(bb);
                            if (ratio >= 2147483646.0) {
                                wt = 0x7FFFFFFF;
                                ++st_sat;
                            } else {
                                wt = 1 + (int32_t)ratio;
                            }
                        }
                    }
                }
                ch.tq = t;
                ch.pos = j;
                ++ch.step;
            }
        }
        stage.push(acc, (int32_t)ch.id, dst_id, wt, A.out);
    }
    stage.flush(A.out);

    if (STATS) {
        const unsigned long long v0 = wave_sum((unsigned long long)st_steps);
        const unsigned long long v1 = wave_sum((unsigned long long)st_props);
        const unsigned long long v2 = wave_sum((unsigned long long)st_acc);
        const unsigned long long v3 = wave_sum((unsigned long long)st_segs);
        const unsigned long long v4 = wave_sum((unsigned long long)st_sat);
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(&A.ctr->stats[ST_STEPS], v0);
            atomicAdd(&A.ctr->stats[ST_PROPOSALS], v1);
            atomicAdd(&A.ctr->stats[ST_ACCEPTS], v2);
            atomicAdd(&A.ctr->stats[ST_SEGMENTS], v3);
            atomicAdd(&A.ctr->stats[ST_SATURATED], v4);
        }
    }
}

struct Layout {
    Counters* ctr;
    int32_t* perm;
    double* zs;
    double* ys;
    double* c;
    uint64_t* P;
    int32_t* nseg;
    int32_t* jend;
    uint64_t* mq;
    uint64_t* hoff;
    char* scratch;
    size_t scratch_bytes;
};

template <typename A>
void carve(A& ar, int64_t n, bool weighted, bool segmented, Layout* L) {
    auto c = ar.template take<Counters>(1);
    auto perm = ar.template take<int32_t>(n);
    auto zs = ar.template take<double>(n);
    auto ys = ar.template take<double>(weighted ? n : 0);
    auto cc = ar.template take<double>(weighted ? n : 0);
    auto P = ar.template take<uint64_t>(segmented ? n + 1 : 0);
    auto nseg = ar.template take<int32_t>(n);
    auto jend = ar.template take<int32_t>(segmented ? n : 0);
    auto mq = ar.template take<uint64_t>(segmented ? n : 0);
    auto hoff = ar.template take<uint64_t>(segmented ? n + 1 : 0);
    if (L) {
        L->ctr = (Counters*)c;
        L->perm = (int32_t*)perm;
        L->zs = (double*)zs;
        L->ys = weighted ? (double*)ys : nullptr;
        L->c = weighted ? (double*)cc : nullptr;
        L->P = segmented ? (uint64_t*)P : nullptr;
        L->nseg = (int32_t*)nseg;
        L->jend = segmented ? (int32_t*)jend : nullptr;
        L->mq = segmented ? (uint64_t*)mq : nullptr;
        L->hoff = segmented ? (uint64_t*)hoff : nullptr;
    }
}

// Sizer has the same take<T>() calls but returns void; this adapter lets carve() run on both.
struct SizerAdapter {
    Sizer s;
    template <typename T>
    T* take(size_t count) {
        s.take<T>(count);
        return nullptr;
    }
};

size_t sample_workspace_bytes(int64_t n, bool weighted, int32_t T) {
    if (n < 0) return 0;
    SizerAdapter sz;
    carve(sz, n, weighted, T > 0, nullptr);
    size_t scratch = order_workspace_bytes(n);
    size_t s2 = scan_workspace_bytes(n + 1);
    size_t s3 = bound_workspace_bytes(n);
    if (s2 > scratch) scratch = s2;
    if (s3 > scratch) scratch = s3;
    return sz.s.used + scratch + 512;
}

int sweep_grid(int64_t n) {
    int cus = 256;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
    }
    // about one item per lane to start with; at most 8 blocks (32 waves) per CU
    int64_t want = (n + kWave - 1) / kWave;
    if (want < 16) want = 16;
    const int64_t cap = (int64_t)cus * 8;
    return (int)(want < cap ? want : cap);
}

mh_status sample_impl(const double* x, const double* y, int64_t n, uint64_t seed, uint32_t replica,
                      const mh_plan_params* plan, int32_t* src, int32_t* dst, int32_t* w, int64_t capacity,
                      int64_t* n_edges_host, void* workspace, size_t ws_bytes, mh_stats* stats_host,
                      hipStream_t stream) {
    const bool weighted = (y != nullptr);
    if (!n_edges_host || n < 0 || n > 0x7FFFFFFFll || capacity < 0) return MH_EINVAL;
    if (!x && n > 0) return MH_EINVAL;
    if (capacity > 0 && (!src || !dst || (weighted && !w))) return MH_EINVAL;
    const int32_t T = plan ? plan->seg_work : 32;
    if (T < 0 || (plan && plan->flags != 0)) return MH_EINVAL;
    *n_edges_host = 0;
    if (stats_host) *stats_host = mh_stats{0, 0, 0, 0, 0, 0};
    if (n == 0) return MH_OK;
    if (!workspace || ws_bytes < sample_workspace_bytes(n, weighted, T)) return MH_EWORKSPACE;
    const bool seg = T > 0;

    Arena ar(workspace, ws_bytes);
    Layout L;
    carve(ar, n, weighted, seg, &L);
    if (ar.overflow) return MH_EWORKSPACE;
    const size_t off = (ar.used + 255) & ~size_t(255);
    void* scratch = ar.base + off;
    const size_t scratch_bytes = ws_bytes - off;

    hipEvent_t* ev = plan ? plan->stage_events : nullptr;
    if (ev) MH_HIP_TRY(hipEventRecord(ev[0], stream));
    hipLaunchKernelGGL(k_init_counters, dim3(1), dim3(64), 0, stream, L.ctr);
    MH_HIP_TRY(hipGetLastError());
    int32_t* status = &L.ctr->status;
    mh_status st = order_nodes(x, y, n, L.perm, L.zs, L.ys, status, L.P, scratch, scratch_bytes, stream);
    if (st != MH_OK) return st;
    if (ev) MH_HIP_TRY(hipEventRecord(ev[1], stream));
    if (weighted) {
        st = bound_suffix_top2(L.ys, n, L.c, status, scratch, scratch_bytes, stream);
        if (st != MH_OK) return st;
    }
    if (seg) {
        st = scan_exclusive_u64(L.P, L.P, n, scratch, scratch_bytes, stream);
        if (st != MH_OK) return st;
    }
    const unsigned rows_grid = (unsigned)((n + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_row_plan, dim3(rows_grid), dim3(kThreads), 0, stream, L.zs, L.c, n, T, L.P, L.nseg, L.jend,
                       L.mq, L.hoff);
    MH_HIP_TRY(hipGetLastError());
    if (seg) {
        st = scan_exclusive_u64(L.hoff, L.hoff, n, scratch, scratch_bytes, stream);
        if (st != MH_OK) return st;
    }

    if (ev) MH_HIP_TRY(hipEventRecord(ev[2], stream));
    SweepArgs A;
    A.zs = L.zs;
    A.ys = L.ys;
    A.c = L.c;
    A.perm = L.perm;
    A.nseg = L.nseg;
    A.jend = L.jend;
    A.mq = L.mq;
    A.P = L.P;
    A.hoff = L.hoff;
    A.n = n;
    A.T = T;
    A.key0 = (uint32_t)seed;
    A.key1 = (uint32_t)(seed >> 32);
    A.replica = replica;
    A.out = EdgeOut{src, dst, w, capacity, &L.ctr->n_edges};
    A.ctr = L.ctr;
    const dim3 grid(sweep_grid(n));
    if (weighted) {
        if (stats_host) hipLaunchKernelGGL((k_sweep<true, true>), grid, dim3(kThreads), 0, stream, A);
        else hipLaunchKernelGGL((k_sweep<true, false>), grid, dim3(kThreads), 0, stream, A);
    } else {
        if (stats_host) hipLaunchKernelGGL((k_sweep<false, true>), grid, dim3(kThreads), 0, stream, A);
        else hipLaunchKernelGGL((k_sweep<false, false>), grid, dim3(kThreads), 0, stream, A);
    }
    MH_HIP_TRY(hipGetLastError());
    if (ev) MH_HIP_TRY(hipEventRecord(ev[3], stream));

    Counters hc;
    MH_HIP_TRY(hipMemcpyAsync(&hc, L.ctr, sizeof(Counters), hipMemcpyDeviceToHost, stream));
    MH_HIP_TRY(hipStreamSynchronize(stream));
    if (hc.status != 0) return (mh_status)hc.status;
    *n_edges_host = (int64_t)hc.n_edges;
    if (stats_host) {
        stats_host->steps = (int64_t)hc.stats[ST_STEPS];
        stats_host->proposals = (int64_t)hc.stats[ST_PROPOSALS];
        stats_host->accepts = (int64_t)hc.stats[ST_ACCEPTS];
        stats_host->segments = (int64_t)hc.stats[ST_SEGMENTS];
        stats_host->saturated_w = (int64_t)hc.stats[ST_SATURATED];
        stats_host->n_edges = (int64_t)hc.n_edges;
    }
    if ((int64_t)hc.n_edges > capacity) return MH_ECAPACITY;
    return MH_OK;
}

}  // namespace

// ---- plan counts entry (also used by the C-ABI) ----
size_t plan_workspace_bytes_impl(int64_t n) {
    Sizer s;
    s.take<uint64_t>(n + 1);
    s.take<int32_t>(n);
    s.take<uint64_t>(n);
    return s.used + scan_workspace_bytes(n + 1) + 512;
}

mh_status plan_counts_impl(const double* zs, const double* c, int64_t n, int32_t T, int32_t* nseg, void* ws,
                           size_t ws_bytes, hipStream_t stream) {
    if (n < 0 || T < 0 || (n > 0 && (!zs || !nseg))) return MH_EINVAL;
    if (n == 0) return MH_OK;
    Arena ar(ws, ws_bytes);
    uint64_t* P = ar.take<uint64_t>(n + 1);
    int32_t* jend = ar.take<int32_t>(n);
    uint64_t* mq = ar.take<uint64_t>(n);
    if (ar.overflow) return MH_EWORKSPACE;
    const size_t off = (ar.used + 255) & ~size_t(255);
    const unsigned grid = (unsigned)((n + kThreads - 1) / kThreads);
    if (T > 0) {
        hipLaunchKernelGGL(k_mass_of_sorted, dim3(grid), dim3(kThreads), 0, stream, zs, n, P);
        MH_HIP_TRY(hipGetLastError());
        mh_status st = scan_exclusive_u64(P, P, n, ar.base + off, ws_bytes - off, stream);
        if (st != MH_OK) return st;
    }
    hipLaunchKernelGGL(k_row_plan, dim3(grid), dim3(kThreads), 0, stream, zs, c, n, T, P, nseg, jend, mq,
                       (uint64_t*)nullptr);
    MH_HIP_TRY(hipGetLastError());
    return MH_OK;
}

}  // namespace mh

extern "C" {

size_t mh_workspace_bytes(int64_t n, int weighted, const mh_plan_params* plan) {
    return mh::sample_workspace_bytes(n, weighted != 0, plan ? plan->seg_work : 32);
}

mh_status mh_sample_unweighted(const double* x, int64_t n, uint64_t seed, uint32_t replica,
                               const mh_plan_params* plan, int32_t* src, int32_t* dst, int64_t capacity,
                               int64_t* n_edges_host, void* workspace, size_t ws_bytes, mh_stats* stats_host,
                               hipStream_t stream) {
    return mh::sample_impl(x, nullptr, n, seed, replica, plan, src, dst, nullptr, capacity, n_edges_host, workspace,
                           ws_bytes, stats_host, stream);
}

mh_status mh_sample_weighted(const double* x, const double* y, int64_t n, uint64_t seed, uint32_t replica,
                             const mh_plan_params* plan, int32_t* src, int32_t* dst, int32_t* w, int64_t capacity,
                             int64_t* n_edges_host, void* workspace, size_t ws_bytes, mh_stats* stats_host,
                             hipStream_t stream) {
    if (!y && n > 0) return MH_EINVAL;
    if (n == 0) {
        if (!n_edges_host) return MH_EINVAL;
        *n_edges_host = 0;
        if (stats_host) *stats_host = mh_stats{0, 0, 0, 0, 0, 0};
        return MH_OK;
    }
    return mh::sample_impl(x, y, n, seed, replica, plan, src, dst, w, capacity, n_edges_host, workspace, ws_bytes,
                           stats_host, stream);
}

size_t mh_plan_workspace_bytes(int64_t n) { return mh::plan_workspace_bytes_impl(n); }

mh_status mh_plan_counts(const double* zs, const double* c, int64_t n, int32_t seg_work, int32_t* nseg,
                         void* workspace, size_t ws_bytes, hipStream_t stream) {
    return mh::plan_counts_impl(zs, c, n, seg_work, nseg, workspace, ws_bytes, stream);
}

}  // extern "C"

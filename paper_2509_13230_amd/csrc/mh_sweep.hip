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

struct HeavyRec {
    int32_t r, g, a, b;
};

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
    const HeavyRec* rec;   // records of the first rec_cap heavy items
    int64_t rec_cap;
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

// Row, segment index and column range of heavy item `it` (it < H).
__device__ HeavyRec heavy_record(const SweepArgs& A, int64_t it) {
    const int64_t n = A.n;
    int64_t lo = 0, hi = n;  // first row index with hoff > it, minus one
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (A.hoff[mid] > (uint64_t)it) hi = mid; else lo = mid + 1;
    }
    const int64_t r = lo - 1;
    const int64_t g = it - (int64_t)A.hoff[r];
    const int64_t nsg = (int64_t)(A.hoff[r + 1] - A.hoff[r]);
    const int64_t J = A.jend[r];
    const int64_t T = A.T;
    const int64_t nd = (J - r - 1 + T - 1) / T;
    int64_t a, b;
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
    return HeavyRec{(int32_t)r, (int32_t)g, (int32_t)a, (int32_t)b};
}

__global__ __launch_bounds__(kThreads) void k_heavy_records(SweepArgs A, HeavyRec* __restrict__ rec) {
    if (A.ctr->status != 0) return;
    const int64_t H = (int64_t)A.hoff[A.n];
    const int64_t lim = H < A.rec_cap ? H : A.rec_cap;
    for (int64_t it = (int64_t)blockIdx.x * kThreads + threadIdx.x; it < lim; it += (int64_t)gridDim.x * kThreads)
        rec[it] = heavy_record(A, it);
}

// Lane states of the sweep.  Every loop iteration a lane consumes the global
// loads it issued in the previous iteration and issues the next ones, so one
// memory round trip per iteration is overlapped with the Philox block and the
// logarithm of the next draw, which need no loaded data.
enum : uint32_t { S_IDLE = 0, S_REC, S_LOAD, S_STEP, S_DONE };

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
    const int32_t n32 = (int32_t)A.n;
    const uint64_t lt = lanemask_lt();

    WaveStage<WEIGHTED> stage{s_src[wave], s_dst[wave], WEIGHTED ? s_w[wave] : nullptr, 0u};

    uint32_t st_steps = 0, st_props = 0, st_acc = 0, st_segs = 0, st_sat = 0;
    uint32_t state = S_IDLE;
    bool check_light = false;
    int32_t r = 0, pos = 0, end = 0, jc = 0;
    uint32_t step = 0, tag = 0, scand = 0;
    int32_t id = 0;
    double s = 0.0, cr = 1.0, ysr = 0.0, tq = 0.0, U2 = 0.0;
    // values in flight from the previous iteration's loads
    double ld_s = 0.0, ld_z = 0.0, ld_c = 1.0, ld_y = 0.0;
    int32_t ld_id = 0, ld_n = 1;
    HeavyRec ld_rec{0, 0, 0, 0};
    int64_t kbase = 0;

    for (;;) {
        // 1. the next draw of every lane that will draw this iteration (no loaded data needed)
        const bool draws = (state == S_STEP) || (state == S_LOAD);
        double E = 0.0, U2n = 0.0;
        if (draws) {
            const u32x4 R = philox4x32_10(step, (uint32_t)r, A.replica, tag, A.key0, A.key1);
            E = -log(uniform53(R.v0, R.v1));
            U2n = uniform53(R.v2, R.v3);
        }
        // 2. consume the loads of the previous iteration
        bool acc = false, go = false;
        int32_t dst_id = 0, wt = 0;
        if (state == S_STEP) {
            const double t = s * ld_z;
            double lhs, rhs;
            if (WEIGHTED) {
                const double e = 1.0 - ysr * ld_y;
                lhs = (U2 * tq) * (e + t);
                rhs = t * (cr + tq);
            } else {
                lhs = (U2 * tq) * (1.0 + t);
                rhs = t * (1.0 + tq);
            }
            ++st_props;
            if (lhs < rhs) {
                acc = true;
                ++st_acc;
                dst_id = ld_id;
                if (WEIGHTED) {
                    const double bb = ysr * ld_y;
                    if (bb == 0.0) {
                        wt = 1;
                    } else {
                        const u32x4 V = philox4x32_10(scand, (uint32_t)r, A.replica, tag | 1u, A.key0, A.key1);
                        const double ratio = log(uniform53(V.v0, V.v1)) / log(bb);
                        if (ratio >= 2147483646.0) {
                            wt = 0x7FFFFFFF;
                            ++st_sat;
                        } else {
                            wt = 1 + (int32_t)ratio;
                        }
                    }
                }
            }
            tq = t;
            pos = jc;
            go = true;
        } else if (state == S_LOAD) {
            if (check_light && ld_n != 1) {
                state = S_IDLE;
            } else {
                s = ld_s;
                id = ld_id;
                tq = s * ld_z;
                cr = WEIGHTED ? ld_c : 1.0;
                ysr = WEIGHTED ? ld_y : 0.0;
                ++st_segs;
                go = true;
            }
        } else if (state == S_REC) {
            r = ld_rec.r;
            pos = ld_rec.a - 1;
            end = ld_rec.b;
            tag = (uint32_t)ld_rec.g << 1;
            step = 0;
            check_light = false;
            if (ld_rec.a >= ld_rec.b) {
                state = S_IDLE;
            } else {
                ld_s = A.zs[r];
                ld_z = A.zs[pos];
                ld_id = A.perm[r];
                if (WEIGHTED) {
                    ld_c = A.c[r];
                    ld_y = A.ys[r];
                }
                state = S_LOAD;
            }
        }
        // 3. the skip: candidate pos + 1 + floor(-log U1 / -log(1 - q)), or the end of the segment
        if (go) {
            if (tq == 0.0) {
                state = S_IDLE;
            } else {
                ++st_steps;
                const double lq = WEIGHTED ? log1p(tq / cr) : log1p(tq);
                const double d = E / lq;
                const double room = (double)(end - 1 - pos);
                if (d >= room) {
                    state = S_IDLE;
                } else {
                    jc = pos + 1 + (int32_t)d;
                    U2 = U2n;
                    scand = step;
                    ++step;
                    ld_z = A.zs[jc];
                    ld_id = A.perm[jc];
                    if (WEIGHTED) ld_y = A.ys[jc];
                    state = S_STEP;
                }
            }
        }
        // 4. idle lanes take the wave's next items and issue their loads
        const uint64_t idle = __ballot(state == S_IDLE);
        if (idle) {
            if (state == S_IDLE) {
                const int64_t it = gwave + (kbase + __popcll(idle & lt)) * nwaves;
                if (it >= total) {
                    state = S_DONE;
                } else if (it < H) {
                    ld_rec = (it < A.rec_cap) ? A.rec[it] : heavy_record(A, it);
                    state = S_REC;
                } else {
                    r = (int32_t)(it - H);
                    pos = r;
                    end = n32;
                    tag = 0;
                    step = 0;
                    check_light = true;
                    ld_n = A.nseg[r];
                    ld_s = A.zs[r];
                    ld_z = ld_s;
                    ld_id = A.perm[r];
                    if (WEIGHTED) {
                        ld_c = A.c[r];
                        ld_y = A.ys[r];
                    }
                    state = S_LOAD;
                }
            }
            kbase += __popcll(idle);
        }
        stage.push(acc, id, dst_id, wt, A.out);
        if (__ballot(state != S_DONE) == 0) break;
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
    HeavyRec* rec;
    int64_t rec_cap;
    char* scratch;
    size_t scratch_bytes;
};

// Records kept for up to this many heavy items; items beyond it are located
// inside the sweep (slower, same result).
int64_t heavy_record_capacity(int64_t n) { return n + 4096; }

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
    const int64_t rec_cap = segmented ? heavy_record_capacity(n) : 0;
    auto rec = ar.template take<HeavyRec>(rec_cap);
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
        L->rec = (HeavyRec*)rec;
        L->rec_cap = rec_cap;
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

template <typename K>
int resident_grid(K kernel, int64_t n) {
    int cus = 256, dev = 0, per_cu = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0) != hipSuccess || per_cu < 1)
        per_cu = 4;
    // every block resident at once: the sweep's waves take their items in turn
    int64_t want = (n + kWave - 1) / kWave;
    if (want < 16) want = 16;
    const int64_t cap = (int64_t)cus * per_cu;
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
    A.rec = L.rec;
    A.rec_cap = L.rec_cap;
    A.n = n;
    A.T = T;
    A.key0 = (uint32_t)seed;
    A.key1 = (uint32_t)(seed >> 32);
    A.replica = replica;
    A.out = EdgeOut{src, dst, w, capacity, &L.ctr->n_edges};
    A.ctr = L.ctr;
    if (seg) {
        hipLaunchKernelGGL(k_heavy_records, dim3(512), dim3(kThreads), 0, stream, A, L.rec);
        MH_HIP_TRY(hipGetLastError());
    }
    if (ev) MH_HIP_TRY(hipEventRecord(ev[2], stream));
    if (weighted) {
        if (stats_host) hipLaunchKernelGGL((k_sweep<true, true>), dim3(resident_grid(k_sweep<true, true>, n)), dim3(kThreads), 0, stream, A);
        else hipLaunchKernelGGL((k_sweep<true, false>), dim3(resident_grid(k_sweep<true, false>, n)), dim3(kThreads), 0, stream, A);
    } else {
        if (stats_host) hipLaunchKernelGGL((k_sweep<false, true>), dim3(resident_grid(k_sweep<false, true>, n)), dim3(kThreads), 0, stream, A);
        else hipLaunchKernelGGL((k_sweep<false, false>), dim3(resident_grid(k_sweep<false, false>, n)), dim3(kThreads), 0, stream, A);
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

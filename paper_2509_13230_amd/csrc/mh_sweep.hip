// Single-sample entry points: node order, bound, plan of row segments, and
// the per-segment rejection sweep (Sec. 2.3-2.5, Alg. 1; the sweep itself is
// in mh_sweep_core.hpp).
#include <mutex>

#include "mh_common.hpp"
#include "mh_internal.hpp"
#include "mh_lookback.hpp"
#include "mh_stage.hpp"
#include "mh_sweep_core.hpp"
#include "mh_prepare.hpp"

namespace mh {

// seg_work when no plan is given: the measured optimum on N = 1e6 power-law
// networks (whole sample, sweep and plan together)
constexpr int32_t kDefaultSegWork = 8;

namespace {

constexpr int kThreads = kSweepThreads;

// Packs separately given sorted z into node records and their column masses
// (used by the stand-alone plan entry point).
__global__ __launch_bounds__(kThreads) void k_pack_sorted(const double* __restrict__ zs, int64_t n,
                                                          NodeRec* __restrict__ node, uint64_t* __restrict__ mass) {
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r >= n) return;
    node[r].z = zs[r];
    node[r].id = (int32_t)r;
    if (mass) mass[r] = mass_q(zs[r]);
}

__global__ __launch_bounds__(kThreads) void k_unpack_nseg(const NodeRec* __restrict__ node, int64_t n,
                                                          int32_t* __restrict__ nseg) {
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r < n) nseg[r] = node[r].nseg;
}

__global__ void k_init_counters(Counters* c) {
    if (threadIdx.x == 0) {
        c->n_edges = 0;
        for (int i = 0; i < ST_COUNT; ++i) c->stats[i].v = 0;
        c->status = 0;
        c->prep_status = 0;
    }
}

// ---- plan: per row, the number of segments and the data to locate them ----
// Row r's columns are [first, nc) with first = r + 1 (one node set, col ==
// node) or 0 (two node sets).  Dense part: the columns j < J with
// s z_j >= c_r, cut every T columns; sparse part: [J, nc) cut where the column
// mass (prefix sums P of floor(z 2^32)) reaches multiples of
// m = floor(T c_r / s 2^32), the mass whose expected candidate count is ~T.
// J and m are stored for rows of two or more segments only (no other row reads
// them).  One row per thread; a block that holds a row with a dense part (the
// hubs, a few blocks at most) stages z of every zstep-th column in LDS, so the
// search for J takes its bracket from LDS and ends with log2(zstep) loads.
constexpr int kPlanThreads = 1024;
constexpr int kPlanSamples = 4096;
// z of the columns right after a tile's first row, staged with the samples:
// the dense part of a hub row ends within a few thousand columns (J is where
// s z_j drops below c_r, and only the largest z reach that far), so most
// searches for J end in LDS.
constexpr int kPlanHead = 4096;

// z of every zstep-th column into LDS (zstep: the smallest power of two >= 256
// that leaves at most kPlanSamples samples); returns zstep, sets *nz.  From
// zsamp (z[256 k], contiguous) when given: a gather of one record per 4 KB
// page costs an address translation each.  With s_zh, also z of the columns
// [h0, h0 + nh) (nh = min(kPlanHead, nc - h0)), all loads in flight together.
__device__ __forceinline__ int64_t stage_col_samples(const NodeRec* __restrict__ col, const double* zsamp,
                                                     int64_t nc, double* s_z, int64_t* nz, double* s_zh = nullptr,
                                                     int64_t h0 = 0, int64_t* nh = nullptr) {
    int64_t zstep = 256;
    while ((nc - 1) / zstep + 1 > kPlanSamples) zstep *= 2;
    *nz = (nc - 1) / zstep + 1;
    static_assert(kPlanSamples <= 4 * kPlanThreads && kPlanHead <= 4 * kPlanThreads, "four values per thread");
    const int64_t sstep = zstep >> kSampleShift;
    const int64_t cnt = *nz;
    const int64_t hcnt = s_zh ? (nc - h0 < kPlanHead ? nc - h0 : kPlanHead) : 0;
    if (nh) *nh = hcnt > 0 ? hcnt : 0;
    double v[4], w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t j = threadIdx.x + (int64_t)q * blockDim.x;
        const int64_t jj = j < cnt ? j : cnt - 1;
        v[q] = zsamp ? zsamp[jj * sstep] : col[jj * zstep].z;
        const int64_t k = j < hcnt ? j : (hcnt > 0 ? hcnt - 1 : 0);
        w[q] = hcnt > 0 ? col[h0 + k].z : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t j = threadIdx.x + (int64_t)q * blockDim.x;
        if (j < cnt) s_z[j] = v[q];
        if (j < hcnt) s_zh[j] = w[q];
    }
    return zstep;
}

// J of a row with a dense part: first j in [first + 1, nc) with s z_j < cr
// (nc if none).  Within the staged head columns [h0, h0 + nh) when it lies
// there (a binary search in LDS), else bracketed by the LDS samples and found
// by a binary search in global memory.
__device__ __forceinline__ int64_t dense_end(const NodeRec* __restrict__ col, int64_t nc, double s, double cr,
                                             int64_t first, const double* s_z, int64_t nz, int64_t zstep,
                                             const double* s_zh, int64_t h0, int64_t nh) {
    int64_t from = first + 1;
    if (nh > 0 && from >= h0 && from < h0 + nh) {
        if (h0 + nh == nc || s * s_zh[nh - 1] < cr) {
            int lo = (int)(from - h0), hi = (int)nh;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (s * s_zh[mid] < cr) hi = mid; else lo = mid + 1;
            }
            return h0 + lo;
        }
        from = h0 + nh;  // s z_j >= cr over the whole window
    }
    int ql = 0, qh = (int)nz;  // first sample where s z < cr
    while (ql < qh) {
        const int mid = (ql + qh) >> 1;
        if (s * s_z[mid] < cr) qh = mid; else ql = mid + 1;
    }
    int64_t lo = from;
    if (ql > 0 && (int64_t)(ql - 1) * zstep + 1 > lo) lo = (int64_t)(ql - 1) * zstep + 1;
    int64_t hi = nc;  // s z < cr holds at hi (or hi = nc)
    if (ql < (int)nz) hi = (int64_t)ql * zstep > lo ? (int64_t)ql * zstep : lo;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (s * col[mid].z < cr) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// Plan of row r given J: segment count (0 for an empty row), J and m stored
// for rows of two or more segments, nseg into the record.
__device__ __forceinline__ int64_t plan_row(NodeRec* __restrict__ node, int64_t r, double s, double cr,
                                            int64_t first, int64_t J, bool active, int64_t nc, int32_t T,
                                            const uint64_t* __restrict__ P, int32_t* __restrict__ jend,
                                            uint64_t* __restrict__ mq) {
    int64_t total = 0;
    if (active) {
        if (T <= 0) {
            total = 1;
        } else {
            // (J - first < 2^31 and mass <= m for most rows: no 64-bit division then)
            const int64_t nd = J > first ? (int64_t)((uint32_t)(J - first + T - 1) / (uint32_t)T) : 0;
            int64_t ns = 0;
            uint64_t m = 0;
            if (J < nc) {
                const double md = ((double)T * cr / s) * 4294967296.0;
                if (!(md < 4611686018427387904.0)) m = (uint64_t)1 << 62;
                else if (md < 1.0) m = 1;
                else m = (uint64_t)md;
                const uint64_t mass = P[nc] - P[J];
                ns = (mass <= m) ? 1 : (int64_t)((mass + m - 1) / m);
            }
            total = nd + ns;
            if (total >= 2) {
                jend[r] = (int32_t)J;
                mq[r] = m;
            }
        }
    }
    node[r].nseg = total > 0x7FFFFFFF ? 0x7FFFFFFF : (int32_t)total;
    return total;
}

// One row per thread.  A block that holds a row with a dense part (the hubs,
// a few blocks at most) stages column samples in LDS first.
__global__ __launch_bounds__(kPlanThreads) void k_row_plan(NodeRec* __restrict__ node, const double* __restrict__ c,
                                                           int64_t n, const NodeRec* __restrict__ col,
                                                           const double* __restrict__ zsamp, int64_t nc,
                                                           int32_t bip, int32_t T, const uint64_t* __restrict__ P,
                                                           int32_t* __restrict__ jend, uint64_t* __restrict__ mq,
                                                           uint64_t* __restrict__ hn) {
    __shared__ double s_z[kPlanSamples];
    const int64_t r = (int64_t)blockIdx.x * kPlanThreads + threadIdx.x;
    const bool in = r < n;
    double s = 0.0, cr = 1.0;
    int64_t first = 0;
    bool dense = false, active = false;
    if (in) {
        s = node[r].z;
        first = bip ? 0 : r + 1;
        active = first < nc && s != 0.0;
        if (active && T > 0) {
            cr = c ? c[r] : 1.0;
            dense = s * col[first].z >= cr;
        }
    }
    int64_t J = first;
    if (__syncthreads_or(dense)) {
        int64_t nz;
        const int64_t zstep = stage_col_samples(col, zsamp, nc, s_z, &nz);
        __syncthreads();
        if (dense) J = dense_end(col, nc, s, cr, first, s_z, nz, zstep, nullptr, 0, 0);
    }
    if (!in) return;
    const int64_t total = plan_row(node, r, s, cr, first, J, active, nc, T, P, jend, mq);
    if (hn) hn[r] = total >= 2 ? (uint64_t)total : 0ull;
}

// The row plan and the prefix sums hoff of the heavy-item counts in one
// look-back pass over tiles of 4096 rows (counts below 2^62: up to 2^30 rows).
// For every round of kHrThreads stored items, the row that holds the round's
// first item goes to hbrow[round] (each row writes the rounds that begin inside
// it: at most a few stores per row).  The tile of hub rows stages column
// samples for its dense searches; the other tiles publish their sums at once.
constexpr int kHrThreads = 1024;  // heavy items per round of k_heavy_records

__global__ __launch_bounds__(kLbThreads) void k_row_plan_scan(NodeRec* __restrict__ node,
                                                              const double* __restrict__ c, int64_t n,
                                                              const NodeRec* __restrict__ col,
                                                              const double* __restrict__ zsamp, int64_t nc,
                                                              int32_t bip, int32_t T, const uint64_t* __restrict__ P,
                                                              int32_t* __restrict__ jend, uint64_t* __restrict__ mq,
                                                              uint64_t* __restrict__ hoff, int64_t tiles,
                                                              uint64_t* state, int32_t* __restrict__ hbrow,
                                                              int64_t rec_cap, int32_t* err) {
    __shared__ LbShared sh;
    __shared__ double s_z[kPlanSamples];
    __shared__ double s_zh[kPlanHead];
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t base = tile * kLbTile;
        double s[kLbItems], cr[kLbItems];
        int64_t J[kLbItems];
        bool dense[kLbItems], active[kLbItems];
        bool any = false;
#pragma unroll
        for (int k = 0; k < kLbItems; ++k) {
            const int64_t r = base + k * kLbThreads + threadIdx.x;
            s[k] = 0.0;
            cr[k] = 1.0;
            dense[k] = active[k] = false;
            const int64_t first = bip ? 0 : r + 1;
            J[k] = first;
            if (r < n) {
                s[k] = node[r].z;
                active[k] = first < nc && s[k] != 0.0;
                if (active[k] && T > 0) {
                    cr[k] = c ? c[r] : 1.0;
                    dense[k] = s[k] * col[first].z >= cr[k];
                }
            }
            any = any || dense[k];
        }
        if (__syncthreads_or(any)) {
            int64_t nz, nh;
            const int64_t h0 = bip ? 0 : (base + 1 < nc ? base + 1 : nc);
            const int64_t zstep = stage_col_samples(col, zsamp, nc, s_z, &nz, s_zh, h0, &nh);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kLbItems; ++k)
                if (dense[k]) J[k] = dense_end(col, nc, s[k], cr[k], J[k], s_z, nz, zstep, s_zh, h0, nh);
        }
        uint64_t cnt[kLbItems];
#pragma unroll
        for (int k = 0; k < kLbItems; ++k) {
            const int idx = k * kLbThreads + threadIdx.x;
            const int64_t r = base + idx;
            cnt[k] = 0;
            if (r < n) {
                const int64_t first = bip ? 0 : r + 1;
                const int64_t total = plan_row(node, r, s[k], cr[k], first, J[k], active[k], nc, T, P, jend, mq);
                cnt[k] = total >= 2 ? (uint64_t)total : 0ull;
            }
            sh.items[lb_at(idx)] = cnt[k];
        }
        const uint64_t end = lb_tile_scan(sh, tile, state, err);
#pragma unroll
        for (int k = 0; k < kLbItems; ++k) {
            const int idx = k * kLbThreads + threadIdx.x;
            const int64_t i = base + idx;
            if (i < n) {
                const uint64_t v = sh.items[lb_at(idx)];
                hoff[i] = v;
                const uint64_t stop = v + cnt[k] < (uint64_t)rec_cap ? v + cnt[k] : (uint64_t)rec_cap;
                for (uint64_t b = (v + kHrThreads - 1) / kHrThreads; b * kHrThreads < stop; ++b)
                    hbrow[b] = (int32_t)i;
            }
        }
        if (threadIdx.x == 0 && base + kLbTile >= n) hoff[n] = end;
    }
}

// ---- node records, column masses and row plan in one pass (one unweighted node set) ----
// Made from the sorted keys directly: each tile of 4096 ranks makes its ranks'
// z and id, scans their column masses (look-back 1: P), plans its rows from z
// held in LDS, scans the heavy-item counts (look-back 2: hoff) and writes each
// node record once, segment count included.  P[n], which every row's plan
// needs, is the zeroing kernel's per-tile mass sums added up (their total does
// not depend on the order).  J of a dense row is searched over the tile's
// ranks and the next tile's first one in LDS, else in the sorted keys beyond;
// P at such a J is read from J's tile once that tile has written its P: it
// stores P through to the device's coherence point and then marks its
// look-back word done with a release, which the reader waits for (bounded
// spin) and acquires; so every tile must be resident (one block each).  Only
// a tile that some row's dense part can reach does so: J >= base needs
// s z_(base - 1) >= 1 for a row's s <= z_0, so a tile with
// z_0 z_(base - 1) < 1 is never read this way (fl(s z) <= fl(z_0 z)).
__device__ __forceinline__ double sorted_rank_z(const uint32_t* __restrict__ keys, const uint64_t* __restrict__ vals,
                                                int64_t j, uint32_t kb) {
    return key_value(((uint64_t)(keys[j] + kb) << 32) | (vals[j] >> 32));
}

// First j in [first + 1, n) with s z_j < 1 (n if none), z of ranks base ..
// base + kLbTile in s_zt.
__device__ __forceinline__ int64_t fused_dense_end(const uint32_t* __restrict__ keys, const uint64_t* __restrict__ vals,
                                                   uint32_t kb, int64_t n, int64_t base, const double* s_zt, double s,
                                                   int64_t first) {
    const int64_t wend = base + kLbTile + 1 < n ? base + kLbTile + 1 : n;  // staged ranks [base, wend)
    int64_t lo = first + 1;
    if (lo < wend) {
        if (wend == n || s * s_zt[wend - 1 - base] < 1.0) {
            int a = (int)(lo - base), b = (int)(wend - base);
            while (a < b) {
                const int mid = (a + b) >> 1;
                if (s * s_zt[mid] < 1.0) b = mid; else a = mid + 1;
            }
            return base + a;
        }
        lo = wend;  // s z >= 1 over every staged rank
    }
    int64_t hi = n;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (s * sorted_rank_z(keys, vals, mid, kb) < 1.0) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// P[J] for base + kLbTile < J < n, from J's tile (a later one) once it is
// done writing P.
__device__ __forceinline__ uint64_t fused_prefix_beyond(const uint64_t* P, const uint64_t* state1, int64_t J,
                                                        int32_t* status) {
    const int64_t u = J / kLbTile;  // J's tile, after this one
    uint32_t spins = 0;
    for (;;) {
        const uint64_t w = __hip_atomic_load(&state1[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((w & ~kLbValue) == kLbDone) break;
        if (++spins > kLbSpinLimit) {
            raise_status(status, MH_EHIP);
            return 0;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return __hip_atomic_load(&P[J], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kLbThreads) void k_finish_plan_scan(
    const uint32_t* __restrict__ keys, const uint64_t* __restrict__ vals, const uint32_t* __restrict__ kbase,
    const uint64_t* __restrict__ tile_mass, int64_t n, NodeRec* __restrict__ node, uint64_t* __restrict__ P,
    uint64_t* __restrict__ Psamp, double* __restrict__ Zsamp, int32_t T, int32_t* __restrict__ jend,
    uint64_t* __restrict__ mq, uint64_t* __restrict__ hoff, int64_t tiles, uint64_t* state1, uint64_t* state2,
    int32_t* __restrict__ hbrow, int64_t rec_cap, int32_t* status) {
    __shared__ LbShared sh;
    __shared__ double s_zt[kLbTile + 1];
    __shared__ uint64_t s_pt[kLbTile + 1];
    __shared__ uint64_t s_red[kLbThreads / kWave];
    const uint32_t kb = *kbase;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // P[n]: the per-tile mass sums added up
    uint64_t tm = 0;
    for (int64_t t = threadIdx.x; t < tiles; t += kLbThreads) tm += tile_mass[t];
    tm = wave_sum(tm);
    if (lane == 0) s_red[wave] = tm;
    __syncthreads();
    uint64_t Ptot = 0;
#pragma unroll
    for (int w = 0; w < kLbThreads / kWave; ++w) Ptot += s_red[w];
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t base = tile * kLbTile;
        double z[kLbItems];
        int32_t id[kLbItems];
        // 1. z, id and column mass of the tile's ranks
#pragma unroll
        for (int k = 0; k < kLbItems; ++k) {
            const int idx = k * kLbThreads + threadIdx.x;
            const int64_t r = base + idx;
            z[k] = 0.0;
            id[k] = 0;
            uint64_t m = 0;
            if (r < n) {
                const uint64_t v = vals[r];
                id[k] = (int32_t)(uint32_t)v;
                z[k] = key_value(((uint64_t)(keys[r] + kb) << 32) | (v >> 32));
                m = mass_q(z[k]);
                if ((r & ((1 << kSampleShift) - 1)) == 0) Zsamp[r >> kSampleShift] = z[k];
                if (r == 0 && !isfinite(z[k] * z[k])) raise_status(status, MH_EINVAL);
            }
            s_zt[idx] = z[k];
            sh.items[lb_at(idx)] = m;
        }
        if (threadIdx.x == 0) s_zt[kLbTile] = base + kLbTile < n ? sorted_rank_z(keys, vals, base + kLbTile, kb) : 0.0;
        // whether any row's dense part can reach this tile (then its P is read by other tiles)
        const bool reached = tile > 0 && sorted_rank_z(keys, vals, 0, kb) * sorted_rank_z(keys, vals, base - 1, kb) >= 1.0;
        // 2. P, the exclusive prefix of the masses (look-back 1)
        const uint64_t end1 = lb_tile_scan(sh, tile, state1, status);
#pragma unroll
        for (int k = 0; k < kLbItems; ++k) {
            const int idx = k * kLbThreads + threadIdx.x;
            const int64_t r = base + idx;
            const uint64_t v = sh.items[lb_at(idx)];
            s_pt[idx] = v;
            if (r < n) {
                // a reached tile's P goes through to the coherence point: other
                // tiles of this launch read it
                if (reached) __hip_atomic_store(&P[r], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                else P[r] = v;
                if ((r & ((1 << kSampleShift) - 1)) == 0) Psamp[r >> kSampleShift] = v;
            }
        }
        if (threadIdx.x == 0) {
            s_pt[kLbTile] = end1;  // P at base + kLbTile
            if (base + kLbTile >= n) {
                __hip_atomic_store(&P[n], end1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((n & ((1 << kSampleShift) - 1)) == 0) Psamp[n >> kSampleShift] = end1;
            }
        }
        // a reached tile's P out: every wave's stores complete, then the
        // look-back word marked done with a release (reached is uniform over
        // the block); the barrier also makes s_pt whole for the plan
        if (reached) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        __syncthreads();
        if (reached && threadIdx.x == 0)
            __hip_atomic_store(&state1[tile], kLbDone | end1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        // 3. the row plan, and the records
        uint64_t cnt[kLbItems];
#pragma unroll
        for (int k = 0; k < kLbItems; ++k) {
            const int idx = k * kLbThreads + threadIdx.x;
            const int64_t r = base + idx;
            const int64_t first = r + 1;
            const double s = z[k];
            const double cr = 1.0;
            int64_t total = 0;
            if (r < n && first < n && s != 0.0) {
                if (T <= 0) {
                    total = 1;
                } else {
                    int64_t J = first;
                    uint64_t PJ = s_pt[idx + 1];  // P[r + 1]
                    if (s * s_zt[idx + 1] >= cr) {
                        J = fused_dense_end(keys, vals, kb, n, base, s_zt, s, first);
                        if (J < n) PJ = J <= base + kLbTile ? s_pt[J - base] : fused_prefix_beyond(P, state1, J, status);
                    }
                    const int64_t nd = J > first ? (int64_t)((uint32_t)(J - first + T - 1) / (uint32_t)T) : 0;
                    int64_t ns = 0;
                    uint64_t m = 0;
                    if (J < n) {
                        const double md = ((double)T * cr / s) * 4294967296.0;
                        if (!(md < 4611686018427387904.0)) m = (uint64_t)1 << 62;
                        else if (md < 1.0) m = 1;
                        else m = (uint64_t)md;
                        const uint64_t mass = Ptot - PJ;
                        ns = (mass <= m) ? 1 : (int64_t)((mass + m - 1) / m);
                    }
                    total = nd + ns;
                    if (total >= 2) {
                        jend[r] = (int32_t)J;
                        mq[r] = m;
                    }
                }
            }
            if (r < n) node[r] = NodeRec{s, id[k], total > 0x7FFFFFFF ? 0x7FFFFFFF : (int32_t)total};
            cnt[k] = total >= 2 ? (uint64_t)total : 0ull;
            sh.items[lb_at(idx)] = cnt[k];
        }
        // 4. hoff, the exclusive prefix of the heavy-item counts (look-back 2)
        const uint64_t end2 = lb_tile_scan(sh, tile, state2, status);
#pragma unroll
        for (int k = 0; k < kLbItems; ++k) {
            const int idx = k * kLbThreads + threadIdx.x;
            const int64_t i = base + idx;
            if (i < n) {
                const uint64_t v = sh.items[lb_at(idx)];
                hoff[i] = v;
                const uint64_t stop = v + cnt[k] < (uint64_t)rec_cap ? v + cnt[k] : (uint64_t)rec_cap;
                for (uint64_t b = (v + kHrThreads - 1) / kHrThreads; b * kHrThreads < stop; ++b)
                    hbrow[b] = (int32_t)i;
            }
        }
        if (threadIdx.x == 0 && base + kLbTile >= n) hoff[n] = end2;
    }
}

static mh_status launch_row_plan(NodeRec* node, const double* c, int64_t n, const NodeRec* col, const double* zsamp,
                                 int64_t nc, int32_t bip, int32_t T, const uint64_t* P, int32_t* jend, uint64_t* mq,
                                 uint64_t* hn, hipStream_t stream) {
    const unsigned grid = (unsigned)((n + kPlanThreads - 1) / kPlanThreads);
    hipLaunchKernelGGL(k_row_plan, dim3(grid), dim3(kPlanThreads), 0, stream, node, c, n, col, zsamp, nc, bip, T, P,
                       jend, mq, hn);
    MH_HIP_TRY(hipGetLastError());
    return MH_OK;
}

// Records (16 bytes each) are kept for up to kRecPerRow n + 4096 heavy items;
// the sweep locates any further ones itself, by searches in global memory
// that stall their lanes.  The weighted bound is loose where y is near 1:
// UECM with N = 200,000 (degrees 2.3 on [1, 5000]) has 7.1 n heavy items at
// seg_work 8, against 0.2 n for the unweighted N = 1e6 workload.
constexpr int64_t kRecPerRow = 8;
constexpr int kHrSamples = 4096;  // P samples a block of k_heavy_records stages in LDS
constexpr int kHrRows = 4096;     // rows of hoff a block of k_heavy_records stages in LDS

// Row and column range of the first rec_cap heavy items, the same as
// heavy_record() computes them.  With hbrow and Psamp (P[256 k]): a block takes
// a round of items, stages hoff over the rows from the round's first row on
// (one contiguous load) and the P samples (every step-th one when there are
// more than kHrSamples) in LDS, so each item finds its row in LDS and each cut
// search takes its bracket from LDS and ends with a short binary search in
// global memory.  Otherwise each record is computed whole by plain searches.
__device__ __forceinline__ int64_t first_above_u64(const uint64_t* __restrict__ a, int64_t lo, int64_t hi, uint64_t v) {
    while (lo < hi) {  // first index in [lo, hi) with a[i] > v (hi if none)
        const int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] > v) hi = mid; else lo = mid + 1;
    }
    return lo;
}

__global__ __launch_bounds__(kHrThreads) void k_heavy_records(NetDesc D, HeavyRec* __restrict__ rec,
                                                            const uint64_t* __restrict__ Psamp,
                                                            const int32_t* __restrict__ hbrow,
                                                            const int32_t* status) {
    __shared__ uint64_t s_p[kHrSamples];
    __shared__ uint64_t s_h[kHrRows + 1];
    __shared__ int32_t s_a[kHrThreads];
    if (*status != 0) return;
    const int64_t H = heavy_items(D);
    const int64_t lim = H < D.rec_cap ? H : D.rec_cap;
    if ((int64_t)blockIdx.x * kHrThreads >= lim) return;  // the grid is sized for rec_cap items
    if (!hbrow || !Psamp) {
        for (int64_t it = (int64_t)blockIdx.x * kHrThreads + threadIdx.x; it < lim;
             it += (int64_t)gridDim.x * kHrThreads)
            rec[it] = heavy_record(D, it);
        return;
    }
    const int64_t n = D.n, nc = D.ncol, T = D.T;
    const bool bip = (D.flags & NET_BIPARTITE) != 0;
    // sample stride ps (a multiple of 256 columns) and count
    int64_t pstep = 1;
    while (lb_samples(nc) > pstep * (kHrSamples - 1) + 1) pstep *= 2;
    const int64_t np = (lb_samples(nc) - 1) / pstep + 1;
    const int64_t ps = pstep << kSampleShift;
    static_assert(kHrSamples <= 4 * kHrThreads && kHrRows + 1 <= 5 * kHrThreads, "staging per thread");
    stage_lds<4>(s_p, np, [=](int64_t j) { return Psamp[j * pstep]; });
    for (int64_t round = blockIdx.x; round * kHrThreads < lim; round += gridDim.x) {
        const int64_t R0 = hbrow[round];
        __syncthreads();  // s_h and s_a of the previous round are no longer read
        const uint64_t* hoff = D.hoff;
        stage_lds<5>(s_h, kHrRows + 1, [=](int64_t j) {
            const uint64_t v = hoff[R0 + j <= n ? R0 + j : n];  // loaded unconditionally
            return R0 + j <= n ? v : ~0ull;
        });
        __syncthreads();
        const int64_t it = round * kHrThreads + threadIdx.x;
        const bool active = it < lim;
        int64_t r = 0, g = 0, nsg = 0, a = 0, b = 0;
        bool b_next = false;  // b is the next item's a (the next thread's search)
        if (active) {
            // row: hoff[r] <= it < hoff[r + 1], from the staged rows R0 .. R0 + kHrRows
            int rl = 1, ru = kHrRows + 1;  // first staged index with hoff > it (s_h[0] <= it)
            while (rl < ru) {
                const int mid = (rl + ru) >> 1;
                if (s_h[mid] > (uint64_t)it) ru = mid; else rl = mid + 1;
            }
            if (rl <= kHrRows) {
                r = R0 + rl - 1;
                g = it - (int64_t)s_h[rl - 1];
                nsg = (int64_t)(s_h[rl] - s_h[rl - 1]);
            } else {  // a round spread over more rows than staged (rows without items in between)
                r = first_above_u64(D.hoff, R0 + kHrRows, n + 1, (uint64_t)it) - 1;
                g = it - (int64_t)D.hoff[r];
                nsg = (int64_t)(D.hoff[r + 1] - D.hoff[r]);
            }
            const int64_t J = D.jend[r];
            const int64_t first = bip ? 0 : r + 1;
            const int64_t nd = (J - first + T - 1) / T;
            if (g < nd) {
                a = first + g * T;
                b = a + T < J ? a + T : J;
            } else {
                const int64_t kk = g - nd;
                const int64_t ns = nsg - nd;
                const uint64_t pb = D.P[J];
                const uint64_t m = D.mq[r];
                // The segment's two cuts: first j in [J, nc) with P[j] >= v (nc if
                // none), v = pb + k m for k = kk, kk + 1; the first cut of the row
                // is J and the last nc.  The second is the next item's first when
                // that item (same row) is this round's next thread; otherwise both
                // searches advance in lockstep, so their dependent loads overlap:
                // bracket from the LDS samples, P[(q-1) ps] < v <= P[q ps], then a
                // binary search in global memory.
                b_next = kk + 1 < ns && threadIdx.x + 1 < kHrThreads && it + 1 < lim;
                int64_t lo[2], hi[2];
                uint64_t v[2];
                // interpolation points: P is xp[0] -> yp[0], xp[1] -> yp[1] (sample
                // positions and values around the cut, then probed ones)
                double xl[2], xr[2], yl[2], yr[2];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int64_t k2 = kk + e;
                    v[e] = pb + (uint64_t)k2 * m;
                    xl[e] = xr[e] = 0.0;
                    yl[e] = yr[e] = 0.0;
                    if ((e == 0 && k2 == 0) || (e == 1 && (k2 == ns || b_next))) {
                        lo[e] = hi[e] = (e == 0) ? J : nc;
                        continue;
                    }
                    int ql = 0, qh = (int)np;
                    while (ql < qh) {
                        const int mid = (ql + qh) >> 1;
                        if (s_p[mid] >= v[e]) qh = mid; else ql = mid + 1;
                    }
                    int64_t clo = J, chi = nc;
                    if (ql > 0 && (int64_t)(ql - 1) * ps + 1 > clo) clo = (int64_t)(ql - 1) * ps + 1;
                    if (ql < (int)np && (int64_t)ql * ps < chi) chi = (int64_t)ql * ps;
                    if (clo > nc) clo = nc;
                    if (chi < clo) chi = clo;
                    lo[e] = clo;
                    hi[e] = chi;
                    if (ql > 0 && ql < (int)np) {
                        xl[e] = (double)((int64_t)(ql - 1) * ps);
                        yl[e] = (double)s_p[ql - 1];
                        xr[e] = (double)((int64_t)ql * ps);
                        yr[e] = (double)s_p[ql];
                    }
                }
                // The first two probes of each search where the line through the
                // known points of P meets v (the masses within a bracket change
                // slowly, so the cut is close), then bisection; each probe keeps
                // the bracket exact, so the cut found is the same.
                for (int step = 0; lo[0] < hi[0] || lo[1] < hi[1]; ++step) {
                    int64_t mid[2];
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        mid[e] = lo[e] + (hi[e] - lo[e]) / 2;
                        if (step < 2 && lo[e] < hi[e] && yr[e] > yl[e]) {
                            const double f = ((double)v[e] - yl[e]) / (yr[e] - yl[e]);
                            const double x = xl[e] + f * (xr[e] - xl[e]);
                            int64_t g = x < (double)lo[e] ? lo[e] : (x > (double)(hi[e] - 1) ? hi[e] - 1 : (int64_t)x);
                            mid[e] = g;
                        }
                    }
                    const bool a0 = lo[0] < hi[0], a1 = lo[1] < hi[1];
                    const uint64_t p0 = a0 ? D.P[mid[0]] : 0, p1 = a1 ? D.P[mid[1]] : 0;
                    if (a0) {
                        if (p0 >= v[0]) {
                            hi[0] = mid[0];
                            xr[0] = (double)mid[0];
                            yr[0] = (double)p0;
                        } else {
                            lo[0] = mid[0] + 1;
                            xl[0] = (double)mid[0];
                            yl[0] = (double)p0;
                        }
                    }
                    if (a1) {
                        if (p1 >= v[1]) {
                            hi[1] = mid[1];
                            xr[1] = (double)mid[1];
                            yr[1] = (double)p1;
                        } else {
                            lo[1] = mid[1] + 1;
                            xl[1] = (double)mid[1];
                            yl[1] = (double)p1;
                        }
                    }
                }
                a = lo[0];
                b = lo[1];
            }
        }
        s_a[threadIdx.x] = (int32_t)a;
        __syncthreads();
        if (!active) continue;
        if (b_next) b = s_a[threadIdx.x + 1];
        rec[it] = HeavyRec{(int32_t)r, (int32_t)g, (int32_t)a, (int32_t)b};
    }
}

}  // namespace

// Blocks for the heavy records: one item per thread in rounds of kHrThreads,
// at most the blocks resident at once (the item count is known only on the
// device, so most of a grid sized by rec_cap would be dispatched only to exit;
// the blocks loop over the rounds instead).
static unsigned heavy_grid(int64_t rec_cap) {
    const int64_t want = (rec_cap + kHrThreads - 1) / kHrThreads;
    const int64_t cap = resident_blocks(k_heavy_records, kHrThreads);
    return (unsigned)(want < 1 ? 1 : (want < cap ? want : cap));
}

// A3: segment counts of every row (and J, m) and, when segmented, the prefix
// sums hoff of the heavy rows' counts.  While the sums stay below 2^62 (up to
// 2^30 rows) one look-back kernel plans the rows, scans the counts and writes
// the first row of every round of stored heavy items to hbrow (rows_known);
// beyond, the row plan and three scan kernels.
static mh_status plan_rows(NodeRec* node, const double* c, int64_t n, const NodeRec* col, const double* zsamp,
                           int64_t nc, int32_t bip,
                           int32_t T, const uint64_t* P, int32_t* jend, uint64_t* mq, uint64_t* hoff,
                           uint64_t* hoff_state, int32_t* hbrow, int64_t rec_cap, int32_t* status, void* scratch,
                           size_t scratch_bytes, bool* rows_known, hipStream_t stream) {
    *rows_known = false;
    if (nc > (int64_t)1 << 30) zsamp = nullptr;  // written by the order's one-pass scan only
    if (hoff && n <= (int64_t)1 << 30) {
        const int64_t tiles = lb_tiles(n);
        const int64_t resident = resident_blocks(k_row_plan_scan, kLbThreads);
        const int64_t grid = tiles < resident ? tiles : resident;
        hipLaunchKernelGGL(k_row_plan_scan, dim3((unsigned)grid), dim3(kLbThreads), 0, stream, node, c, n, col,
                           zsamp, nc, bip, T, P, jend, mq, hoff, tiles, hoff_state, hbrow, rec_cap, status);
        MH_HIP_TRY(hipGetLastError());
        *rows_known = true;
        return MH_OK;
    }
    mh_status st = launch_row_plan(node, c, n, col, zsamp, nc, bip, T, P, jend, mq, hoff, stream);
    if (st != MH_OK || !hoff) return st;
    return scan_exclusive_u64(hoff, hoff, n, scratch, scratch_bytes, stream);
}

// ---- one prepared network: buffers, sizes and preparation ----
template <typename A>
static NetBuffers carve_network_impl(A& ar, int64_t n, bool weighted, int32_t T) {
    const bool seg = T > 0;
    NetBuffers B{};
    B.node = ar.template take<NodeRec>(n);
    B.ys = ar.template take<double>(weighted ? n : 0);
    B.c = ar.template take<double>(weighted ? n : 0);
    B.P = ar.template take<uint64_t>(seg ? n + 1 : 0);
    B.jend = ar.template take<int32_t>(seg ? n : 0);
    B.mq = ar.template take<uint64_t>(seg ? n : 0);
    B.hoff = ar.template take<uint64_t>(seg ? n + 1 : 0);
    B.rec_cap = seg ? kRecPerRow * n + 4096 : 0;
    B.scan_words = seg ? 2 * lb_tiles(n) : 0;
    B.scan_state = ar.template take<uint64_t>(B.scan_words);
    B.Psamp = ar.template take<uint64_t>(seg ? lb_samples(n) : 0);
    B.Zsamp = ar.template take<double>(seg ? lb_samples(n) : 0);
    B.hbrow = ar.template take<int32_t>(seg ? B.rec_cap / kHrThreads + 2 : 0);
    B.rec = ar.template take<HeavyRec>(B.rec_cap);  // last: the large, mostly unused reserve
    if (!weighted) B.ys = B.c = nullptr;
    if (!seg)
        B.P = nullptr, B.jend = nullptr, B.mq = nullptr, B.hoff = nullptr, B.scan_state = nullptr, B.Psamp = nullptr,
        B.Zsamp = nullptr, B.hbrow = nullptr;
    B.n = n;
    B.T = T;
    B.weighted = weighted;
    return B;
}

namespace {
struct SizerAdapter {
    Sizer s;
    template <typename T>
    T* take(size_t count) {
        s.take<T>(count);
        return nullptr;
    }
};
}  // namespace

size_t network_bytes(int64_t n, bool weighted, int32_t T) {
    SizerAdapter sz;
    carve_network_impl(sz, n, weighted, T);
    return sz.s.used + 256;
}

NetBuffers carve_network(Arena& ar, int64_t n, bool weighted, int32_t T) {
    return carve_network_impl(ar, n, weighted, T);
}

size_t prepare_scratch_bytes(int64_t n) {
    size_t scratch = order_workspace_bytes(n);
    const size_t s2 = scan_workspace_bytes(n + 1);
    const size_t s3 = bound_workspace_bytes(n);
    if (s2 > scratch) scratch = s2;
    if (s3 > scratch) scratch = s3;
    return scratch + 256;
}

NetDesc net_desc(const NetBuffers& B) {
    NetDesc D;
    D.node = B.node;
    D.ys = B.ys;
    D.c = B.c;
    D.jend = B.jend;
    D.mq = B.mq;
    D.P = B.P;
    D.hoff = B.hoff;
    D.rec = B.rec;
    D.rec_cap = B.rec_cap;
    D.col = B.node;
    D.ysc = B.ys;
    D.n = B.n;
    D.ncol = B.n;
    D.T = B.T;
    D.flags = 0;
    return D;
}

mh_status init_counters(Counters* c, hipStream_t stream) {
    hipLaunchKernelGGL(k_init_counters, dim3(1), dim3(64), 0, stream, c);
    MH_HIP_TRY(hipGetLastError());
    return MH_OK;
}

// Order (A1), bound (A2, weighted) and plan (A3) of one network into B.
mh_status prepare_network(const double* x, const double* y, const NetBuffers& B, int32_t* status, void* scratch,
                          size_t scratch_bytes, hipStream_t stream, hipEvent_t* ev, ZeroRange counters) {
    const int64_t n = B.n;
    if (n <= 0) return MH_OK;
    const bool seg = B.T > 0;
    // one unweighted node set, segmented, every tile resident: records, P and
    // the row plan in one kernel from the sorted keys
    const int64_t tiles = lb_tiles(n);
    const bool try_fused = !B.weighted && seg && n <= (int64_t)1 << 30 && radix_prepares_keys(n) &&
                           tiles <= resident_blocks(k_finish_plan_scan, kLbThreads);
    SortedKeys sk;
    mh_status st = order_nodes(x, B.weighted ? y : nullptr, n, nullptr, nullptr, B.ys, B.node, status, B.P,
                               B.scan_state, B.Psamp, B.Zsamp, scratch, scratch_bytes, stream, true,
                               ZeroRange{B.scan_state, B.scan_words}, counters, try_fused ? &sk : nullptr);
    if (st != MH_OK) return st;
    if (ev && ev[1]) MH_HIP_TRY(hipEventRecord(ev[1], stream));
    if (sk.keys) {
        if (sk.tiles != tiles) return MH_EINVAL;
        hipLaunchKernelGGL(k_finish_plan_scan, dim3((unsigned)tiles), dim3(kLbThreads), 0, stream, sk.keys, sk.vals,
                           sk.kbase, sk.tile_mass, n, B.node, B.P, B.Psamp, B.Zsamp, B.T, B.jend, B.mq, B.hoff, tiles,
                           B.scan_state, B.scan_state + tiles, B.hbrow, B.rec_cap, status);
        MH_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_heavy_records, dim3(heavy_grid(B.rec_cap)), dim3(kHrThreads), 0, stream, net_desc(B),
                           B.rec, (const uint64_t*)B.Psamp, (const int32_t*)B.hbrow, (const int32_t*)status);
        MH_HIP_TRY(hipGetLastError());
        return MH_OK;
    }
    if (B.weighted) {
        st = bound_suffix_top2(B.ys, n, B.c, status, scratch, scratch_bytes, stream);
        if (st != MH_OK) return st;
    }
    bool rows_known = false;
    st = plan_rows(B.node, B.c, n, B.node, B.Zsamp, n, 0, B.T, B.P, B.jend, B.mq, B.hoff,
                   seg ? B.scan_state + lb_tiles(n) : nullptr, B.hbrow, B.rec_cap, status, scratch,
                   scratch_bytes, &rows_known, stream);
    if (st != MH_OK) return st;
    if (seg) {
        // P's samples come from the one-pass scan of the order (up to 2^30 nodes), as rows_known
        hipLaunchKernelGGL(k_heavy_records, dim3(heavy_grid(B.rec_cap)), dim3(kHrThreads), 0, stream, net_desc(B),
                           B.rec, (const uint64_t*)(rows_known ? B.Psamp : nullptr),
                           (const int32_t*)(rows_known ? B.hbrow : nullptr), (const int32_t*)status);
        MH_HIP_TRY(hipGetLastError());
    }
    return MH_OK;
}

namespace {

size_t sample_workspace_bytes(int64_t n, bool weighted, int32_t T) {
    if (n < 0) return 0;
    Sizer s;
    s.take<Counters>(1);
    return s.used + network_bytes(n, weighted, T) + prepare_scratch_bytes(n) + 512;
}

template <bool W, bool S, bool BIP = false, int OUT = OUT_EDGES, bool CL = false>
void launch_sweep(const SweepLaunch& A, int64_t n, int32_t grid_blocks, hipStream_t stream) {
    auto kern = k_sweep<W, S, false, OUT, BIP, CL>;
    int64_t want = (n + kWave - 1) / kWave;
    if (want < 16) want = 16;
    // Default: every block that fits at once (4 per CU unweighted, 3 weighted:
    // the LDS stages bound it).  On N = 1e6 the unweighted sweep takes 64, 53
    // and 51 us at 2, 3 and 4 blocks per CU: more waves per SIMD hide more of
    // each iteration's load.
    int64_t cap = resident_blocks(kern, kThreads);
    if (grid_blocks > 0 && grid_blocks < cap) cap = grid_blocks;
    hipLaunchKernelGGL(kern, dim3((unsigned)(want < cap ? want : cap)), dim3(kThreads), 0, stream, A);
}

// Reads a sample's counters back (waits for the stream).
mh_status read_counters(const Counters* ctr, int64_t capacity, int64_t* n_edges_host, mh_stats* stats_host,
                        hipStream_t stream) {
    Counters hc;
    MH_HIP_TRY(hipMemcpyAsync(&hc, ctr, sizeof(Counters), hipMemcpyDeviceToHost, stream));
    MH_HIP_TRY(hipStreamSynchronize(stream));
    if (hc.status != 0) return (mh_status)hc.status;
    *n_edges_host = (int64_t)hc.n_edges;
    if (stats_host) {
        stats_host->steps = (int64_t)hc.stats[ST_STEPS].v;
        stats_host->proposals = (int64_t)hc.stats[ST_PROPOSALS].v;
        stats_host->accepts = (int64_t)hc.stats[ST_ACCEPTS].v;
        stats_host->segments = (int64_t)hc.stats[ST_SEGMENTS].v;
        stats_host->saturated_w = (int64_t)hc.stats[ST_SATURATED].v;
        stats_host->n_edges = (int64_t)hc.n_edges;
    }
    if ((int64_t)hc.n_edges > capacity) return MH_ECAPACITY;
    return MH_OK;
}

__global__ __launch_bounds__(kThreads) void k_zero_i32(int32_t* __restrict__ a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) a[i] = 0;
}

// Checks the arguments and enqueues a whole sample on `stream`; the counters
// (edge count, status, statistics) are left at the start of the workspace.
// chung_lu: the Chung-Lu chain (unweighted).  rank_cnt: counts by rank
// instead of the edge list (src, dst, w unused; cleared here).
mh_status enqueue_sample(const double* x, const double* y, int64_t n, uint64_t seed, uint32_t replica,
                         const mh_plan_params* plan, int32_t* src, int32_t* dst, int32_t* w, int64_t capacity,
                         void* workspace, size_t ws_bytes, bool stats, hipStream_t stream, bool chung_lu = false,
                         int32_t* rank_cnt = nullptr) {
    const bool weighted = (y != nullptr);
    if (n < 0 || n > 0x7FFFFFFFll || capacity < 0) return MH_EINVAL;
    if (!x && n > 0) return MH_EINVAL;
    if (chung_lu && weighted) return MH_EINVAL;
    if (rank_cnt) {
        if (weighted) return MH_EINVAL;
    } else if (capacity > 0 && (!src || !dst || (weighted && !w))) {
        return MH_EINVAL;
    }
    const int32_t T = plan ? plan->seg_work : kDefaultSegWork;
    if (T < 0 || (plan && (plan->flags != 0 || plan->grid_blocks < 0))) return MH_EINVAL;
    if (!workspace || ws_bytes < sample_workspace_bytes(n, weighted, T)) return MH_EWORKSPACE;

    Arena ar(workspace, ws_bytes);
    Counters* ctr = ar.take<Counters>(1);
    NetBuffers B = carve_network(ar, n, weighted, T);
    if (ar.overflow) return MH_EWORKSPACE;
    const size_t off = (ar.used + 255) & ~size_t(255);
    void* scratch = ar.base + off;
    const size_t scratch_bytes = ws_bytes - off;

    hipEvent_t* ev = plan ? plan->stage_events : nullptr;
    if (ev && ev[0]) MH_HIP_TRY(hipEventRecord(ev[0], stream));
    // the counters are cleared by the order's first kernel (n > 0)
    if (n == 0) return init_counters(ctr, stream);
    static_assert(sizeof(Counters) % sizeof(uint64_t) == 0, "counters clear as u64 words");
    mh_status st = prepare_network(x, y, B, &ctr->status, scratch, scratch_bytes, stream, ev,
                                   ZeroRange{reinterpret_cast<uint64_t*>(ctr), (int64_t)(sizeof(Counters) / 8)});
    if (st != MH_OK) return st;
    if (ev && ev[2]) MH_HIP_TRY(hipEventRecord(ev[2], stream));

    SweepLaunch A{};
    A.net = net_desc(B);
    A.replica = replica;
    A.key0 = (uint32_t)seed;
    A.key1 = (uint32_t)(seed >> 32);
    A.out = EdgeOut{src, dst, w, rank_cnt ? 0 : capacity, &ctr->n_edges};
    A.sid = nullptr;
    A.rank_cnt = rank_cnt;
    A.ctr = ctr;
    const int32_t gb = plan ? plan->grid_blocks : 0;
    if (rank_cnt) {
        // statistics always: the edge count is the number of accepts
        const int64_t zb = (n + kThreads - 1) / kThreads;
        hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)(zb < 1024 ? zb : 1024)), dim3(kThreads), 0, stream, rank_cnt,
                           n);
        MH_HIP_TRY(hipGetLastError());
        if (chung_lu) launch_sweep<false, true, false, OUT_RANKS, true>(A, n, gb, stream);
        else launch_sweep<false, true, false, OUT_RANKS, false>(A, n, gb, stream);
    } else if (chung_lu) {
        if (stats) launch_sweep<false, true, false, OUT_EDGES, true>(A, n, gb, stream);
        else launch_sweep<false, false, false, OUT_EDGES, true>(A, n, gb, stream);
    } else if (weighted) {
        if (stats) launch_sweep<true, true>(A, n, gb, stream);
        else launch_sweep<true, false>(A, n, gb, stream);
    } else {
        if (stats) launch_sweep<false, true>(A, n, gb, stream);
        else launch_sweep<false, false>(A, n, gb, stream);
    }
    MH_HIP_TRY(hipGetLastError());
    if (ev && ev[3]) MH_HIP_TRY(hipEventRecord(ev[3], stream));
    return MH_OK;
}

mh_status sample_impl(const double* x, const double* y, int64_t n, uint64_t seed, uint32_t replica,
                      const mh_plan_params* plan, int32_t* src, int32_t* dst, int32_t* w, int64_t capacity,
                      int64_t* n_edges_host, void* workspace, size_t ws_bytes, mh_stats* stats_host,
                      hipStream_t stream, bool chung_lu = false) {
    if (!n_edges_host) return MH_EINVAL;
    *n_edges_host = 0;
    if (stats_host) *stats_host = mh_stats{0, 0, 0, 0, 0, 0};
    if (n == 0) return (n >= 0 && capacity >= 0) ? MH_OK : MH_EINVAL;
    mh_status st = enqueue_sample(x, y, n, seed, replica, plan, src, dst, w, capacity, workspace, ws_bytes,
                                  stats_host != nullptr, stream, chung_lu);
    if (st != MH_OK) return st;
    return read_counters(static_cast<const Counters*>(workspace), capacity, n_edges_host, stats_host, stream);
}

// Counts by rank of one unweighted sample (UBCM or Chung-Lu): the edge count is
// the statistics' accepts.
mh_status rank_counts_impl(const double* x, int64_t n, bool chung_lu, uint64_t seed, uint32_t replica,
                           const mh_plan_params* plan, int32_t* rank_cnt, int64_t* n_edges_host, void* workspace,
                           size_t ws_bytes, mh_stats* stats_host, hipStream_t stream) {
    if (!n_edges_host) return MH_EINVAL;
    *n_edges_host = 0;
    if (stats_host) *stats_host = mh_stats{0, 0, 0, 0, 0, 0};
    if (n < 0) return MH_EINVAL;
    if (n == 0) return MH_OK;
    if (!rank_cnt) return MH_EINVAL;
    mh_status st = enqueue_sample(x, nullptr, n, seed, replica, plan, nullptr, nullptr, nullptr, 0, workspace,
                                  ws_bytes, true, stream, chung_lu, rank_cnt);
    if (st != MH_OK) return st;
    mh_stats sh;
    int64_t unused = 0;
    st = read_counters(static_cast<const Counters*>(workspace), INT64_MAX, &unused, &sh, stream);
    if (st != MH_OK) return st;
    *n_edges_host = sh.accepts;
    if (stats_host) {
        *stats_host = sh;
        stats_host->n_edges = sh.accepts;
    }
    return MH_OK;
}

// ---- the allocation-free sampler's scratch ----
// Device memory of the library itself for callers that cannot allocate: one
// copy per GPU, held from the library's load on that GPU until the process
// ends.  Host code never passes `scratch` itself to a kernel (in host code
// the name stands for a host-side shadow): it takes each device's address of
// the array once, with that device current, and uses that address.
__device__ __align__(256) unsigned char scratch[MH_NOALLOC_SCRATCH_BYTES];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kScratchDevices];  // the array's address on each device, once taken

mh_status device_scratch(void** out) {
    int dev = -1;
    MH_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices) return MH_EHIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return MH_EHIP;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return MH_OK;
}

}  // namespace

// ---- plan counts entry (also used by the C-ABI) ----
size_t plan_workspace_bytes_impl(int64_t n) {
    Sizer s;
    s.take<NodeRec>(n);
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
    NodeRec* node = ar.take<NodeRec>(n);
    uint64_t* P = ar.take<uint64_t>(n + 1);
    int32_t* jend = ar.take<int32_t>(n);
    uint64_t* mq = ar.take<uint64_t>(n);
    if (ar.overflow) return MH_EWORKSPACE;
    const size_t off = (ar.used + 255) & ~size_t(255);
    const unsigned grid = (unsigned)((n + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_pack_sorted, dim3(grid), dim3(kThreads), 0, stream, zs, n, node, T > 0 ? P : nullptr);
    MH_HIP_TRY(hipGetLastError());
    if (T > 0) {
        mh_status st = scan_exclusive_u64(P, P, n, ar.base + off, ws_bytes - off, stream);
        if (st != MH_OK) return st;
    }
    mh_status pst = launch_row_plan(node, c, n, node, nullptr, n, 0, T, P, jend, mq, nullptr, stream);
    if (pst != MH_OK) return pst;
    hipLaunchKernelGGL(k_unpack_nseg, dim3(grid), dim3(kThreads), 0, stream, node, n, nseg);
    MH_HIP_TRY(hipGetLastError());
    return MH_OK;
}

// ---- two node sets: bipartite and directed networks (Sec. 2.6) ----
namespace {

// Largest column y, as the bit pattern of a non-negative double (which orders
// like the value), reduced with one atomic max per wave into *bits.
__global__ __launch_bounds__(kThreads) void k_max_bits(const double* __restrict__ v, int64_t n,
                                                       unsigned long long* __restrict__ bits) {
    unsigned long long m = 0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const double x = v[i];
        const unsigned long long b = (x > 0.0) ? (unsigned long long)__double_as_longlong(x) : 0ull;
        m = b > m ? b : m;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off, kWave);
        m = o > m ? o : m;
    }
    if ((threadIdx.x & 63) == 0 && m) atomicMax(bits, m);
}

__global__ void k_zero_bits(unsigned long long* bits) {
    if (threadIdx.x == 0) *bits = 0;
}

// Row bound c_r = 1 - y_r * max_j y_j (the smallest beta+_r + beta-_j row r can
// meet), and the checks of the two sets together: the largest t (product of
// the two largest z) is finite and every y_r y_j < 1.
__global__ __launch_bounds__(kThreads) void k_bip_bound(const NodeRec* __restrict__ rows,
                                                        const NodeRec* __restrict__ cols,
                                                        const double* __restrict__ ys, int64_t nr,
                                                        const unsigned long long* __restrict__ ymax_bits,
                                                        double* __restrict__ c, int32_t* status) {
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r == 0 && !isfinite(rows[0].z * cols[0].z)) raise_status(status, MH_EINVAL);
    if (!c || r >= nr) return;
    const double ym = __longlong_as_double((long long)*ymax_bits);
    const double Y = ys[r] * ym;
    c[r] = 1.0 - Y;
    if (!(Y < 1.0)) raise_status(status, MH_EINVAL);
}

// Device buffers of a prepared bipartite network.
struct BipBuffers {
    NodeRec* rows;
    double* ysr;
    double* c;
    int32_t* jend;
    uint64_t* mq;
    uint64_t* hoff;
    HeavyRec* rec;
    int64_t rec_cap;
    NodeRec* cols;
    double* ysc;
    uint64_t* P;
    unsigned long long* ymax;
    uint64_t* scan_state;  // look-back state: P scan over the columns, then hoff over the rows
    int64_t scan_words;
    uint64_t* Psamp;  // P[256 k] over the columns
    double* Zsamp;    // z[256 k] over the columns
    int32_t* hbrow;   // first row of every round of heavy items over the rows
};

template <typename A>
BipBuffers carve_bipartite(A& ar, int64_t nr, int64_t nc, bool weighted, int32_t T) {
    const bool seg = T > 0;
    BipBuffers B{};
    B.rows = ar.template take<NodeRec>(nr);
    B.ysr = ar.template take<double>(weighted ? nr : 0);
    B.c = ar.template take<double>(weighted ? nr : 0);
    B.jend = ar.template take<int32_t>(seg ? nr : 0);
    B.mq = ar.template take<uint64_t>(seg ? nr : 0);
    B.hoff = ar.template take<uint64_t>(seg ? nr + 1 : 0);
    B.rec_cap = seg ? kRecPerRow * nr + 4096 : 0;
    B.cols = ar.template take<NodeRec>(nc);
    B.ysc = ar.template take<double>(weighted ? nc : 0);
    B.P = ar.template take<uint64_t>(seg ? nc + 1 : 0);
    B.ymax = ar.template take<unsigned long long>(1);
    B.scan_words = seg ? lb_tiles(nc) + lb_tiles(nr) : 0;
    B.scan_state = ar.template take<uint64_t>(B.scan_words);
    B.Psamp = ar.template take<uint64_t>(seg ? lb_samples(nc) : 0);
    B.Zsamp = ar.template take<double>(seg ? lb_samples(nc) : 0);
    B.hbrow = ar.template take<int32_t>(seg ? B.rec_cap / kHrThreads + 2 : 0);
    B.rec = ar.template take<HeavyRec>(B.rec_cap);  // last: the large, mostly unused reserve
    if (!weighted) B.ysr = B.c = B.ysc = nullptr;
    if (!seg)
        B.jend = nullptr, B.mq = nullptr, B.hoff = nullptr, B.P = nullptr, B.scan_state = nullptr, B.Psamp = nullptr,
        B.Zsamp = nullptr, B.hbrow = nullptr;
    return B;
}

size_t bipartite_workspace_bytes(int64_t nr, int64_t nc, bool weighted, int32_t T) {
    if (nr < 0 || nc < 0) return 0;
    SizerAdapter sz;
    sz.s.take<Counters>(1);
    carve_bipartite(sz, nr, nc, weighted, T);
    size_t scratch = prepare_scratch_bytes(nr);
    const size_t s2 = prepare_scratch_bytes(nc);
    if (s2 > scratch) scratch = s2;
    return sz.s.used + scratch + 768;
}

NetDesc bip_desc(const BipBuffers& B, int64_t nr, int64_t nc, int32_t T, uint32_t flags) {
    NetDesc D;
    D.node = B.rows;
    D.ys = B.ysr;
    D.c = B.c;
    D.col = B.cols;
    D.ysc = B.ysc;
    D.jend = B.jend;
    D.mq = B.mq;
    D.P = B.P;
    D.hoff = B.hoff;
    D.rec = B.rec;
    D.rec_cap = B.rec_cap;
    D.n = nr;
    D.ncol = nc;
    D.T = T;
    D.flags = NET_BIPARTITE | ((flags & MH_BIP_NO_SELF) ? NET_NO_SELF : 0);
    return D;
}

mh_status sample_bipartite_impl(const double* xr, const double* yr, int64_t nr, const double* xc, const double* yc,
                                int64_t nc, uint32_t flags, uint64_t seed, uint32_t replica,
                                const mh_plan_params* plan, int32_t* src, int32_t* dst, int32_t* w,
                                int64_t capacity, int64_t* n_edges_host, void* workspace, size_t ws_bytes,
                                mh_stats* stats_host, hipStream_t stream) {
    const bool weighted = (yr != nullptr);
    if (!n_edges_host || nr < 0 || nc < 0 || nr > 0x7FFFFFFFll || nc > 0x7FFFFFFFll || capacity < 0)
        return MH_EINVAL;
    if ((yr == nullptr) != (yc == nullptr) || (flags & ~MH_BIP_NO_SELF) != 0) return MH_EINVAL;
    if ((!xr && nr > 0) || (!xc && nc > 0)) return MH_EINVAL;
    if (capacity > 0 && (!src || !dst || (weighted && !w))) return MH_EINVAL;
    const int32_t T = plan ? plan->seg_work : kDefaultSegWork;
    if (T < 0 || (plan && (plan->flags != 0 || plan->grid_blocks < 0))) return MH_EINVAL;
    *n_edges_host = 0;
    if (stats_host) *stats_host = mh_stats{0, 0, 0, 0, 0, 0};
    if (nr == 0 || nc == 0) return MH_OK;
    if (!workspace || ws_bytes < bipartite_workspace_bytes(nr, nc, weighted, T)) return MH_EWORKSPACE;

    Arena ar(workspace, ws_bytes);
    Counters* ctr = ar.take<Counters>(1);
    BipBuffers B = carve_bipartite(ar, nr, nc, weighted, T);
    if (ar.overflow) return MH_EWORKSPACE;
    const size_t off = (ar.used + 255) & ~size_t(255);
    void* scratch = ar.base + off;
    const size_t scratch_bytes = ws_bytes - off;
    int32_t* status = &ctr->status;
    const bool seg = T > 0;

    hipEvent_t* ev = plan ? plan->stage_events : nullptr;
    if (ev && ev[0]) MH_HIP_TRY(hipEventRecord(ev[0], stream));
    mh_status st = init_counters(ctr, stream);
    if (st != MH_OK) return st;
    // A1: each set sorted by its own z; the column masses for the plan
    // (the rows' first kernel zeroes the look-back state of both plan scans)
    st = order_nodes(xr, yr, nr, nullptr, nullptr, B.ysr, B.rows, status, nullptr, nullptr, nullptr, nullptr, scratch,
                     scratch_bytes, stream, false, ZeroRange{B.scan_state, B.scan_words});
    if (st != MH_OK) return st;
    st = order_nodes(xc, yc, nc, nullptr, nullptr, B.ysc, B.cols, status, B.P, B.scan_state, B.Psamp, B.Zsamp, scratch,
                     scratch_bytes, stream, false);
    if (st != MH_OK) return st;
    if (ev && ev[1]) MH_HIP_TRY(hipEventRecord(ev[1], stream));
    // A2: row bounds and the joint checks
    if (weighted) {
        hipLaunchKernelGGL(k_zero_bits, dim3(1), dim3(64), 0, stream, B.ymax);
        MH_HIP_TRY(hipGetLastError());
        int64_t g = (nc + kThreads - 1) / kThreads;
        if (g > 1024) g = 1024;
        hipLaunchKernelGGL(k_max_bits, dim3((unsigned)g), dim3(kThreads), 0, stream, (const double*)B.ysc, nc,
                           B.ymax);
        MH_HIP_TRY(hipGetLastError());
    }
    const unsigned rows_grid = (unsigned)((nr + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_bip_bound, dim3(weighted ? rows_grid : 1u), dim3(kThreads), 0, stream,
                       (const NodeRec*)B.rows, (const NodeRec*)B.cols, (const double*)B.ysr, nr,
                       (const unsigned long long*)B.ymax, B.c, status);
    MH_HIP_TRY(hipGetLastError());
    // A3: plan over the columns
    bool rows_known = false;
    st = plan_rows(B.rows, B.c, nr, B.cols, B.Zsamp, nc, 1, T, B.P, B.jend, B.mq, B.hoff,
                   seg ? B.scan_state + lb_tiles(nc) : nullptr, B.hbrow, B.rec_cap, status, scratch,
                   scratch_bytes, &rows_known, stream);
    if (st != MH_OK) return st;
    const NetDesc D = bip_desc(B, nr, nc, T, flags);
    if (seg) {
        const bool samples = nc <= (int64_t)1 << 30;  // P's samples: the columns' one-pass scan
        hipLaunchKernelGGL(k_heavy_records, dim3(heavy_grid(B.rec_cap)), dim3(kHrThreads), 0, stream, D, B.rec,
                           (const uint64_t*)(samples ? B.Psamp : nullptr),
                           (const int32_t*)(rows_known ? B.hbrow : nullptr), (const int32_t*)status);
        MH_HIP_TRY(hipGetLastError());
    }
    if (ev && ev[2]) MH_HIP_TRY(hipEventRecord(ev[2], stream));

    SweepLaunch A{};
    A.net = D;
    A.replica = replica;
    A.key0 = (uint32_t)seed;
    A.key1 = (uint32_t)(seed >> 32);
    A.out = EdgeOut{src, dst, w, capacity, &ctr->n_edges};
    A.sid = nullptr;
    A.ctr = ctr;
    const int32_t gb = plan ? plan->grid_blocks : 0;
    if (weighted) {
        if (stats_host) launch_sweep<true, true, true>(A, nr, gb, stream);
        else launch_sweep<true, false, true>(A, nr, gb, stream);
    } else {
        if (stats_host) launch_sweep<false, true, true>(A, nr, gb, stream);
        else launch_sweep<false, false, true>(A, nr, gb, stream);
    }
    MH_HIP_TRY(hipGetLastError());
    if (ev && ev[3]) MH_HIP_TRY(hipEventRecord(ev[3], stream));

    Counters hc;
    MH_HIP_TRY(hipMemcpyAsync(&hc, ctr, sizeof(Counters), hipMemcpyDeviceToHost, stream));
    MH_HIP_TRY(hipStreamSynchronize(stream));
    if (hc.status != 0) return (mh_status)hc.status;
    *n_edges_host = (int64_t)hc.n_edges;
    if (stats_host) {
        stats_host->steps = (int64_t)hc.stats[ST_STEPS].v;
        stats_host->proposals = (int64_t)hc.stats[ST_PROPOSALS].v;
        stats_host->accepts = (int64_t)hc.stats[ST_ACCEPTS].v;
        stats_host->segments = (int64_t)hc.stats[ST_SEGMENTS].v;
        stats_host->saturated_w = (int64_t)hc.stats[ST_SATURATED].v;
        stats_host->n_edges = (int64_t)hc.n_edges;
    }
    if ((int64_t)hc.n_edges > capacity) return MH_ECAPACITY;
    return MH_OK;
}

}  // namespace

}  // namespace mh

extern "C" {

size_t mh_workspace_bytes(int64_t n, int weighted, const mh_plan_params* plan) {
    return mh::sample_workspace_bytes(n, weighted != 0, plan ? plan->seg_work : mh::kDefaultSegWork);
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

mh_status mh_sample_chung_lu(const double* w, int64_t n, uint64_t seed, uint32_t replica, const mh_plan_params* plan,
                             int32_t* src, int32_t* dst, int64_t capacity, int64_t* n_edges_host, void* workspace,
                             size_t ws_bytes, mh_stats* stats_host, hipStream_t stream) {
    return mh::sample_impl(w, nullptr, n, seed, replica, plan, src, dst, nullptr, capacity, n_edges_host, workspace,
                           ws_bytes, stats_host, stream, true);
}

mh_status mh_sample_rank_counts(const double* x, int64_t n, int32_t model, uint64_t seed, uint32_t replica,
                                const mh_plan_params* plan, int32_t* rank_counts, int64_t* n_edges_host,
                                void* workspace, size_t ws_bytes, mh_stats* stats_host, hipStream_t stream) {
    if (model != MH_MODEL_UBCM && model != MH_MODEL_CHUNG_LU) return MH_EINVAL;
    return mh::rank_counts_impl(x, n, model == MH_MODEL_CHUNG_LU, seed, replica, plan, rank_counts, n_edges_host,
                                workspace, ws_bytes, stats_host, stream);
}

mh_status mh_sample_unweighted_noalloc(const double* x, int64_t n, uint64_t seed, uint32_t replica,
                                       const mh_plan_params* plan, int32_t* src, int32_t* dst, int64_t capacity,
                                       int64_t* n_edges_host, mh_stats* stats_host, hipStream_t stream) {
    if (!n_edges_host) return MH_EINVAL;
    *n_edges_host = 0;
    if (stats_host) *stats_host = mh_stats{0, 0, 0, 0, 0, 0};
    if (n < 0 || n > MH_NOALLOC_MAX_NODES) return MH_EINVAL;
    const int32_t T = plan ? plan->seg_work : mh::kDefaultSegWork;
    if (T < 0 || mh::sample_workspace_bytes(n, false, T) > (size_t)MH_NOALLOC_SCRATCH_BYTES) return MH_EWORKSPACE;
    void* ws = nullptr;
    const mh_status st = mh::device_scratch(&ws);
    if (st != MH_OK) return st;
    return mh::sample_impl(x, nullptr, n, seed, replica, plan, src, dst, nullptr, capacity, n_edges_host, ws,
                           (size_t)MH_NOALLOC_SCRATCH_BYTES, stats_host, stream);
}

mh_status mh_sample_unweighted_async(const double* x, int64_t n, uint64_t seed, uint32_t replica,
                                     const mh_plan_params* plan, int32_t* src, int32_t* dst, int64_t capacity,
                                     void* workspace, size_t ws_bytes, hipStream_t stream) {
    return mh::enqueue_sample(x, nullptr, n, seed, replica, plan, src, dst, nullptr, capacity, workspace, ws_bytes,
                              false, stream);
}

mh_status mh_sample_weighted_async(const double* x, const double* y, int64_t n, uint64_t seed, uint32_t replica,
                                   const mh_plan_params* plan, int32_t* src, int32_t* dst, int32_t* w,
                                   int64_t capacity, void* workspace, size_t ws_bytes, hipStream_t stream) {
    if (!y && n > 0) return MH_EINVAL;
    return mh::enqueue_sample(x, y, n, seed, replica, plan, src, dst, w, capacity, workspace, ws_bytes, false,
                              stream);
}

mh_status mh_sample_result(const void* workspace, size_t ws_bytes, int64_t capacity, int64_t* n_edges_host,
                           hipStream_t stream) {
    if (!n_edges_host || capacity < 0) return MH_EINVAL;
    *n_edges_host = 0;
    if (!workspace || ws_bytes < sizeof(mh::Counters)) return MH_EWORKSPACE;
    return mh::read_counters(static_cast<const mh::Counters*>(workspace), capacity, n_edges_host, nullptr, stream);
}

size_t mh_plan_workspace_bytes(int64_t n) { return mh::plan_workspace_bytes_impl(n); }

mh_status mh_plan_counts(const double* zs, const double* c, int64_t n, int32_t seg_work, int32_t* nseg,
                         void* workspace, size_t ws_bytes, hipStream_t stream) {
    return mh::plan_counts_impl(zs, c, n, seg_work, nseg, workspace, ws_bytes, stream);
}

}  // extern "C"

extern "C" {

size_t mh_bipartite_workspace_bytes(int64_t n_rows, int64_t n_cols, int weighted, const mh_plan_params* plan) {
    return mh::bipartite_workspace_bytes(n_rows, n_cols, weighted != 0,
                                         plan ? plan->seg_work : mh::kDefaultSegWork);
}

mh_status mh_sample_bipartite(const double* x_rows, const double* y_rows, int64_t n_rows, const double* x_cols,
                              const double* y_cols, int64_t n_cols, uint32_t flags, uint64_t seed, uint32_t replica,
                              const mh_plan_params* plan, int32_t* src, int32_t* dst, int32_t* w, int64_t capacity,
                              int64_t* n_edges_host, void* workspace, size_t ws_bytes, mh_stats* stats_host,
                              hipStream_t stream) {
    return mh::sample_bipartite_impl(x_rows, y_rows, n_rows, x_cols, y_cols, n_cols, flags, seed, replica, plan,
                                     src, dst, w, capacity, n_edges_host, workspace, ws_bytes, stats_host, stream);
}

}  // extern "C"

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

// The item table: item_tab[c] = the sample holding item c 2^shift, with the
// least shift that keeps ceil(items / 2^shift) within kItemTab entries (one
// thread per entry, a search among the samples each).
constexpr int64_t kItemTab = int64_t(1) << 18;
__global__ __launch_bounds__(kThreads) void k_batch_item_table(const uint64_t* __restrict__ item_off,
                                                               int32_t n_samples, int32_t* __restrict__ tab,
                                                               int32_t* __restrict__ shift_out) {
    const uint64_t total = item_off[n_samples];
    int32_t sh = 0;
    while ((total + (uint64_t(1) << sh) - 1) >> sh > (uint64_t)kItemTab) ++sh;
    const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (c == 0) *shift_out = sh;
    if ((uint64_t)c >= (total + (uint64_t(1) << sh) - 1) >> sh) return;
    const uint64_t it = (uint64_t)c << sh;
    int32_t lo = 0, hi = n_samples;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (item_off[mid] <= it) lo = mid; else hi = mid;
    }
    tab[c] = lo;
}

// ---- batched edge output: filling the chunks' unused tails ----
// Each wave of the sweep reserved output slots kOutChunk at a time; every
// chunk but a wave's last is full.  With G slots reserved and T unused in the
// waves' last chunks, the list has n = G - T edges; the unused slots below n
// (holes) take the edges found at n and beyond, so the list ends up in
// [0, n).  The order of a batch's edges is unspecified, so any one-to-one
// matching of holes and those edges does.
constexpr int kMaxChunkWaves = 4096;  // waves of a launch with edge output (grid capped to match)
constexpr int kGapThreads = 1024;
constexpr int kGapPer = (kMaxChunkWaves + 2 + kGapThreads - 1) / kGapThreads;

struct GapLists {
    uint64_t* hole_pos;  // [kMaxChunkWaves]: first hole slot of wave w's last chunk below n
    uint64_t* hole_off;  // [kMaxChunkWaves]: exclusive prefix of the holes' lengths
    uint64_t* src_pos;   // [kMaxChunkWaves + 2]: first edge at or beyond n of chunk c0 + i
    uint64_t* src_off;   // [kMaxChunkWaves + 2]: exclusive prefix of those edge counts
    uint64_t* meta;      // [4]: holes H, waves W, chunks m
};

// Block-wide exclusive scan of v[0..count) (count <= kGapThreads * kGapPer),
// each thread taking a run of kGapPer entries; returns the total.
__device__ uint64_t gap_scan(const uint64_t* v, uint64_t* out, int count, uint64_t* s_part) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int b = t * kGapPer;
    uint64_t run = 0;
    for (int i = 0; i < kGapPer; ++i)
        if (b + i < count) run += v[b + i];
    uint64_t inc = run;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint64_t u = __shfl_up(inc, off, kWave);
        if (lane >= off) inc += u;
    }
    if (lane == 63) s_part[wave] = inc;
    __syncthreads();
    if (t == 0) {
        uint64_t acc = 0;
        for (int w = 0; w < kGapThreads / kWave; ++w) {
            const uint64_t x = s_part[w];
            s_part[w] = acc;
            acc += x;
        }
        s_part[kGapThreads / kWave] = acc;
    }
    __syncthreads();
    uint64_t pre = s_part[wave] + inc - run;
    for (int i = 0; i < kGapPer; ++i)
        if (b + i < count) {
            out[b + i] = pre;
            pre += v[b + i];
        }
    const uint64_t total = s_part[kGapThreads / kWave];
    __syncthreads();
    return total;
}

// One block: n, the holes below n and the edges at or beyond n, as lists with
// prefixes; the call's edge count becomes n.  Reserved slots beyond the
// capacity were not written: then the count reported is n plus a chunk per
// wave, a capacity that suffices, and nothing moves.
__global__ __launch_bounds__(kGapThreads) void k_gap_plan(Counters* ctr, const unsigned long long* __restrict__ rec,
                                                         int32_t W, int64_t capacity, GapLists g) {
    __shared__ uint64_t s_v[kGapThreads * kGapPer];
    __shared__ uint32_t s_len[kGapThreads * kGapPer];
    __shared__ uint64_t s_part[kGapThreads / kWave + 1];
    __shared__ uint64_t s_sum[kGapThreads / kWave];
    const int t = threadIdx.x;
    if (ctr->status != 0) {
        if (t == 0) g.meta[0] = 0;
        return;
    }
    const uint64_t G = ctr->n_edges;
    const uint64_t C = kOutChunk;
    uint64_t tail = 0;
    for (int w = t; w < W; w += kGapThreads)
        if (rec[2 * w] != ~0ull) tail += C - rec[2 * w + 1];
    tail = wave_sum(tail);
    if ((t & 63) == 0) s_sum[t >> 6] = tail;
    __syncthreads();
    uint64_t T = 0;
    for (int w = 0; w < kGapThreads / kWave; ++w) T += s_sum[w];
    const uint64_t n = G - T;
    if (G > (uint64_t)capacity) {
        if (t == 0) {
            g.meta[0] = 0;
            ctr->n_edges = n + (uint64_t)W * C;
        }
        return;
    }
    // holes below n, one per wave's last chunk
    for (int w = t; w < kGapThreads * kGapPer; w += kGapThreads) {
        uint64_t h = 0, pos = 0;
        if (w < W && rec[2 * w] != ~0ull) {
            pos = rec[2 * w] + rec[2 * w + 1];
            const uint64_t end = rec[2 * w] + C < n ? rec[2 * w] + C : n;
            h = pos < end ? end - pos : 0;
        }
        s_v[w] = h;
        if (w < W) g.hole_pos[w] = pos;
    }
    __syncthreads();
    const uint64_t H = gap_scan(s_v, g.hole_off, W, s_part);
    // edges at or beyond n: chunks c0 .. c1 - 1, full but for the waves' last ones
    const uint64_t c0 = n / C, c1 = G / C;
    const int m = (int)(c1 - c0);
    for (int i = t; i < kGapThreads * kGapPer; i += kGapThreads) s_len[i] = (uint32_t)C;
    __syncthreads();
    for (int w = t; w < W; w += kGapThreads) {
        const uint64_t st = rec[2 * w];
        if (st != ~0ull && st / C >= c0 && st / C < c1) s_len[st / C - c0] = (uint32_t)rec[2 * w + 1];
    }
    __syncthreads();
    for (int i = t; i < kGapThreads * kGapPer; i += kGapThreads) {
        uint64_t len = 0, lo = 0;
        if (i < m) {
            const uint64_t start = (c0 + (uint64_t)i) * C;
            lo = start > n ? start : n;
            const uint64_t e = start + s_len[i];
            len = e > lo ? e - lo : 0;
            g.src_pos[i] = lo;
        }
        s_v[i] = len;
    }
    __syncthreads();
    const uint64_t S = gap_scan(s_v, g.src_off, m, s_part);
    if (t == 0) {
        if (S != H) raise_status(&ctr->status, MH_EHIP);  // the two counts always agree
        g.meta[0] = S == H ? H : 0;
        g.meta[1] = (uint64_t)W;
        g.meta[2] = (uint64_t)m;
        ctr->n_edges = n;
    }
}

// The moves: the k-th hole slot takes the k-th edge at or beyond n.
__global__ __launch_bounds__(kThreads) void k_gap_move(GapLists g, int32_t* __restrict__ src, int32_t* __restrict__ dst,
                                                      int32_t* __restrict__ w, int32_t* __restrict__ sid) {
    const uint64_t H = g.meta[0];
    const int32_t W = (int32_t)g.meta[1], m = (int32_t)g.meta[2];
    for (uint64_t k = (uint64_t)blockIdx.x * kThreads + threadIdx.x; k < H; k += (uint64_t)gridDim.x * kThreads) {
        int32_t lo = 0, hi = W;
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (g.hole_off[mid] <= k) lo = mid; else hi = mid;
        }
        const uint64_t p = g.hole_pos[lo] + (k - g.hole_off[lo]);
        int32_t a = 0, b = m;
        while (b - a > 1) {
            const int32_t mid = (a + b) >> 1;
            if (g.src_off[mid] <= k) a = mid; else b = mid;
        }
        const uint64_t q = g.src_pos[a] + (k - g.src_off[a]);
        src[p] = src[q];
        dst[p] = dst[q];
        if (w) w[p] = w[q];
        if (sid) sid[p] = sid[q];
    }
}

// ---- staged degree counts (MH_BATCH_DEGREES_STAGED) ----
// The sweep writes each accepted column's node id into the slot region of its
// key (sample, window of 2^15 ids); one counting block per key then adds the
// region up in LDS.  A region is sized from a bound on the expected column
// hits of its window's nodes; what does not fit is added by atomics.
constexpr int64_t kWinCols = int64_t(1) << kSlotWinShift;

__host__ __device__ inline int64_t windows_of(int64_t n) { return (n + kWinCols - 1) / kWinCols; }

// Per network and window: the sum over the window's nodes of a bound on the
// node's expected hits as a column.  Column rank j is proposed by the rows of
// smaller rank at most once each and, from row r, with probability at most
// z_r z_j (the skip's rate), so its hits are at most min(j, z_j Z_j), Z_j the
// mass of the ranks before j (P[j]).  The weighted chain proposes with its
// row bound as well, so there the bound is looser than the truth can be:
// its regions overflow into atomics sooner.  Without a plan (no column
// masses) the bound is 0.  Grid (chunks, networks); est zeroed beforehand.
constexpr int kEstThreads = 1024;
__global__ __launch_bounds__(kEstThreads) void k_net_estimate(const NetDesc* __restrict__ nets, int32_t n_networks,
                                                              const uint64_t* __restrict__ net_win_off,
                                                              double* __restrict__ est) {
    __shared__ double s_w[kSlotBins];
    for (int32_t k = blockIdx.y; k < n_networks; k += gridDim.y) {
        const NetDesc D = nets[k];
        const int64_t nwin = windows_of(D.n);
        __syncthreads();
        for (int i = threadIdx.x; i < kSlotBins; i += kEstThreads) s_w[i] = 0.0;
        __syncthreads();
        if (D.P && nwin <= kSlotBins) {
            for (int64_t j = (int64_t)blockIdx.x * kEstThreads + threadIdx.x; j < D.n;
                 j += (int64_t)gridDim.x * kEstThreads) {
                const NodeRec rec = D.node[j];
                const double mass = (double)D.P[j] * 0x1.0p-32 * rec.z;
                atomicAdd(&s_w[rec.id >> kSlotWinShift], mass < (double)j ? mass : (double)j);
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nwin && i < kSlotBins; i += kEstThreads)
            if (s_w[i] > 0.0) atomicAdd(&est[net_win_off[k] + i], s_w[i]);
    }
}

__global__ void k_fill_f64(double* a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0.0;
}

// Per sample: its count of windows (0 for a bad network index: the call fails).
__global__ __launch_bounds__(kThreads) void k_batch_wins(const NetDesc* __restrict__ nets, int32_t n_networks,
                                                         const int32_t* __restrict__ sample_net, int32_t n_samples,
                                                         uint64_t* __restrict__ wins) {
    const int32_t s = blockIdx.x * kThreads + threadIdx.x;
    if (s >= n_samples) return;
    const int32_t k = sample_net[s];
    wins[s] = (k >= 0 && k < n_networks) ? (uint64_t)windows_of(nets[k].n) : 0;
}

// Sample of key g: the last s with win_off[s] <= g (samples without windows
// share their successor's offset and are skipped).
__device__ __forceinline__ int32_t key_sample(const uint64_t* __restrict__ win_off, int32_t n_samples, uint64_t g) {
    int32_t lo = 0, hi = n_samples;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (win_off[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// Per key (grid: n_keys upper bound): its region's size (1.25 times its
// window's bound, plus 512) and an empty cursor; keys past the last are empty.
__global__ __launch_bounds__(kThreads) void k_batch_regions(const int32_t* __restrict__ sample_net, int32_t n_samples,
                                                            const uint64_t* __restrict__ win_off,
                                                            const uint64_t* __restrict__ net_win_off,
                                                            const double* __restrict__ est, int64_t n_keys,
                                                            uint64_t* __restrict__ cap,
                                                            unsigned long long* __restrict__ cursor) {
    const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (g >= n_keys) return;
    cursor[g * kCursorStride] = 0;
    if ((uint64_t)g >= win_off[n_samples]) {
        cap[g] = 0;
        return;
    }
    const int32_t s = key_sample(win_off, n_samples, (uint64_t)g);
    const double e = est[net_win_off[sample_net[s]] + ((uint64_t)g - win_off[s])];
    cap[g] = (uint64_t)(1.25 * e) + 512;
}

// Regions end at the slot capacity: a region reaching past it is cut.
__global__ __launch_bounds__(kThreads) void k_batch_clip(int64_t n_keys, const uint64_t* __restrict__ off,
                                                         uint64_t* __restrict__ cap, int64_t capacity) {
    const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (g >= n_keys) return;
    const uint64_t room = off[g] < (uint64_t)capacity ? (uint64_t)capacity - off[g] : 0;
    if (cap[g] > room) cap[g] = room;
}

// One block per key: counts its region's node ids in LDS and adds the counts
// to its sample's degrees (the window's ids belong to this block alone).  The
// region is read once, 8 values a thread in flight.
constexpr int kCountThreads = 1024;
constexpr int kCountPer = 8;
__global__ __launch_bounds__(kCountThreads) void k_batch_count(const NetDesc* __restrict__ nets,
                                                               const int32_t* __restrict__ sample_net, int32_t n_samples,
                                                               const uint64_t* __restrict__ win_off,
                                                               const uint64_t* __restrict__ region_off,
                                                               const uint64_t* __restrict__ region_cap,
                                                               const unsigned long long* __restrict__ cursor,
                                                               const int32_t* __restrict__ slots,
                                                               int32_t* __restrict__ degrees,
                                                               const int64_t* __restrict__ deg_off,
                                                               const int32_t* status) {
    __shared__ uint32_t s_cnt[kWinCols];
    if (*status != 0) return;
    const uint64_t g = blockIdx.x;
    if (g >= win_off[n_samples]) return;
    const int32_t s = key_sample(win_off, n_samples, g);
    const int64_t w0 = (int64_t)(g - win_off[s]) * kWinCols;
    const int64_t n = nets[sample_net[s]].n;
    const int64_t wn = n - w0 < kWinCols ? n - w0 : kWinCols;
    for (int i = threadIdx.x; i < kWinCols; i += kCountThreads) s_cnt[i] = 0;
    __syncthreads();
    const uint64_t used = cursor[g * kCursorStride];
    const uint64_t taken = used < region_cap[g] ? used : region_cap[g];
    const int32_t* reg = slots + region_off[g];
    for (uint64_t k0 = 0; k0 < taken; k0 += (uint64_t)kCountThreads * kCountPer) {
        int32_t v[kCountPer];
#pragma unroll
        for (int u = 0; u < kCountPer; ++u) {
            const uint64_t k = k0 + (uint64_t)u * kCountThreads + threadIdx.x;
            v[u] = k < taken ? reg[k] : -1;
        }
#pragma unroll
        for (int u = 0; u < kCountPer; ++u) {
            const int64_t c = (int64_t)v[u] - w0;
            if (v[u] >= 0 && c >= 0 && c < wn) atomicAdd(&s_cnt[c], 1u);
        }
    }
    __syncthreads();
    int32_t* d = degrees + deg_off[s] + w0;
    for (int64_t i = threadIdx.x; i < wn; i += kCountThreads)
        if (s_cnt[i]) d[i] += (int32_t)s_cnt[i];
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
    // staged degree counts (when every network has at most kSlotBins windows)
    int64_t max_win;           // windows of the largest network
    int64_t total_win;         // windows of all networks
    uint64_t* net_win_off;     // per network (+1): its first window's bound
    double* est;               // per network and window: the bound on its column hits
    uint64_t* win_off;         // per sample (+1): its first key
    int32_t* item_tab;         // kItemTab entries: the sample of every 2^item_shift-th item
    int32_t* item_shift;
    unsigned long long* chunk_rec;  // edge output: per wave, its last chunk (start, used)
    GapLists gap;
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
        int64_t tw = 0, mw = 0;
        for (int32_t i = 0; i < n_networks; ++i) {
            tw += windows_of(nets[i].n);
            mw = windows_of(nets[i].n) > mw ? windows_of(nets[i].n) : mw;
        }
        s.take<uint64_t>((size_t)n_networks + 1);
        s.take<double>((size_t)tw);
        s.take<uint64_t>((size_t)max_samples + 1);
        s.take<int32_t>((size_t)kItemTab);
        s.take<int32_t>(1);
        s.take<unsigned long long>(2 * (size_t)kMaxChunkWaves);
        s.take<uint64_t>((size_t)kMaxChunkWaves);
        s.take<uint64_t>((size_t)kMaxChunkWaves);
        s.take<uint64_t>((size_t)kMaxChunkWaves + 2);
        s.take<uint64_t>((size_t)kMaxChunkWaves + 2);
        s.take<uint64_t>(4);
        bytes = s.used;
        for (int32_t i = 0; i < n_networks; ++i) {
            bytes = ((bytes + 255) & ~size_t(255)) + network_bytes(nets[i].n, nets[i].y != nullptr, nets[i].seg_work);
            if (nets[i].n > max_n) max_n = nets[i].n;
        }
        size_t scratch = prepare_scratch_bytes(max_n);
        size_t s2 = scan_workspace_bytes((int64_t)max_samples + 1);
        if (s2 > scratch) scratch = s2;
        // the scan over the keys of a staged call
        if (mw <= kSlotBins) s2 = scan_workspace_bytes((int64_t)max_samples * mw + 1);
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
    L->max_win = 0;
    L->total_win = 0;
    for (int32_t i = 0; i < n_networks; ++i) {
        L->total_win += windows_of(nets[i].n);
        L->max_win = windows_of(nets[i].n) > L->max_win ? windows_of(nets[i].n) : L->max_win;
    }
    L->net_win_off = ar.take<uint64_t>((size_t)n_networks + 1);
    L->est = ar.take<double>((size_t)L->total_win);
    L->win_off = ar.take<uint64_t>((size_t)max_samples + 1);
    L->item_tab = ar.take<int32_t>((size_t)kItemTab);
    L->item_shift = ar.take<int32_t>(1);
    L->chunk_rec = ar.take<unsigned long long>(2 * (size_t)kMaxChunkWaves);
    L->gap.hole_pos = ar.take<uint64_t>((size_t)kMaxChunkWaves);
    L->gap.hole_off = ar.take<uint64_t>((size_t)kMaxChunkWaves);
    L->gap.src_pos = ar.take<uint64_t>((size_t)kMaxChunkWaves + 2);
    L->gap.src_off = ar.take<uint64_t>((size_t)kMaxChunkWaves + 2);
    L->gap.meta = ar.take<uint64_t>(4);
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
mh_status launch_batch(const SweepLaunch& A, int32_t grid_blocks, hipStream_t stream, int64_t* grid_out = nullptr) {
    auto kern = k_sweep<W, false, true, OUT>;
    int64_t cap = resident_blocks(kern, kThreads);
    // edge output keeps one chunk record per wave
    if (OUT == OUT_EDGES && cap > kMaxChunkWaves / kSweepWaves) cap = kMaxChunkWaves / kSweepWaves;
    const int64_t g = (grid_blocks > 0 && grid_blocks < cap) ? grid_blocks : cap;
    hipLaunchKernelGGL(kern, dim3((unsigned)g), dim3(kThreads), 0, stream, A);
    MH_HIP_TRY(hipGetLastError());
    if (grid_out) *grid_out = g;
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
    // the column-hit bounds that size the regions of staged degree counts
    std::vector<uint64_t> wo((size_t)n_networks + 1, 0);
    for (int32_t i = 0; i < n_networks; ++i) wo[i + 1] = wo[i] + (uint64_t)windows_of(nets[i].n);
    MH_HIP_TRY(hipMemcpyAsync(L.net_win_off, wo.data(), sizeof(uint64_t) * wo.size(), hipMemcpyHostToDevice, stream));
    if (L.total_win > 0 && L.max_win <= kSlotBins) {
        hipLaunchKernelGGL(k_fill_f64, dim3(64), dim3(256), 0, stream, L.est, L.total_win);
        MH_HIP_TRY(hipGetLastError());
        int64_t max_n = 0;
        for (int32_t i = 0; i < n_networks; ++i) max_n = nets[i].n > max_n ? nets[i].n : max_n;
        const int64_t gx = (max_n + kEstThreads - 1) / kEstThreads;
        const dim3 eg((unsigned)(gx < 64 ? gx : 64), (unsigned)(n_networks < 4096 ? n_networks : 4096));
        hipLaunchKernelGGL(k_net_estimate, eg, dim3(kEstThreads), 0, stream, L.nets, n_networks, L.net_win_off, L.est);
        MH_HIP_TRY(hipGetLastError());
    }
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
    } else if (mode == MH_BATCH_DEGREES || mode == MH_BATCH_DEGREES_STAGED) {
        if (n_samples > 0 && (!degrees || !deg_off)) return MH_EINVAL;
        if (mode == MH_BATCH_DEGREES_STAGED && (capacity < 0 || (capacity > 0 && !src))) return MH_EINVAL;
    } else {
        return MH_EINVAL;
    }
    bool staged = mode == MH_BATCH_DEGREES_STAGED;
    BatchLayout L;
    if (!layout(nets, n_networks, max_samples, workspace, ws_bytes, &L, nullptr)) return MH_EWORKSPACE;
    // staged counts: the keys' arrays at the front of src (128-byte aligned:
    // cursors, one line each, then sizes and offsets), then the slots; with
    // too little room (or networks of more than kSlotBins windows) every
    // column is added by atomics instead
    int64_t n_keys = 0, slot_cap = 0;
    uint64_t *region_cap = nullptr, *region_off = nullptr;
    unsigned long long* cursor = nullptr;
    int32_t* slot_base = nullptr;
    if (staged) {
        n_keys = L.max_win <= kSlotBins ? (int64_t)n_samples * L.max_win : 0;
        const uintptr_t p0 = reinterpret_cast<uintptr_t>(src);
        const uintptr_t p8 = (p0 + 127) & ~uintptr_t(127);
        const int64_t skip = src ? (int64_t)((p8 - p0) / sizeof(int32_t)) : 0;
        const int64_t words = 2 * ((kCursorStride + 2) * n_keys + 1);
        if (n_keys == 0 || n_keys > 0x7FFFFFFFll || !src || capacity < skip + words) {
            staged = false;
        } else {
            uint64_t* k64 = reinterpret_cast<uint64_t*>(p8);
            cursor = reinterpret_cast<unsigned long long*>(k64);
            region_cap = k64 + kCursorStride * n_keys;
            region_off = region_cap + n_keys;
            slot_base = src + skip + words;
            slot_cap = capacity - skip - words;
        }
    }
    hipLaunchKernelGGL(k_batch_init, dim3(1), dim3(64), 0, stream, L.ctr);
    MH_HIP_TRY(hipGetLastError());
    if (n_samples == 0) return MH_OK;
    hipLaunchKernelGGL(k_batch_items, dim3((unsigned)((n_samples + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                       stream, L.nets, n_networks, sample_net, n_samples, L.item_off, &L.ctr->status);
    MH_HIP_TRY(hipGetLastError());
    mh_status st = scan_exclusive_u64(L.item_off, L.item_off, n_samples, L.scratch, L.scratch_bytes, stream);
    if (st != MH_OK) return st;
    hipLaunchKernelGGL(k_batch_item_table, dim3((unsigned)(kItemTab / kThreads)), dim3(kThreads), 0, stream,
                       L.item_off, n_samples, L.item_tab, L.item_shift);
    MH_HIP_TRY(hipGetLastError());
    if (mode != MH_BATCH_EDGES) {
        const dim3 zg(64, (unsigned)(n_samples < 4096 ? n_samples : 4096));
        hipLaunchKernelGGL(k_batch_zero_degrees, zg, dim3(kThreads), 0, stream, L.nets, n_networks, sample_net, deg_off,
                           n_samples, degrees);
        MH_HIP_TRY(hipGetLastError());
    }
    if (staged) {
        // each key's (sample, window) slot region, cut at the slot capacity
        const unsigned sgrid = (unsigned)((n_samples + kThreads - 1) / kThreads);
        hipLaunchKernelGGL(k_batch_wins, dim3(sgrid), dim3(kThreads), 0, stream, L.nets, n_networks, sample_net,
                           n_samples, L.win_off);
        MH_HIP_TRY(hipGetLastError());
        st = scan_exclusive_u64(L.win_off, L.win_off, n_samples, L.scratch, L.scratch_bytes, stream);
        if (st != MH_OK) return st;
        const unsigned kgrid = (unsigned)((n_keys + kThreads - 1) / kThreads);
        hipLaunchKernelGGL(k_batch_regions, dim3(kgrid), dim3(kThreads), 0, stream, sample_net, n_samples, L.win_off,
                           L.net_win_off, L.est, n_keys, region_cap, cursor);
        MH_HIP_TRY(hipGetLastError());
        st = scan_exclusive_u64(region_cap, region_off, n_keys, L.scratch, L.scratch_bytes, stream);
        if (st != MH_OK) return st;
        hipLaunchKernelGGL(k_batch_clip, dim3(kgrid), dim3(kThreads), 0, stream, n_keys, region_off, region_cap,
                           slot_cap);
        MH_HIP_TRY(hipGetLastError());
    }
    SweepLaunch A{};
    A.batch.nets = L.nets;
    A.batch.sample_net = sample_net;
    A.batch.sample_rep = sample_rep;
    A.batch.item_off = L.item_off;
    A.batch.item_tab = L.item_tab;
    A.batch.item_shift = L.item_shift;
    A.batch.chunk_rec = L.chunk_rec;
    A.batch.n_samples = n_samples;
    A.batch.degrees = degrees;
    A.batch.deg_off = deg_off;
    A.batch.slots = slot_base;
    A.batch.win_off = L.win_off;
    A.batch.region_off = region_off;
    A.batch.region_cap = region_cap;
    A.batch.cursor = cursor;
    A.batch.slot_wins = (int32_t)L.max_win;
    A.key0 = (uint32_t)seed;
    A.key1 = (uint32_t)(seed >> 32);
    A.out = EdgeOut{src, dst, w, mode == MH_BATCH_EDGES ? capacity : 0, &L.ctr->n_edges};
    A.sid = sid;
    A.ctr = L.ctr;
    if (mode == MH_BATCH_EDGES) {
        int64_t g = 0;
        st = weighted ? launch_batch<true, OUT_EDGES>(A, grid_blocks, stream, &g)
                      : launch_batch<false, OUT_EDGES>(A, grid_blocks, stream, &g);
        if (st != MH_OK) return st;
        // the waves' unused chunk tails filled from the end of the list
        hipLaunchKernelGGL(k_gap_plan, dim3(1), dim3(kGapThreads), 0, stream, L.ctr, L.chunk_rec,
                           (int32_t)(g * kSweepWaves), capacity, L.gap);
        MH_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_gap_move, dim3(1024), dim3(kThreads), 0, stream, L.gap, src, dst, weighted ? w : nullptr,
                           sid);
        MH_HIP_TRY(hipGetLastError());
        return MH_OK;
    }
    if (!staged)
        return weighted ? launch_batch<true, OUT_DEGREES>(A, grid_blocks, stream)
                        : launch_batch<false, OUT_DEGREES>(A, grid_blocks, stream);
    st = weighted ? launch_batch<true, OUT_SLOTS>(A, grid_blocks, stream)
                  : launch_batch<false, OUT_SLOTS>(A, grid_blocks, stream);
    if (st != MH_OK) return st;
    // the regions' counts, one block per key
    hipLaunchKernelGGL(k_batch_count, dim3((unsigned)n_keys), dim3(kCountThreads), 0, stream, L.nets, sample_net,
                       n_samples, L.win_off, region_off, region_cap, cursor, slot_base, degrees, deg_off,
                       &L.ctr->status);
    MH_HIP_TRY(hipGetLastError());
    return MH_OK;
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

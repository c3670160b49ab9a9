// The rejection sweep (Sec. 2.3-2.5, Alg. 1) as a lane state machine, shared
// by the single-sample kernel and the batched persistent kernel.
//
// Work items are (row, segment) pairs of a prepared network.  Rows cut into
// two or more segments ("heavy" rows, the large-z hubs) come first in a
// network's item space, one item per segment in row order; then every row in
// rank order (r < n-1 for one node set, every row for two), which is an item
// only if the row has exactly one segment.
//
// One node set (Secs. 2.3-2.5): row r sweeps columns r+1..n-1 of the same
// sorted list, its chain starting at column r.  Two node sets (Sec. 2.6): the
// rows are the "+" nodes, the columns the "-" nodes, each sorted by its own
// parameters; every row sweeps columns 0..n_col-1 and a chain over the column
// range [a, b) starts with the proposal probability of column a itself.
//
// Each lane runs one item's chain; a lane whose chain ends takes its wave's
// next item, so the 64 lanes stay busy whatever the spread of chain lengths.
// Every loop iteration a lane consumes the global loads it issued in the
// previous iteration and issues the next ones: one memory round trip per
// iteration, overlapped with the Philox block and the logarithm of the next
// draw, which need no loaded data.
#pragma once

#include "mh_common.hpp"
#include "mh_stage.hpp"

namespace mh {

constexpr int kSweepThreads = 256;
constexpr int kSweepWaves = kSweepThreads / kWave;

enum { ST_STEPS = 0, ST_PROPOSALS, ST_ACCEPTS, ST_SEGMENTS, ST_SATURATED, ST_COUNT };

// A statistics counter alone in 256 bytes: the blocks' atomics on different
// counters then go to different lines and proceed side by side.
struct alignas(256) StatSlot {
    unsigned long long v;
    unsigned long long pad[31];
};

struct Counters {
    unsigned long long n_edges;
    int32_t status;       // first error of the current call (0: none)
    int32_t prep_status;  // a batch's preparation error, restored into status by every call on it
    StatSlot stats[ST_COUNT];
};

struct HeavyRec {
    int32_t r, g, a, b;
};

// One node by rank, packed so that a candidate costs one 16-byte load (one
// cache line) instead of separate gathers of z and id.
struct __attribute__((aligned(16))) NodeRec {
    double z;      // sorted key z (descending)
    int32_t id;    // node id at this rank
    int32_t nseg;  // segments of this rank's row
};

enum : int32_t { NET_BIPARTITE = 1, NET_NO_SELF = 2 };

// A prepared network: sorted parameters, bound and plan.  With one node set
// the column arrays alias the row arrays.
struct NetDesc {
    const NodeRec* node;   // rows by rank
    const double* ys;      // row y by rank (weighted only)
    const double* c;       // row bound 1 - Y_r (weighted only)
    const NodeRec* col;    // columns by rank
    const double* ysc;     // column y by rank (weighted only)
    const int32_t* jend;
    const uint64_t* mq;
    const uint64_t* P;     // prefix masses of the columns
    const uint64_t* hoff;  // null when unsegmented
    const HeavyRec* rec;   // records of the first rec_cap heavy items
    int64_t rec_cap;
    int64_t n;             // rows
    int64_t ncol;          // columns
    int32_t T;
    int32_t flags;         // NET_BIPARTITE, NET_NO_SELF
};

__device__ __forceinline__ int64_t lower_bound_u64(const MH_GLOBAL uint64_t* __restrict__ a, int64_t lo, int64_t hi,
                                                   uint64_t v) {
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] >= v) hi = mid; else lo = mid + 1;
    }
    return lo;
}

__device__ __forceinline__ int64_t heavy_items(const NetDesc& D) {
    return D.hoff ? (int64_t)in_global(D.hoff)[D.n] : 0;
}

__device__ __forceinline__ int64_t light_rows(const NetDesc& D) {
    return (D.flags & NET_BIPARTITE) ? D.n : (D.n > 1 ? D.n - 1 : 0);
}

__device__ __forceinline__ int64_t total_items(const NetDesc& D) { return heavy_items(D) + light_rows(D); }

// Row, segment index and column range of heavy item `it` (it < H).
__device__ inline HeavyRec heavy_record(const NetDesc& D, int64_t it) {
    const MH_GLOBAL uint64_t* hoff = in_global(D.hoff);
    const MH_GLOBAL uint64_t* P = in_global(D.P);
    const int64_t n = D.n;
    int64_t lo = 0, hi = n;  // first row index with hoff > it, minus one
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (hoff[mid] > (uint64_t)it) hi = mid; else lo = mid + 1;
    }
    const int64_t r = lo - 1;
    const int64_t g = it - (int64_t)hoff[r];
    const int64_t nsg = (int64_t)(hoff[r + 1] - hoff[r]);
    const int64_t J = in_global(D.jend)[r];
    const int64_t T = D.T;
    const int64_t first = (D.flags & NET_BIPARTITE) ? 0 : r + 1;
    const int64_t nc = D.ncol;
    const int64_t nd = (J - first + T - 1) / T;
    int64_t a, b;
    if (g < nd) {
        a = first + g * T;
        b = a + T < J ? a + T : J;
    } else {
        const int64_t kk = g - nd;
        const int64_t ns = nsg - nd;
        const uint64_t base = P[J];
        const uint64_t m = in_global(D.mq)[r];
        a = (kk == 0) ? J : lower_bound_u64(P, J, nc, base + (uint64_t)kk * m);
        b = (kk == ns - 1) ? nc : lower_bound_u64(P, J, nc, base + (uint64_t)(kk + 1) * m);
    }
    return HeavyRec{(int32_t)r, (int32_t)g, (int32_t)a, (int32_t)b};
}

// Where the items of a launch come from.  Single: one network, one replica.
// Batch: a list of (network, replica) samples laid end to end.
struct BatchRef {
    const NetDesc* nets;        // [n_networks]
    const int32_t* sample_net;  // [n_samples]
    const uint32_t* sample_rep; // [n_samples]
    const uint64_t* item_off;   // [n_samples + 1] exclusive prefix of items
    // item_tab[c]: the sample holding item c 2^item_shift[0] (c below
    // ceil(items / 2^shift)), so that a lane finds an item's sample between
    // two table entries instead of among all samples
    const int32_t* item_tab;
    const int32_t* item_shift;
    int32_t n_samples;
    int32_t* degrees;           // degree-sink output, or null
    const int64_t* deg_off;     // [n_samples] start of each sample's degree array
    // OUT_SLOTS: the accepted columns of sample s in window w (node ids
    // [w 2^15, (w + 1) 2^15)) go to the region of key g = win_off[s] + w:
    // slots[region_off[g] + k] for k < region_cap[g] (k taken from
    // cursor[g * kCursorStride], one cache line per key);
    // beyond, straight to the degrees.  slot_wins: windows of the batch's
    // largest network (at most kSlotBins).
    int32_t* slots;
    // OUT_EDGES: per wave of the launch, its last output chunk's start (or
    // ~0 when it reserved none) and the slots of it used
    unsigned long long* chunk_rec;
    const uint64_t* win_off;
    const uint64_t* region_off;
    const uint64_t* region_cap;
    unsigned long long* cursor;
    int32_t slot_wins;
};

// Output of a sweep: the edge list; per-node degrees (batched); or, for one
// network, counts by rank: cnt[j] += 1 for every edge whose endpoint of larger
// rank is j (the edges among the first K ranks number cnt[0] + ... + cnt[K-1]);
// or (batched) per-node degrees with the rows' counts added as by OUT_DEGREES
// and every accepted column written to its sample's slot region (counted later
// in LDS) instead of added by a device atomic.
enum SweepOut { OUT_EDGES = 0, OUT_DEGREES = 1, OUT_RANKS = 2, OUT_SLOTS = 3 };

// Staged degree counts: a window holds 2^kSlotWinShift node ids; a wave bins
// its staged columns into at most kSlotBins (sample, window) keys per flush.
constexpr int kSlotWinShift = 15;
constexpr int kSlotBins = 128;
// keys' cursors one 128-byte line apart: the reservations of the keys in
// flight (a few samples' windows) do not queue on one line
constexpr int kCursorStride = 16;
// LDS of one wave's flush: kSlotBins slot addresses (u64) and room counts (u32)
constexpr int kSlotLdsWords = kSlotBins * 3;

// A wave's staged (column, sample) pairs into their keys' slot regions.  The
// keys of one flush are binned by (sample - lowest sample, window): an LDS
// atomic gives each pair its rank in its bin, one device atomic per non-empty
// bin reserves the bin's run in its region, and the pairs are written there.
// Pairs of a sample too far from the lowest one to bin, and pairs past their
// region's end, add to the degrees directly.  s_col holds node ids, s_smp
// samples (overwritten); s_lds: kSlotLdsWords words of this wave.
__device__ __forceinline__ void flush_slots(const int32_t* s_col, int32_t* s_smp, int32_t* s_lds, uint32_t fill,
                                            const BatchRef& B) {
    if (fill == 0) return;
    __builtin_amdgcn_wave_barrier();
    uint64_t* s_start = reinterpret_cast<uint64_t*>(s_lds);
    uint32_t* s_room = reinterpret_cast<uint32_t*>(s_lds + 2 * kSlotBins);
    const int lane = (int)(threadIdx.x & 63);
    const int32_t nw = B.slot_wins;
    const int32_t span = kSlotBins / nw;
    int32_t lo = 0x7FFFFFFF;
    for (uint32_t k = (uint32_t)lane; k < fill; k += kWave) lo = min(lo, s_smp[k]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lo = min(lo, __shfl_xor(lo, off, kWave));
    for (int b = lane; b < kSlotBins; b += kWave) s_room[b] = 0u;
    __builtin_amdgcn_wave_barrier();
    // 1. each pair's bin and rank in it (code >= 0), or -(sample + 1)
    for (uint32_t k = (uint32_t)lane; k < fill; k += kWave) {
        const int32_t smp = s_smp[k];
        const int32_t d = smp - lo;
        int32_t code = -(smp + 1);
        if (d < span) {
            const uint32_t bin = (uint32_t)(d * nw + (s_col[k] >> kSlotWinShift));
            const uint32_t r = atomicAdd(&s_room[bin], 1u);
            code = (int32_t)((bin << 16) | r);
        }
        s_smp[k] = code;
    }
    __builtin_amdgcn_wave_barrier();
    // 2. one reservation per non-empty bin: where its run starts, and how much
    //    of it fits in the region
    for (int b = lane; b < kSlotBins; b += kWave) {
        const uint32_t c = s_room[b];
        if (c == 0) continue;
        const int32_t smp = lo + b / nw;
        const uint64_t g = B.win_off[smp] + (uint64_t)(b % nw);
        const uint64_t at = atomicAdd(&B.cursor[g * kCursorStride], (unsigned long long)c);
        const uint64_t cap = B.region_cap[g];
        const uint64_t room = at < cap ? cap - at : 0;
        s_start[b] = B.region_off[g] + at;
        s_room[b] = room < c ? (uint32_t)room : c;
    }
    __builtin_amdgcn_wave_barrier();
    // 3. the writes
    for (uint32_t k = (uint32_t)lane; k < fill; k += kWave) {
        const int32_t code = s_smp[k];
        const int32_t col = s_col[k];
        if (code >= 0) {
            const uint32_t bin = (uint32_t)code >> 16, r = (uint32_t)code & 0xFFFFu;
            if (r < s_room[bin]) {
                B.slots[s_start[bin] + r] = col;
            } else {
                const int32_t smp = lo + (int32_t)bin / nw;
                atomicAdd(&B.degrees[B.deg_off[smp] + col], 1);
            }
        } else {
            atomicAdd(&B.degrees[B.deg_off[-code - 1] + col], 1);
        }
    }
    __builtin_amdgcn_wave_barrier();
}

struct SweepLaunch {
    NetDesc net;        // single-sample network (unused in batch launches)
    uint32_t replica;   // single-sample replica
    BatchRef batch;
    uint32_t key0, key1;
    EdgeOut out;
    int32_t* sid;       // batch edge output: sample id per edge (may be null)
    int32_t* rank_cnt;  // OUT_RANKS: counts by the larger endpoint's rank [n]
    Counters* ctr;
};

// Lane states
enum : uint32_t { S_IDLE = 0, S_REC, S_LOAD, S_STEP, S_DONE };
// Idle lanes a batched wave gathers before it refills them (edge and slot
// output; measured on a 4,096-sample ensemble: 1 -> 8 took edge output from
// 15,730 to 17,359 replicas/s and the staged degree sink from 14,383 to
// 17,579; the atomic sink, bound by its atomics, lost 4%, and one sample of
// N = 1M, whose lanes finish an item every few steps, did not change).
constexpr int kRefillMin = 8;

// BIP: two node sets (single-sample launches only); the column arrays and the
// chain start differ, and NET_NO_SELF rejects the candidate with the row's id.
// CL: the Chung-Lu model read as probabilities, p = min(t, 1) (Sec. 2.1), by
// the Miller-Hagberg chain of Sec. 2.3 (unweighted, one node set): proposal
// q = min(t_q, 1), skip -log U1 / -log(1 - q), 0 when q = 1, accept U2 q < p.
// Returns the number of edges left in the wave's stage (written by the caller).
// STATS: the wave's counts are left in st_out[ST_COUNT] (LDS) for the block.
template <bool WEIGHTED, bool STATS, bool BATCH, int OUT, bool BIP, bool CL = false>
__device__ __forceinline__ uint32_t sweep_body(const SweepLaunch& A, int32_t* s_src, int32_t* s_dst, int32_t* s_w,
                                           int32_t* s_sid, unsigned long long* st_out) {
    static_assert(!(BIP && BATCH), "two-set networks are sampled one at a time");
    static_assert(!(CL && (WEIGHTED || BIP || BATCH)), "the Chung-Lu chain is unweighted, one set, one sample");
    static_assert(OUT != OUT_RANKS || !(BATCH || BIP), "counts by rank are kept for one network");
    static_assert(OUT != OUT_SLOTS || BATCH, "slot regions belong to batched samples");
    const int wave = threadIdx.x >> 6;
    const int64_t gwave = (int64_t)blockIdx.x * kSweepWaves + wave;
    const int64_t nwaves = (int64_t)gridDim.x * kSweepWaves;
    const uint64_t lt = lanemask_lt();
    int64_t total;
    int64_t H_single = 0;
    int32_t ishift = 0;
    int64_t nchunks = 0;
    if (BATCH) {
        total = (int64_t)A.batch.item_off[A.batch.n_samples];
        ishift = *A.batch.item_shift;
        nchunks = (total + (int64_t(1) << ishift) - 1) >> ishift;
    } else {
        H_single = heavy_items(A.net);
        total = H_single + light_rows(A.net);
    }
    const bool no_self = BIP && (A.net.flags & NET_NO_SELF);

    WaveStage<WEIGHTED> stage{s_src, s_dst, WEIGHTED ? s_w : nullptr, 0u};

    uint32_t st_steps = 0, st_props = 0, st_acc = 0, st_segs = 0, st_sat = 0;
    uint32_t state = S_IDLE;
    bool check_light = false;
    int32_t r = 0, pos = 0, end = 0, jc = 0;
    uint32_t step = 0, tag = 0, scand = 0, replica = A.replica;
    int32_t id = 0, sample = 0, row_deg = 0;
    double s = 0.0, cr = 1.0, ysr = 0.0, tq = 0.0, U2 = 0.0;
    // the lane's network
    const MH_GLOBAL NodeRec* node = in_global(A.net.node);
    const MH_GLOBAL double* ys = in_global(A.net.ys);
    // column arrays: their own only with two node sets (never batched); with
    // one set the candidates are read through `node` / `ys`, which follow the
    // lane's current network
    const MH_GLOBAL NodeRec* col = in_global(BIP ? A.net.col : nullptr);
    const MH_GLOBAL double* ysc = in_global(BIP ? A.net.ysc : nullptr);
    int32_t* deg = nullptr;
    // Values in flight from the previous iteration's loads.  The steps below
    // only choose addresses; each value is then loaded at one place at the end
    // of the iteration and read in the next, so its latency overlaps the next
    // draw (a value merged from several loads would need a copy, and the copy
    // a wait for the load).
    NodeRec ra{0.0, 0, 1};     // the candidate (z, id), or the row being set up (z, id, nseg)
    double rb = 0.0;           // z of the column before a segment's chain (heavy segments, light rows of two sets)
    HeavyRec rc{0, 0, 0, 0};   // a heavy segment's record
    double ry = 0.0, rcc = 1.0;  // weighted: y of the candidate or of the row; the row's bound
    bool start_rb = false;     // the chain of the row being set up starts at rb, else at the row itself
    bool rec_direct = false;   // rc is beyond the stored records: computed in S_REC from rc_it
    int64_t rc_it = 0;
    int64_t kbase = 0;

    for (;;) {
        const MH_GLOBAL NodeRec* pa = nullptr;
        const MH_GLOBAL double* pb = nullptr;
        const MH_GLOBAL double* py = nullptr;
        const MH_GLOBAL double* pc = nullptr;
        const MH_GLOBAL HeavyRec* prc = nullptr;
        // 1. the next draw of every lane that will draw this iteration
        const bool draws = (state == S_STEP) || (state == S_LOAD);
        double E = 0.0, U2n = 0.0;
        if (draws) {
            const u32x4 R = philox4x32_10(step, (uint32_t)r, replica, tag, A.key0, A.key1);
            E = -log_fast(uniform53(R.v0, R.v1));
            U2n = uniform53(R.v2, R.v3);
        }
        // 2. consume the loads of the previous iteration
        bool acc = false, go = false;
        int32_t dst_id = 0, wt = 0;
        if (state == S_STEP) {
            const double t = s * ra.z;
            double lhs, rhs;
            if (CL) {
                lhs = U2 * (tq < 1.0 ? tq : 1.0);
                rhs = t < 1.0 ? t : 1.0;
            } else if (WEIGHTED) {
                const double e = 1.0 - ysr * ry;
                lhs = (U2 * tq) * (e + t);
                rhs = t * (cr + tq);
            } else {
                lhs = (U2 * tq) * (1.0 + t);
                rhs = t * (1.0 + tq);
            }
            ++st_props;
            if (lhs < rhs && !(BIP && no_self && ra.id == id)) {
                acc = true;
                ++st_acc;
                dst_id = ra.id;
                if (WEIGHTED) {
                    const double bb = ysr * ry;
                    if (bb == 0.0) {
                        wt = 1;
                    } else {
                        const u32x4 V = philox4x32_10(scand, (uint32_t)r, replica, tag | 1u, A.key0, A.key1);
                        const double ratio = log_fast(uniform53(V.v0, V.v1)) / log_fast(bb);
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
            if (check_light && ra.nseg != 1) {
                state = S_IDLE;
            } else {
                s = ra.z;
                id = ra.id;
                tq = s * (start_rb ? rb : ra.z);
                cr = WEIGHTED ? rcc : 1.0;
                ysr = WEIGHTED ? ry : 0.0;
                ++st_segs;
                go = true;
            }
        } else if (state == S_REC) {
            const NetDesc& D = BATCH ? A.batch.nets[A.batch.sample_net[sample]] : A.net;
            HeavyRec hr = rc;
            if (rec_direct) {
                hr = heavy_record(D, rc_it);
                // Some of heavy_record's loads go unused on some paths; left
                // outstanding, they would make the compiler wait for all loads
                // (the counter is in order) at the top of the next iteration,
                // in front of this iteration's candidate loads.  vmcnt(0) here
                // (expcnt and lgkmcnt at their no-wait maxima) settles them.
                __builtin_amdgcn_s_waitcnt(0x0F70);
            }
            r = hr.r;
            pos = hr.a - 1;
            end = hr.b;
            tag = (uint32_t)hr.g << 1;
            step = 0;
            check_light = false;
            if (hr.a >= hr.b) {
                state = S_IDLE;
            } else {
                pa = &node[r];
                pb = BIP ? &col[hr.a].z : &node[pos].z;
                if (WEIGHTED) {
                    pc = in_global(&D.c[r]);
                    py = &ys[r];
                }
                start_rb = true;
                state = S_LOAD;
            }
        }
        if (OUT == OUT_DEGREES && acc) {
            ++row_deg;
            atomicAdd(&deg[dst_id], 1);
        }
        if (OUT == OUT_SLOTS && acc) ++row_deg;
        if (OUT == OUT_RANKS && acc) atomicAdd(&A.rank_cnt[pos], 1);  // pos: the accepted column's rank
        // the accepted edge's sample: step 4 may move the lane to an item of the next sample
        const int32_t acc_sample = sample;
        // 3. the skip: candidate pos + 1 + floor(-log U1 / -log(1 - q)), or the end of the segment
        if (go) {
            bool ended = true;
            if (tq != 0.0) {
                ++st_steps;
                double d;
                if (CL) {
                    // -log(1 - q) = -log1p(-t_q) for t_q < 1; every column is a candidate at q = 1
                    d = tq >= 1.0 ? 0.0 : E / -log1p_fast(-tq);
                } else {
                    const double lq = WEIGHTED ? log1p_fast(tq / cr) : log1p_fast(tq);
                    d = E / lq;
                }
                const double room = (double)(end - 1 - pos);
                if (d < room) {
                    ended = false;
                    jc = pos + 1 + (int32_t)d;
                    U2 = U2n;
                    scand = step;
                    ++step;
                    pa = &(BIP ? col : node)[jc];
                    if (WEIGHTED) py = &(BIP ? ysc : ys)[jc];
                    state = S_STEP;
                }
            }
            if (ended) {
                state = S_IDLE;
                if ((OUT == OUT_DEGREES || OUT == OUT_SLOTS) && row_deg) atomicAdd(&deg[id], row_deg);
                row_deg = 0;
            }
        }
        // 4. idle lanes take the wave's next items and issue their loads
        // (batched edge and slot output: only once kRefillMin lanes wait, or
        // none is busy, so that the refill's instructions, which run with
        // just the idle lanes active, are shared by several lanes)
        const uint64_t idle = __ballot(state == S_IDLE);
        bool refill = idle != 0;
        if (BATCH && OUT != OUT_DEGREES && refill && __popcll(idle) < kRefillMin)
            refill = __ballot(state == S_REC || state == S_LOAD || state == S_STEP) == 0;
        if (refill) {
            if (state == S_IDLE) {
                int64_t it = gwave + (kbase + __popcll(idle & lt)) * nwaves;
                if (it >= total) {
                    state = S_DONE;
                } else {
                    int64_t H = H_single;
                    const NetDesc* Dp = &A.net;
                    if (BATCH) {
                        // sample with item_off <= it < next: between the samples of
                        // the table's chunk starts around it
                        const int64_t c = it >> ishift;
                        int32_t lo = A.batch.item_tab[c];
                        int32_t hi = c + 1 < nchunks ? A.batch.item_tab[c + 1] + 1 : A.batch.n_samples;
                        while (hi - lo > 1) {
                            const int32_t mid = (lo + hi) >> 1;
                            if (A.batch.item_off[mid] <= (uint64_t)it) lo = mid; else hi = mid;
                        }
                        sample = lo;
                        it -= (int64_t)A.batch.item_off[lo];
                        Dp = &A.batch.nets[A.batch.sample_net[lo]];
                        replica = A.batch.sample_rep[lo];
                        H = heavy_items(*Dp);
                        node = in_global(Dp->node);
                        ys = in_global(Dp->ys);
                        if (OUT == OUT_DEGREES || OUT == OUT_SLOTS) deg = A.batch.degrees + A.batch.deg_off[lo];
                    }
                    if (it < H) {
                        rec_direct = it >= Dp->rec_cap;
                        rc_it = it;
                        if (!rec_direct) prc = in_global(&Dp->rec[it]);
                        state = S_REC;
                    } else {
                        r = (int32_t)(it - H);
                        pos = BIP ? -1 : r;
                        end = (int32_t)(BIP ? Dp->ncol : Dp->n);
                        tag = 0;
                        step = 0;
                        check_light = true;
                        pa = &node[r];
                        if (BIP) pb = &col[0].z;
                        start_rb = BIP;
                        if (WEIGHTED) {
                            pc = in_global(&Dp->c[r]);
                            py = &ys[r];
                        }
                        state = S_LOAD;
                    }
                }
            }
            kbase += __popcll(idle);
        }
        // 5. this iteration's loads, read in the next
        if (pa) ra = *pa;
        if (pb) rb = *pb;
        if (prc) rc = *prc;
        if (WEIGHTED) {
            if (py) ry = *py;
            if (pc) rcc = *pc;
        }
        if (OUT == OUT_EDGES) stage.template push_sid<BATCH>(acc, id, dst_id, wt, acc_sample, s_sid, A.out, A.sid);
        if (OUT == OUT_SLOTS) {
            const uint64_t am = __ballot(acc);
            if (am) {
                if (acc) {
                    const uint32_t o = stage.fill + (uint32_t)__popcll(am & lt);
                    s_dst[o] = dst_id;
                    s_sid[o] = acc_sample;
                }
                stage.fill += (uint32_t)__popcll(am);
                if (stage.fill > (uint32_t)kStageFlushAt) {
                    flush_slots(s_dst, s_sid, s_src, stage.fill, A.batch);
                    stage.fill = 0;
                }
            }
        }
        if (__ballot(state != S_DONE) == 0) break;
    }
    if (OUT == OUT_SLOTS) {
        flush_slots(s_dst, s_sid, s_src, stage.fill, A.batch);
        stage.fill = 0;
    }
    if (BATCH && OUT == OUT_EDGES) {
        stage.flush_chunked(s_sid, A.out, A.sid);
        if ((threadIdx.x & 63) == 0) {
            const bool any = stage.cend != 0;
            A.batch.chunk_rec[2 * gwave] = any ? stage.cend - kOutChunk : ~0ull;
            A.batch.chunk_rec[2 * gwave + 1] = any ? stage.cpos - (stage.cend - kOutChunk) : 0ull;
        }
    }
    if (STATS) {
        const unsigned long long v0 = wave_sum((unsigned long long)st_steps);
        const unsigned long long v1 = wave_sum((unsigned long long)st_props);
        const unsigned long long v2 = wave_sum((unsigned long long)st_acc);
        const unsigned long long v3 = wave_sum((unsigned long long)st_segs);
        const unsigned long long v4 = wave_sum((unsigned long long)st_sat);
        if ((threadIdx.x & 63) == 0) {
            st_out[ST_STEPS] = v0;
            st_out[ST_PROPOSALS] = v1;
            st_out[ST_ACCEPTS] = v2;
            st_out[ST_SEGMENTS] = v3;
            st_out[ST_SATURATED] = v4;
        }
    }
    return stage.fill;
}

template <bool WEIGHTED, bool STATS, bool BATCH, int OUT, bool BIP = false, bool CL = false>
__global__ __launch_bounds__(kSweepThreads) void k_sweep(SweepLaunch A) {
    constexpr int kStage = (OUT == OUT_EDGES || OUT == OUT_SLOTS) ? kStageEdges : 1;
    // OUT_SLOTS: s_src holds the flush's bins (8-byte aligned words)
    __shared__ __attribute__((aligned(8))) int32_t
        s_src[kSweepWaves][OUT == OUT_EDGES ? kStage : (OUT == OUT_SLOTS ? kSlotLdsWords : 1)];
    __shared__ int32_t s_dst[kSweepWaves][kStage];
    __shared__ int32_t s_w[WEIGHTED ? kSweepWaves : 1][WEIGHTED ? kStage : 1];
    __shared__ int32_t s_sid[BATCH ? kSweepWaves : 1][BATCH ? kStage : 1];
    __shared__ uint32_t s_fill[kSweepWaves];
    __shared__ uint32_t s_arrived;
    __shared__ unsigned long long s_st[STATS ? kSweepWaves : 1][ST_COUNT];
    if (A.ctr->status != 0) return;
    if (threadIdx.x == 0) s_arrived = 0;
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const uint32_t fill = sweep_body<WEIGHTED, STATS, BATCH, OUT, BIP, CL>(
        A, s_src[wave], s_dst[wave], WEIGHTED ? s_w[wave] : nullptr, BATCH ? s_sid[wave] : nullptr,
        STATS ? s_st[wave] : nullptr);
    bool last = false;
    if (OUT == OUT_EDGES)
        last = block_final_flush<WEIGHTED, kSweepWaves>(fill, &s_src[0][0], &s_dst[0][0],
                                                        WEIGHTED ? &s_w[0][0] : nullptr, BATCH ? &s_sid[0][0] : nullptr,
                                                        s_fill, &s_arrived, A.out, A.sid);
    else if (STATS)
        last = block_arrive<kSweepWaves>(&s_arrived);
    // the block's statistics: one atomic per counter, from the last wave
    if (STATS && last) {
        const int lane = (int)(threadIdx.x & 63);
        if (lane < ST_COUNT) {
            unsigned long long t = 0;
#pragma unroll
            for (int w = 0; w < kSweepWaves; ++w) t += s_st[w][lane];
            atomicAdd(&A.ctr->stats[lane].v, t);
        }
    }
}

}  // namespace mh

// Host-side preparation of a network (order, bound, plan) shared by the
// single-sample and batched entry points.
#pragma once

#include "mh_internal.hpp"
#include "mh_sweep_core.hpp"

namespace mh {

// Device buffers of one prepared network (writable views of a NetDesc).
struct NetBuffers {
    NodeRec* node;
    double* ys;
    double* c;
    uint64_t* P;
    int32_t* jend;
    uint64_t* mq;
    uint64_t* hoff;
    HeavyRec* rec;
    int64_t rec_cap;
    uint64_t* scan_state;  // look-back state of the two plan scans (P, then hoff)
    int64_t scan_words;
    uint64_t* Psamp;       // P[256 k] (written by the order's one-pass scan)
    double* Zsamp;         // z[256 k] (the same)
    int32_t* hbrow;        // first row of every round of heavy items (written by the plan's scan)
    int64_t n;
    int32_t T;
    bool weighted;
};

size_t network_bytes(int64_t n, bool weighted, int32_t T);
NetBuffers carve_network(Arena& ar, int64_t n, bool weighted, int32_t T);
size_t prepare_scratch_bytes(int64_t n);
NetDesc net_desc(const NetBuffers& B);
mh_status init_counters(Counters* c, hipStream_t stream);
// Records ev[1] after the order step when ev is non-null.
// counters: u64 words (the sample's counters) for the first kernel to clear.
mh_status prepare_network(const double* x, const double* y, const NetBuffers& B, int32_t* status, void* scratch,
                          size_t scratch_bytes, hipStream_t stream, hipEvent_t* ev, ZeroRange counters = {});

}  // namespace mh

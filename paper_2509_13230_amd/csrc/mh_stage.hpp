// Per-wave edge staging: accepted edges are packed into a wave-private LDS
// buffer by ballot + popcount and written out in coalesced runs, with one
// device-scope atomic per run to reserve output slots.
#pragma once

#include "mh_common.hpp"

namespace mh {

constexpr int kStageEdges = 512;               // per wave
constexpr int kStageFlushAt = kStageEdges - kWave;

struct EdgeOut {
    int32_t* src;
    int32_t* dst;
    int32_t* w;  // may be null
    int64_t capacity;
    unsigned long long* count;  // device counter of emitted edges
};

template <bool WEIGHTED>
struct WaveStage {
    int32_t* s_src;
    int32_t* s_dst;
    int32_t* s_w;
    uint32_t fill;  // wave-uniform

    __device__ __forceinline__ void push(bool acc, int32_t a, int32_t b, int32_t wt, const EdgeOut& out) {
        const uint64_t am = __ballot(acc);
        if (am == 0) return;
        if (acc) {
            const uint32_t o = fill + (uint32_t)__popcll(am & lanemask_lt());
            s_src[o] = a;
            s_dst[o] = b;
            if (WEIGHTED) s_w[o] = wt;
        }
        fill += (uint32_t)__popcll(am);
        if (fill > (uint32_t)kStageFlushAt) flush(out);
    }

    // Variants that also stage a sample id per edge (s_sid, sid_out may be null).
    __device__ __forceinline__ void push_sid(bool acc, int32_t a, int32_t b, int32_t wt, int32_t sample,
                                             int32_t* s_sid, const EdgeOut& out, int32_t* sid_out) {
        const uint64_t am = __ballot(acc);
        if (am == 0) return;
        if (acc) {
            const uint32_t o = fill + (uint32_t)__popcll(am & lanemask_lt());
            s_src[o] = a;
            s_dst[o] = b;
            if (WEIGHTED) s_w[o] = wt;
            if (s_sid) s_sid[o] = sample;
        }
        fill += (uint32_t)__popcll(am);
        if (fill > (uint32_t)kStageFlushAt) flush_sid(s_sid, out, sid_out);
    }

    __device__ __forceinline__ void flush_sid(const int32_t* s_sid, const EdgeOut& out, int32_t* sid_out) {
        if (fill == 0) return;
        __builtin_amdgcn_wave_barrier();
        const int lane = (int)__lane_id();
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(out.count, (unsigned long long)fill);
        base = __shfl(base, 0, kWave);
        for (uint32_t k = (uint32_t)lane; k < fill; k += kWave) {
            const unsigned long long idx = base + k;
            if (idx < (unsigned long long)out.capacity) {
                out.src[idx] = s_src[k];
                out.dst[idx] = s_dst[k];
                if (WEIGHTED) out.w[idx] = s_w[k];
                if (s_sid && sid_out) sid_out[idx] = s_sid[k];
            }
        }
        __builtin_amdgcn_wave_barrier();
        fill = 0;
    }

    __device__ __forceinline__ void flush(const EdgeOut& out) {
        if (fill == 0) return;
        __builtin_amdgcn_wave_barrier();
        const int lane = (int)__lane_id();
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(out.count, (unsigned long long)fill);
        base = __shfl(base, 0, kWave);
        for (uint32_t k = (uint32_t)lane; k < fill; k += kWave) {
            const unsigned long long idx = base + k;
            if (idx < (unsigned long long)out.capacity) {
                out.src[idx] = s_src[k];
                out.dst[idx] = s_dst[k];
                if (WEIGHTED) out.w[idx] = s_w[k];
            }
        }
        __builtin_amdgcn_wave_barrier();
        fill = 0;
    }
};

}  // namespace mh

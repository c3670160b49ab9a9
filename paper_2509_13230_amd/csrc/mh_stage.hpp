// Per-wave edge staging: accepted edges are packed into a wave-private LDS
// buffer by ballot + popcount and written out in coalesced runs, with one
// device-scope atomic per run to reserve output slots.  All waves reserve
// from one counter, and a device atomic on one address is serviced about once
// per 12 ns on MI355X, so runs are long (a wave flushes at ~1000 edges) and
// the last, partial runs of a block's waves are written together, with one
// atomic, by the block's last wave to finish.
#pragma once

#include "mh_common.hpp"

namespace mh {

constexpr int kStageEdges = 1024;              // per wave
constexpr int kStageFlushAt = kStageEdges - kWave;
// Batched edge output: a wave reserves output slots kOutChunk at a time
// (flush_chunked), so that the one output counter sees an atomic per
// kOutChunk edges; each wave's last chunk keeps an unused tail that a later
// pass fills from the end of the list.
constexpr uint32_t kOutChunk = 4096;
static_assert(kStageEdges < (int)kOutChunk, "a staged run spans at most two chunks");

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
    unsigned long long cpos = 0, cend = 0;  // flush_chunked: the wave's chunk [cend - kOutChunk, cend), next slot cpos

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

    // Variants that also stage a sample id per edge (s_sid, sid_out may be null);
    // CHUNKED: runs go out through flush_chunked.
    template <bool CHUNKED = false>
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
        if (fill > (uint32_t)kStageFlushAt) {
            if (CHUNKED) flush_chunked(s_sid, out, sid_out);
            else flush_sid(s_sid, out, sid_out);
        }
    }

    // The staged run into the wave's chunk, reserving the next chunk when the
    // current one is full (a run fills at most one chunk and starts the next:
    // kStageEdges < kOutChunk).  Slots at or beyond out.capacity are not written.
    __device__ __forceinline__ void flush_chunked(const int32_t* s_sid, const EdgeOut& out, int32_t* sid_out) {
        if (fill == 0) return;
        __builtin_amdgcn_wave_barrier();
        const int lane = (int)__lane_id();
        uint32_t done = 0;
        while (done < fill) {
            if (cpos == cend) {
                unsigned long long b = 0;
                if (lane == 0) b = atomicAdd(out.count, (unsigned long long)kOutChunk);
                b = __shfl(b, 0, kWave);
                cpos = b;
                cend = b + kOutChunk;
            }
            const uint32_t room = (uint32_t)(cend - cpos);
            const uint32_t take = fill - done < room ? fill - done : room;
            for (uint32_t k = (uint32_t)lane; k < take; k += kWave) {
                const unsigned long long idx = cpos + k;
                if (idx < (unsigned long long)out.capacity) {
                    out.src[idx] = s_src[done + k];
                    out.dst[idx] = s_dst[done + k];
                    if (WEIGHTED) out.w[idx] = s_w[done + k];
                    if (s_sid && sid_out) sid_out[idx] = s_sid[done + k];
                }
            }
            cpos += take;
            done += take;
        }
        __builtin_amdgcn_wave_barrier();
        fill = 0;
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

// A wave counts itself in *s_arrived (LDS, zeroed at block start) once its
// LDS writes are done; true for the block's last wave, which then sees every
// other wave's writes.
template <int WAVES>
__device__ __forceinline__ bool block_arrive(uint32_t* s_arrived) {
    __threadfence_block();
    uint32_t prev = 0;
    if (__lane_id() == 0) prev = atomicAdd(s_arrived, 1u);
    prev = __shfl(prev, 0, kWave);
    if (prev != (uint32_t)(WAVES - 1)) return false;
    __threadfence_block();
    return true;
}

// End of a block's work: each wave leaves its unflushed count in s_fill and
// arrives (block_arrive); the last wave to arrive reserves the slots of all
// the block's stages with one atomic and writes them.  Stage w of kind X is
// at s_X + w * kStageEdges.  Returns whether this wave was the last.
template <bool WEIGHTED, int WAVES>
__device__ __forceinline__ bool block_final_flush(uint32_t fill, const int32_t* s_src, const int32_t* s_dst,
                                                  const int32_t* s_w, const int32_t* s_sid, uint32_t* s_fill,
                                                  uint32_t* s_arrived, const EdgeOut& out, int32_t* sid_out) {
    const int lane = (int)__lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    if (lane == 0) s_fill[wave] = fill;
    if (!block_arrive<WAVES>(s_arrived)) return false;
    uint32_t offs[WAVES];
    uint32_t total = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        offs[w] = total;
        total += s_fill[w];
    }
    if (total == 0) return true;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(out.count, (unsigned long long)total);
    base = __shfl(base, 0, kWave);
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        const uint32_t f = s_fill[w];
        const int off = w * kStageEdges;
        for (uint32_t k = (uint32_t)lane; k < f; k += kWave) {
            const unsigned long long idx = base + offs[w] + k;
            if (idx < (unsigned long long)out.capacity) {
                out.src[idx] = s_src[off + k];
                out.dst[idx] = s_dst[off + k];
                if (WEIGHTED) out.w[idx] = s_w[off + k];
                if (s_sid && sid_out) sid_out[idx] = s_sid[off + k];
            }
        }
    }
    return true;
}

}  // namespace mh

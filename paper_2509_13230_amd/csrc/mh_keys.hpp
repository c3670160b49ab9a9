// Sort keys of the node order and their digit histograms, shared by the key
// preparation kernel and the radix pass that prepares its own keys.
#pragma once

#include "mh_common.hpp"

namespace mh {

// Loaded parameters of a node: z = x (or fl(x y) when weighted), and whether
// they are valid (finite, non-negative; z finite).  Invalid nodes sort as
// z = 0 and the caller raises MH_EINVAL.
__device__ __forceinline__ double node_z(double xi, bool weighted, double yi, bool* ok) {
    double z;
    if (weighted) {
        *ok = (yi >= 0.0) && isfinite(yi) && (xi >= 0.0) && isfinite(xi);
        z = xi * yi;
    } else {
        *ok = (xi >= 0.0) && isfinite(xi);
        z = xi;
    }
    *ok = *ok && isfinite(z);
    return *ok ? z : 0.0;
}

// The split sort key of node i: high half of desc_key(z) as the radix key, the
// low half above the id as payload.
__device__ __forceinline__ void split_key(double z, int64_t i, uint32_t* hi, uint64_t* pay) {
    const uint64_t full = desc_key(z);
    *hi = (uint32_t)(full >> 32);
    *pay = (full << 32) | (uint64_t)(uint32_t)i;
}

// Adds one key per lane (among `valid`) to LDS digit histograms
// h[(p - p0) * 256 + d] for the passes p0 <= p < p1 (byte p of the key).  Lanes holding the key of
// their group's first lane (groups by an 8-bit fold of the key) are counted
// once by that lane: tied parameters, common in fitted inputs, would otherwise
// all hit one LDS bin.
__device__ __forceinline__ void count_key_digits(uint32_t* h, uint32_t key, bool valid, int p0, int p1) {
    const int lane = threadIdx.x & 63;
    const uint32_t fold = (key ^ (key >> 8) ^ (key >> 16) ^ (key >> 24)) & 255u;
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (fold >> b) & 1u;
        const uint64_t vote = __ballot(bit);
        m &= bit ? vote : ~vote;
    }
    const int leader = valid ? (int)__ffsll((unsigned long long)m) - 1 : lane;
    const uint32_t lkey = __shfl(key, leader, kWave);
    const uint64_t same = __ballot(valid && key == lkey);
    if (valid) {
        uint32_t add = 0;
        if (lane == leader) add = (uint32_t)__popcll(same & m);
        else if (!((same >> lane) & 1ull)) add = 1;
        if (add) {
            for (int p = p0; p < p1; ++p) atomicAdd(&h[(p - p0) * 256 + ((key >> (8 * p)) & 255)], add);
        }
    }
}

}  // namespace mh

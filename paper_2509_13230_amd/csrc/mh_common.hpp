// Device helpers shared by the HIP kernels of libmh (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mh.h"

namespace mh {

constexpr int kWave = 64;

// ------------------------------------------------------------------ Philox4x32-10
// Counter-based generator of Salmon, Moraes, Dror and Shaw (SC'11): ten rounds
// of two 32x32->64 multiplies by fixed odd constants, with the 64-bit products'
// halves xored against the other counter words and a Weyl-incremented key.
// The key is wave-uniform (the seed), so its schedule stays in scalar registers.
struct u32x4 {
    uint32_t v0, v1, v2, v3;
};

__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// Uniform in (0, 1] from 53 bits: (((a << 21) | (b >> 11)) + 1) * 2^-53, exact in binary64.
__device__ __forceinline__ double uniform53(uint32_t a, uint32_t b) {
    const uint64_t m = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
    return (double)(m + 1u) * 0x1.0p-53;
}

// ------------------------------------------------------------------ wave primitives
__device__ __forceinline__ uint64_t lanemask_lt() {
    const unsigned lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64u - lane));
}

__device__ __forceinline__ int wave_popc(uint64_t m) { return __popcll(m); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// inclusive scan over the 64 lanes
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
    const int lane = (int)__lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        T u = __shfl_up(v, off, kWave);
        if (lane >= off) v += u;
    }
    return v;
}

// ------------------------------------------------------------------ key bits
// Non-negative binary64 values order like their bit patterns; the complement
// orders them descending.  -0.0 is folded to +0.0 first.
__device__ __forceinline__ uint64_t desc_key(double z) {
    if (z == 0.0) z = 0.0;
    return ~(uint64_t)__double_as_longlong(z);
}

__device__ __forceinline__ double key_value(uint64_t key) {
    return __longlong_as_double((long long)~key);
}

// Column mass of the plan rule: floor(z 2^32), 2^32 when z >= 1.
__device__ __forceinline__ uint64_t mass_q(double z) {
    if (z >= 1.0) return (uint64_t)1 << 32;
    return (uint64_t)(z * 4294967296.0);
}

// Device status word: the first error wins.
__device__ __forceinline__ void raise_status(int32_t* status, int32_t code) {
    if (status) atomicCAS(status, 0, code);
}

}  // namespace mh

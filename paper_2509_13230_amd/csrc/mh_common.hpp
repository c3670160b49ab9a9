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
        // three-input xors: one v_bitop3_b32 each (truth table 0x96 = a ^ b ^ c)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// a * b + c as the three-address v_fma_f64.  In the sweep kernels the
// compiler otherwise evaluates such a step as a copy of the loop-invariant
// constant register followed by the two-address v_fmac_f64 (two instructions
// instead of one); the result is the same correctly rounded fma.
__device__ __forceinline__ double fma_vop3(double a, double b, double c) {
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

// 1/d for d in [2^-1000, 2^1000]: the hardware estimate refined by two
// Newton-Raphson steps, within about 1 ulp (callers route other d elsewhere).
__device__ __forceinline__ double newton_rcp(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    return fma(fma(-d, r, 1.0), r, r);
}

// Uniform in (0, 1] from 53 bits: (((a << 21) | (b >> 11)) + 1) * 2^-53, exact in binary64.
__device__ __forceinline__ double uniform53(uint32_t a, uint32_t b) {
    // m = hi 2^32 + lo with hi = a >> 11 and lo = the low word of (a:b) >> 11;
    // (m + 1) 2^-53 = hi 2^-21 + (lo + 1) 2^-53, each fma exact (each result
    // is a multiple of 2^-53 no larger than 1, so it fits 53 bits)
    const uint32_t hi = a >> 11;
    const uint32_t lo = __builtin_amdgcn_alignbit(a, b, 11);
    return fma_vop3((double)hi, 0x1.0p-21, fma_vop3((double)lo, 0x1.0p-53, 0x1.0p-53));
}

// ------------------------------------------------------------------ wave primitives
// A pointer into device memory, typed as such.  Pointers that a kernel reads
// from device memory (a batch's table of networks) are otherwise compiled as
// generic pointers: their loads become flat loads, and before a flat load the
// compiler waits for every outstanding memory and LDS operation of the wave,
// atomics included.  (The host pass parses device code without running it,
// and its C++ rules refuse a copy out of another address space; there the
// qualifier is left out.)
#if defined(__HIP_DEVICE_COMPILE__)
#define MH_GLOBAL __attribute__((address_space(1)))
#else
#define MH_GLOBAL
#endif
template <class T>
__device__ __forceinline__ const MH_GLOBAL T* in_global(const T* p) {
    return (const MH_GLOBAL T*)p;
}

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

// Copies count values into LDS, value j from load(j), by a block of blockDim.x
// threads, each taking at most PER values: all of a thread's loads are issued
// (indices clamped into range, no branches) before any LDS store, so they are
// in flight together instead of one round trip each.
template <int PER, typename T, typename F>
__device__ __forceinline__ void stage_lds(T* s, int64_t count, F load) {
    if (count <= 0) return;
    T v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int64_t j = threadIdx.x + (int64_t)q * blockDim.x;
        v[q] = load(j < count ? j : count - 1);
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int64_t j = threadIdx.x + (int64_t)q * blockDim.x;
        if (j < count) s[j] = v[q];
    }
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

// ------------------------------------------------------------------ logarithms
// Natural logarithm for the sweep's two per-step logs, written out from the
// series log(m) = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...), s = (m - 1)/(m + 1),
// after the reduction x = m 2^k with m in [sqrt(1/2), sqrt(2)), where
// |s| <= 0.1716 and ten odd terms beyond s leave a truncation below 2^-55
// relative.  About 35 instructions against ~90 for the library's double-double
// evaluation; the error stays within a few ulp, far inside the 1e-12 relative
// margin that the comparisons of the method are checked to.
__device__ __forceinline__ double log_reduced(double m, int k) {
    const double f = m - 1.0;  // exact for m in [1/2, 2]
    const double d = 2.0 + f;
    // s = f / d: hardware reciprocal, two Newton steps, one residual correction
    double y = __builtin_amdgcn_rcp(d);
    y = fma(fma(-d, y, 1.0), y, y);
    y = fma(fma(-d, y, 1.0), y, y);
    double sv = f * y;
    sv = fma(fma(-sv, d, f), y, sv);
    const double z = sv * sv;
    double p = 1.0 / 21.0;
    p = fma_vop3(p, z, 1.0 / 19.0);
    p = fma_vop3(p, z, 1.0 / 17.0);
    p = fma_vop3(p, z, 1.0 / 15.0);
    p = fma_vop3(p, z, 1.0 / 13.0);
    p = fma_vop3(p, z, 1.0 / 11.0);
    p = fma_vop3(p, z, 1.0 / 9.0);
    p = fma_vop3(p, z, 1.0 / 7.0);
    p = fma_vop3(p, z, 1.0 / 5.0);
    p = fma_vop3(p, z, 1.0 / 3.0);
    const double s2 = sv + sv;
    const double lm = fma(s2, z * p, s2);
    // k ln2 in two parts: the high part has trailing zeros, so k * hi is exact
    constexpr double kLn2Hi = 0x1.62e42fefa3800p-1;
    constexpr double kLn2Lo = 0x1.ef35793c76730p-45;
    const double kd = (double)k;
    return fma(kd, kLn2Hi, fma(kd, kLn2Lo, lm));
}

// log(x) for finite x > 0 (normal).
__device__ __forceinline__ double log_fast(double x) {
    double m = __builtin_amdgcn_frexp_mant(x);  // [1/2, 1)
    int k = __builtin_amdgcn_frexp_exp(x);
    if (m < 0.70710678118654752440) {
        m += m;
        --k;
    }
    return log_reduced(m, k);
}

// log(1 + t) for finite t > -1 (1 + t rounded to a normal number): log of
// u = 1 + t rounded, plus the rounding error c = t - (u - 1) divided by u (c
// is exact for |t| <= 1, Fast2Sum; for larger t, c / u is far below an ulp of
// log u).
__device__ __forceinline__ double log1p_fast(double t) {
    // |t| < 2^-27: t - t^2/2 is log1p(t) to within t^3/3 < 2^-54 |t|, one
    // rounding (below, 1 + t would cancel against log u for negative t)
    if (fabs(t) < 0x1.0p-27) return fma(-0.5 * t, t, t);
    const double u = 1.0 + t;
    const double c = t - (u - 1.0);
    double r = __builtin_amdgcn_rcp(u);
    r = fma(fma(-u, r, 1.0), r, r);
    return fma(c, r, log_fast(u));
}

// Device status word: the first error wins.
__device__ __forceinline__ void raise_status(int32_t* status, int32_t code) {
    if (status) atomicCAS(status, 0, code);
}

}  // namespace mh

// Expected degree / strength (Sec. 2.2, 2.5) and its adjoint, O(n^2) in
// binary64.  Each wave owns kRows rows; its lanes stride over the columns, so
// every column value loaded from cache is used kRows times, and each row's
// partial sums are combined across the 64 lanes in a fixed order at the end
// (deterministic, error about (n/64) ulp instead of n ulp).
#include <cfloat>
#include "mh_common.hpp"
#include "mh_internal.hpp"

namespace mh {

namespace {

constexpr int kThreads = 256;
constexpr int kWavesPerBlock = kThreads / kWave;
constexpr int kRows = 4;
constexpr int kRowsPerBlock = kWavesPerBlock * kRows;

// 1/d for d > 0 from the hardware reciprocal refined by two Newton-Raphson
// steps (about 1 ulp).  A quotient n/d becomes n times it, and the quotients
// of one pair share their denominator, so one reciprocal replaces up to five
// divisions.  From d = 2^1000 on, d is scaled by 2^-100 around the reciprocal
// so that the hardware estimate stays in the normal range; that path is taken
// by whole waves, only when one of their lanes needs it.
__device__ __forceinline__ double rcp_refined(double d) {
    if (__builtin_expect(__any(d >= 0x1.0p1000), 0)) {
        const double s = d < 0x1.0p1000 ? 1.0 : 0x1.0p-100;
        return newton_rcp(d * s) * s;
    }
    return newton_rcp(d);
}

template <bool WEIGHTED>
__global__ __launch_bounds__(kThreads) void k_expdeg_fwd(const double* __restrict__ x, const double* __restrict__ y,
                                                         const double* __restrict__ mult, int64_t n,
                                                         double* __restrict__ k, double* __restrict__ s) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i0 = ((int64_t)blockIdx.x * kWavesPerBlock + wave) * kRows;
    if (i0 >= n) return;
    double xi[kRows], yi[kRows], ak[kRows], as[kRows];
    int64_t ii[kRows];
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
        ii[q] = i0 + q;
        const bool ok = ii[q] < n;
        xi[q] = ok ? x[ii[q]] : 0.0;
        yi[q] = (WEIGHTED && ok) ? y[ii[q]] : 0.0;
        ak[q] = 0.0;
        as[q] = 0.0;
    }
    for (int64_t j = lane; j < n; j += kWave) {
        const double xj = x[j];
        const double yj = WEIGHTED ? y[j] : 0.0;
        const double mj = mult ? mult[j] : 1.0;
#pragma unroll
        for (int q = 0; q < kRows; ++q) {
            // straight-line code for every pair: a is clamped to the largest
            // finite double, so that every term is finite and a pair of weight
            // zero (the self-pair of a class of one, whose product alone may
            // overflow) adds an exact zero; rows past n have x = 0 and are
            // never stored
            const double wgt = (j == ii[q]) ? mj - 1.0 : mj;
            const double a = fmin(xi[q] * xj, DBL_MAX);
            if (WEIGHTED) {
                const double b = yi[q] * yj;
                const double ab = a * b;
                // p = ab / D and e = p / (1 - b) from one reciprocal of
                // D (1 - b), which is at least (1 - b)^2 >= 2^-106
                const double ob = 1.0 - b;
                const double e = ab * rcp_refined((1.0 - b + ab) * ob);
                const double p = e * ob;
                ak[q] += wgt * p;
                as[q] += wgt * e;
            } else {
                const double p = a * rcp_refined(1.0 + a);
                ak[q] += wgt * p;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
        const double tk = wave_sum(ak[q]);
        const double ts = WEIGHTED ? wave_sum(as[q]) : 0.0;
        if (lane == 0 && ii[q] < n) {
            k[ii[q]] = tk;
            if (WEIGHTED && s) s[ii[q]] = ts;
        }
    }
}

// dL/dx_d = sum_{c != d} [(gk_d m_c + m_d gk_c) dp/da + (gs_d m_c + m_d gs_c) de/da] x_c
//         + 2 (m_d - 1) [gk_d dp/da + gs_d de/da]_(d,d) x_d            (and likewise for y)
// with a = x_d x_c, b = y_d y_c, D = 1 - b + ab:
//   dp/da = b(1-b)/D^2, dp/db = a/D^2, de/da = b/D^2, de/db = a/(D^2 (1-b)) + ab/(D (1-b)^2);
//   unweighted: dp/da = 1/(1+a)^2.
template <bool WEIGHTED>
__global__ __launch_bounds__(kThreads) void k_expdeg_bwd(const double* __restrict__ x, const double* __restrict__ y,
                                                         const double* __restrict__ mult, int64_t n,
                                                         const double* __restrict__ gk, const double* __restrict__ gs,
                                                         double* __restrict__ gx, double* __restrict__ gy) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t d0 = ((int64_t)blockIdx.x * kWavesPerBlock + wave) * kRows;
    if (d0 >= n) return;
    double xd[kRows], yd[kRows], md[kRows], gkd[kRows], gsd[kRows], ax[kRows], ay[kRows], kdiag[kRows],
        sdiag[kRows];
    int64_t dd[kRows];
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
        dd[q] = d0 + q;
        const bool ok = dd[q] < n;
        xd[q] = ok ? x[dd[q]] : 0.0;
        yd[q] = (WEIGHTED && ok) ? y[dd[q]] : 0.0;
        md[q] = ok ? (mult ? mult[dd[q]] : 1.0) : 0.0;
        gkd[q] = ok ? gk[dd[q]] : 0.0;
        gsd[q] = (WEIGHTED && ok) ? gs[dd[q]] : 0.0;
        ax[q] = 0.0;
        ay[q] = 0.0;
        kdiag[q] = 2.0 * (md[q] - 1.0) * gkd[q];
        sdiag[q] = 2.0 * (md[q] - 1.0) * gsd[q];
    }
    for (int64_t c = lane; c < n; c += kWave) {
        const double xc = x[c];
        const double yc = WEIGHTED ? y[c] : 0.0;
        const double mc = mult ? mult[c] : 1.0;
        const double gkc = gk[c];
        const double gsc = WEIGHTED ? gs[c] : 0.0;
#pragma unroll
        for (int q = 0; q < kRows; ++q) {
            // straight-line as in the forward pass (a clamped, every term
            // finite, zero factors add exact zeros)
            const bool self = c == dd[q];
            const double fk = self ? kdiag[q] : fma(gkd[q], mc, md[q] * gkc);
            const double fs = WEIGHTED ? (self ? sdiag[q] : fma(gsd[q], mc, md[q] * gsc)) : 0.0;
            const double a = fmin(xd[q] * xc, DBL_MAX);
            if (WEIGHTED) {
                const double b = yd[q] * yc;
                const double ob = 1.0 - b;
                const double D = fma(a, b, ob);
                const double r = rcp_refined(D * ob);
                const double iD = ob * r, iob = D * r;
                // x part: b / D^2 (fk (1 - b) + fs);
                // y part: (a / D) (fk / D + fs / (1 - b) (1 / D + b / (1 - b))),
                // grouped so that no factor underflows before the small ones
                // multiply in
                ax[q] = fma(b * (iD * iD) * xc, fma(fk, ob, fs), ax[q]);
                ay[q] = fma(a * iD * yc, fma(fs * iob, fma(b, iob, iD), fk * iD), ay[q]);
            } else {
                const double i1a = rcp_refined(1.0 + a);
                ax[q] = fma(fk * xc, i1a * i1a, ax[q]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
        const double tx = wave_sum(ax[q]);
        const double ty = WEIGHTED ? wave_sum(ay[q]) : 0.0;
        if (lane == 0 && dd[q] < n) {
            gx[dd[q]] = tx;
            if (WEIGHTED && gy) gy[dd[q]] = ty;
        }
    }
}

}  // namespace

}  // namespace mh

extern "C" {

mh_status mh_expected_degree_fwd(const double* x, const double* y, const double* mult, int64_t n, double* k,
                                 double* s, hipStream_t stream) {
    using namespace mh;
    if (n < 0) return MH_EINVAL;
    if (n == 0) return MH_OK;
    if (!x || !k || (y && !s)) return MH_EINVAL;
    const unsigned grid = (unsigned)((n + kRowsPerBlock - 1) / kRowsPerBlock);
    if (y)
        hipLaunchKernelGGL(k_expdeg_fwd<true>, dim3(grid), dim3(kThreads), 0, stream, x, y, mult, n, k, s);
    else
        hipLaunchKernelGGL(k_expdeg_fwd<false>, dim3(grid), dim3(kThreads), 0, stream, x, y, mult, n, k, s);
    MH_HIP_TRY(hipGetLastError());
    return MH_OK;
}

mh_status mh_expected_degree_bwd(const double* x, const double* y, const double* mult, int64_t n, const double* gk,
                                 const double* gs, double* gx, double* gy, hipStream_t stream) {
    using namespace mh;
    if (n < 0) return MH_EINVAL;
    if (n == 0) return MH_OK;
    if (!x || !gk || !gx || (y && (!gs || !gy))) return MH_EINVAL;
    const unsigned grid = (unsigned)((n + kRowsPerBlock - 1) / kRowsPerBlock);
    if (y)
        hipLaunchKernelGGL(k_expdeg_bwd<true>, dim3(grid), dim3(kThreads), 0, stream, x, y, mult, n, gk, gs, gx, gy);
    else
        hipLaunchKernelGGL(k_expdeg_bwd<false>, dim3(grid), dim3(kThreads), 0, stream, x, y, mult, n, gk, gs, gx, gy);
    MH_HIP_TRY(hipGetLastError());
    return MH_OK;
}

}  // extern "C"

/*
 * mh.h -- C-ABI of the MI355X sampler for the maximum-entropy configuration
 * models (Li, Wang, Kojaku, "Fast unbiased sampling of networks with given
 * expected degrees and strengths", arXiv:2509.13230).
 *
 * Models (multiplicative parameters x_i = exp(-alpha_i), y_i = exp(-beta_i)):
 *   unweighted (UBCM, Sec. 2.2):  p_ij = x_i x_j / (1 + x_i x_j)
 *   weighted   (UECM, Sec. 2.5):  p_ij = t / (1 - y_i y_j + t),  t = (x_i y_i)(x_j y_j),
 *                                 P(w | w > 0) = b^(w-1) (1 - b),  b = y_i y_j
 *
 * Conventions for every entry point:
 *   - Pointers named without a _host suffix are device pointers (HIP global
 *     memory) usable on `stream`; *_host pointers are host memory.
 *   - The caller owns every buffer, including the workspace; the library
 *     allocates no memory and keeps no state between calls.  Calls on
 *     different streams with different workspaces may run concurrently.
 *   - Node ids are int32 (n <= 2^31 - 1); counts are int64.
 *   - Parameters must be finite with x >= 0, y >= 0; (max z)^2 must be finite
 *     (z = x, or z = x*y weighted); weighted models need y_(1) y_(2) < 1 (the
 *     product of the two largest y).  Violations return MH_EINVAL.
 *   - Samplers are synchronous on return (they read the edge count back);
 *     mh_order, mh_bound, mh_plan_counts and the expected-degree calls are
 *     asynchronous on `stream`.
 *   - Randomness is counter-based (Philox4x32-10, key = seed), so a call is a
 *     pure function of its inputs: a retry after MH_ECAPACITY returns the same
 *     edge multiset.
 */
#ifndef MH_H
#define MH_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MH_OK = 0,
    MH_EINVAL = -1,     /* invalid parameters or arguments */
    MH_ECAPACITY = -2,  /* output buffer too small; *n_edges_host holds the required count */
    MH_EHIP = -3,       /* a HIP runtime call failed */
    MH_EWORKSPACE = -4  /* workspace missing or smaller than mh_workspace_bytes() */
} mh_status;

/* Plan of the sweep.  A row's columns are cut into segments, each swept by its
 * own chain that restarts with the proposal probability of the column before
 * the segment (exact: that probability bounds every later column of the row,
 * Sec. 2.3).  seg_work = target number of candidates per segment; 0 = one
 * segment per row, which is the sequential algorithm as the paper states it.
 * The rule (identical in the CPU oracle):
 *   J  = first column j > r with z_r z_j < c_r (c_r = 1 unweighted): the range
 *        (r, J) is cut every seg_work columns;
 *   Q(z) = floor(z 2^32) (2^32 for z >= 1), P = prefix sums of Q over ranks;
 *   m  = floor((seg_work c_r / z_r) 2^32) clamped to [1, 2^62];
 *   [J, n) is cut where P[j] - P[J] first reaches k m, k = 1, 2, ...       */
typedef struct {
    int32_t seg_work;
    uint32_t flags; /* reserved, must be 0 */
    /* Optional stage timing: NULL, or an array of MH_STAGE_EVENTS events made
     * by the caller (hipEventCreate).  The samplers record them on `stream` at
     * the start, after the order step, after the bound and plan steps, and after
     * the sweep.  Recording adds no synchronisation. */
    hipEvent_t* stage_events;
} mh_plan_params;

#define MH_STAGE_EVENTS 4

typedef struct {
    int64_t steps;       /* skip draws, including the draw that ends each segment */
    int64_t proposals;   /* candidates evaluated */
    int64_t accepts;     /* edges accepted (may exceed capacity) */
    int64_t segments;    /* non-empty segments swept */
    int64_t saturated_w; /* weights clamped at INT32_MAX */
    int64_t n_edges;     /* same as accepts */
} mh_stats;

/* Bytes of workspace the sampler needs for n nodes (weighted != 0: UECM). */
size_t mh_workspace_bytes(int64_t n, int weighted, const mh_plan_params* plan);

/* Sample one network from the unweighted model (Sec. 2.4).
 *   x[n]          parameters, device, float64.
 *   seed, replica Philox key and counter word: different replicas are
 *                 independent samples.
 *   plan          NULL = {seg_work = 32}.
 *   src, dst      device int32[capacity]: edge endpoints (src has the larger
 *                 x; each undirected edge once, no self-loops; order
 *                 unspecified).
 *   n_edges_host  host: number of edges of the sample (even when it exceeds
 *                 capacity; then MH_ECAPACITY is returned and only some edges
 *                 were written).
 *   workspace     device, >= mh_workspace_bytes(n, 0, plan) bytes, 256-aligned.
 *   stats_host    optional host counters (NULL skips their collection). */
mh_status mh_sample_unweighted(const double* x, int64_t n, uint64_t seed, uint32_t replica,
                               const mh_plan_params* plan, int32_t* src, int32_t* dst,
                               int64_t capacity, int64_t* n_edges_host, void* workspace,
                               size_t ws_bytes, mh_stats* stats_host, hipStream_t stream);

/* Sample one network from the weighted model (Sec. 2.5, Alg. 1): as above,
 * plus y[n] (device float64) and w (device int32[capacity]) for the weights
 * (geometric, >= 1; values beyond INT32_MAX are clamped and counted). */
mh_status mh_sample_weighted(const double* x, const double* y, int64_t n, uint64_t seed,
                             uint32_t replica, const mh_plan_params* plan, int32_t* src,
                             int32_t* dst, int32_t* w, int64_t capacity, int64_t* n_edges_host,
                             void* workspace, size_t ws_bytes, mh_stats* stats_host,
                             hipStream_t stream);

/* Brute-force sampler (Sec. 2.2): every pair i < j with i in [row_begin,
 * row_end) is an edge with probability p_ij, one Philox block per pair.
 * y == NULL selects the unweighted model (w may be NULL then).  Edges are
 * (src = i, dst = j), order unspecified. */
size_t mh_bruteforce_workspace_bytes(int64_t n);
mh_status mh_sample_bruteforce(const double* x, const double* y, int64_t n, uint64_t seed,
                               uint32_t replica, int64_t row_begin, int64_t row_end,
                               int32_t* src, int32_t* dst, int32_t* w, int64_t capacity,
                               int64_t* n_edges_host, void* workspace, size_t ws_bytes,
                               hipStream_t stream);

/* Node order (Sec. 2.4 step (i); Alg. 1): stable sort of node ids by z
 * descending (z = x, or x*y when y != NULL), ties by ascending id.
 * Outputs (device): perm[n] (perm[r] = id at rank r), zs[n] = z[perm],
 * ys[n] = y[perm] (ignored when y == NULL).  Workspace as for the sampler.
 * Invalid parameters are reported through *status_dev (int32, device, set to
 * MH_EINVAL, never cleared; may be NULL). */
mh_status mh_order(const double* x, const double* y, int64_t n, int32_t* perm, double* zs,
                   double* ys, int32_t* status_dev, void* workspace, size_t ws_bytes,
                   hipStream_t stream);

/* Bound of Sec. 2.5 (beta_min over the unprocessed nodes): c[r] = 1 - Y_r with
 * Y_r the product of the two largest ys over ranks r..n-1 (Y_{n-1} = 0).
 * ys, c: device float64[n] by rank. */
size_t mh_bound_workspace_bytes(int64_t n);
mh_status mh_bound(const double* ys, int64_t n, double* c, void* workspace, size_t ws_bytes,
                   hipStream_t stream);

/* Segment counts of the plan rule above: nseg[r] for each rank (0 for the last
 * rank and for rows with z_r = 0).  zs sorted descending; c may be NULL (all 1). */
size_t mh_plan_workspace_bytes(int64_t n);
mh_status mh_plan_counts(const double* zs, const double* c, int64_t n, int32_t seg_work,
                         int32_t* nseg, void* workspace, size_t ws_bytes, hipStream_t stream);

/* Expected degree and strength (Sec. 2.2, 2.5): k_i = sum_{j != i} p_ij,
 * s_i = sum_{j != i} p_ij / (1 - y_i y_j).  With class multiplicities mult
 * (device float64[n], NULL = all 1): k_c = sum_{c' != c} m_c' p_cc' + (m_c - 1) p_cc.
 * y == NULL: unweighted (s ignored).  float64 terms, float64 accumulation. */
mh_status mh_expected_degree_fwd(const double* x, const double* y, const double* mult, int64_t n,
                                 double* k, double* s, hipStream_t stream);

/* Adjoint: gx = d(sum gk.k + gs.s)/dx, gy likewise (gs, gy ignored unweighted). */
mh_status mh_expected_degree_bwd(const double* x, const double* y, const double* mult, int64_t n,
                                 const double* gk, const double* gs, double* gx, double* gy,
                                 hipStream_t stream);

const char* mh_status_string(mh_status s);

#ifdef __cplusplus
}
#endif
#endif

/*
 * CPU oracle for the maximum-entropy configuration-model samplers.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this code: it is used by the test-suite, by the smoke check and by the
 * benchmark's CPU-baseline leg.  It shares no code, header, table or helper
 * with the HIP library; it is written from the paper (Secs. 2.2-2.5, Alg. 1)
 * and from the published definition of Philox4x32-10 (Salmon, Moraes, Dror,
 * Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).
 *
 * Plain, slow and sequential on purpose.  IEEE binary64, round to nearest,
 * compiled without floating-point contraction or fast-math.
 */
#ifndef MH_ORACLE_H
#define MH_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define MHO_OK 0
#define MHO_EINVAL (-1)
#define MHO_ECAPACITY (-2)

typedef struct {
    int64_t steps;       /* Philox draws that drive a skip (includes the draw that ends a segment) */
    int64_t proposals;   /* candidates evaluated */
    int64_t accepts;     /* edges emitted */
    int64_t segments;    /* non-empty segments swept */
    int64_t saturated_w; /* weights clamped at INT32_MAX */
    int64_t near_ties;   /* comparisons within 1e-12 (relative) of their threshold */
} mho_stats;

/* Philox4x32-10 block: out = Philox(ctr, key). */
void mho_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Uniform in (0, 1] with 53 random bits: (((a << 21) | (b >> 11)) + 1) * 2^-53. */
double mho_u53(uint32_t a, uint32_t b);

/* The sampler's skip before flooring: d = -log(u1) / log1p(tq / c), so that
   L = floor(d) is geometric with P(L = l) = (1 - q)^l q, q = tq / (c + tq)
   (c = 1 for the unweighted model).  The sampler calls exactly this; the
   array form applies it to u1[0..n). */
double mho_skip_real(double u1, double tq, double c);
void mho_skip_reals(const double* u1, int64_t n, double tq, double c, double* d);

/* Node order: stable sort of ids by z descending, ties by id ascending. */
int mho_order(const double* z, int64_t n, int32_t* perm);

/* Suffix bound: c[r] = 1 - Y_r, Y_r = product of the two largest ys over ranks r..n-1
   (Y_{n-1} = 0).  ys is indexed by rank. */
int mho_bound(const double* ys, int64_t n, double* c);

/* Segment plan of the sweep.  nseg[r] = number of segments of row r (by rank).
   seg_work = 0 means one segment per row (the sequential algorithm as printed). */
int mho_plan_counts(const double* zs, const double* c, int64_t n, int32_t seg_work, int32_t* nseg);
/* Column ranges [a_k, b_k) of row r's segments, k = 0..nseg[r]-1.  Returns the count. */
int64_t mho_plan_row(const double* zs, const double* c, int64_t n, int32_t seg_work, int64_t r,
                     int64_t* a, int64_t* b, int64_t cap);

/* Miller-Hagberg-style sampler.  y == NULL selects the unweighted model (UBCM),
   otherwise the weighted one (UECM) and w receives the weights.  Edges are
   written in canonical order (row rank, then column rank) as (src, dst[, w]) with
   src the endpoint of larger z.  Returns the number of edges; if it exceeds
   capacity, only the first `capacity` are written.  Negative = error code.
   tie_rows (optional) receives the ids of source nodes whose rows contain a
   near-tie comparison (at most tie_cap of them). */
int64_t mho_sample_mh(const double* x, const double* y, int64_t n, uint64_t seed, uint32_t replica,
                      int32_t seg_work, int32_t* src, int32_t* dst, int32_t* w, int64_t capacity,
                      mho_stats* stats, int32_t* tie_rows, int64_t tie_cap, int64_t* n_tie_rows);

/* Miller-Hagberg sampler of the Chung-Lu model (Sec. 2.3, the comparison model
   of Sec. 2.1): p_ij = min(w_i w_j, 1) with w_i = k_i / sqrt(2M).  The same
   order, plan, counters and chain as mho_sample_mh, with proposal
   q = min(t_q, 1), skip -log U1 / -log1p(-t_q) (0 when t_q >= 1) and
   acceptance U2 * q < min(t, 1). */
int64_t mho_sample_chung_lu(const double* w, int64_t n, uint64_t seed, uint32_t replica, int32_t seg_work,
                            int32_t* src, int32_t* dst, int64_t capacity, mho_stats* stats, int32_t* tie_rows,
                            int64_t tie_cap, int64_t* n_tie_rows);

/* Triangles of a simple undirected graph (edge list, each edge once, either
   orientation, ids < n): unordered triples whose three pairs are edges. */
int64_t mho_count_triangles(const int32_t* src, const int32_t* dst, int64_t m, int64_t n);

/* Bipartite / directed sampler (Sec. 2.6).  Rows are the "+" set (xr, yr, nr),
   columns the "-" set (xc, yc, nc), each sorted by its own z descending (ties
   by id); every row sweeps all columns; yr == NULL selects the unweighted
   model (then yc is ignored).  exclude_self: a candidate whose column id equals
   the row id is never accepted (directed networks without self-loops, both
   sets indexing the same nodes).  Edges are (row id, column id[, w]). */
int64_t mho_sample_bipartite(const double* xr, const double* yr, int64_t nr, const double* xc, const double* yc,
                             int64_t nc, int exclude_self, uint64_t seed, uint32_t replica, int32_t seg_work,
                             int32_t* src, int32_t* dst, int32_t* w, int64_t capacity, mho_stats* stats,
                             int32_t* tie_rows, int64_t tie_cap, int64_t* n_tie_rows);
/* Column ranges of one bipartite row with value s = z_r and bound c (1 for the
   unweighted model) over the sorted column values zcs.  Returns the count. */
int64_t mho_plan_row_bipartite(const double* zcs, int64_t nc, double s, double c, int32_t seg_work,
                               int64_t* a, int64_t* b, int64_t cap);
/* Brute force for the bipartite / directed model: every (row i, column j) pair,
   counter (j, i, replica, 0xFFFFFFFE). */
int64_t mho_sample_bipartite_bf(const double* xr, const double* yr, int64_t nr, const double* xc,
                                const double* yc, int64_t nc, int exclude_self, uint64_t seed, uint32_t replica,
                                int32_t* src, int32_t* dst, int32_t* w, int64_t capacity);

/* Brute-force Bernoulli sampler over pairs i<j with i in [row_begin, row_end),
   j in (i, n).  Edges in (i, j) lexicographic order, src = i, dst = j. */
int64_t mho_sample_bf(const double* x, const double* y, int64_t n, uint64_t seed, uint32_t replica,
                      int64_t row_begin, int64_t row_end, int32_t* src, int32_t* dst, int32_t* w,
                      int64_t capacity, int64_t* n_near_ties);

/* Expected degree k_i = sum_{j != i} p_ij and strength s_i = sum_{j != i} p_ij/(1 - y_i y_j)
   for the listed rows (rows == NULL: all n).  mult (optional) gives the multiplicity of
   each entry (class compression).  Neumaier-compensated binary64 sums. */
int mho_expected_degree(const double* x, const double* y, const double* mult, int64_t n,
                        const int64_t* rows, int64_t n_rows, double* k, double* s);

/* Gradient of L = sum_i gk_i k_i + gs_i s_i with respect to x (and y). */
int mho_expected_degree_grad(const double* x, const double* y, const double* mult, int64_t n,
                             const double* gk, const double* gs, double* gx, double* gy);

#ifdef __cplusplus
}
#endif
#endif

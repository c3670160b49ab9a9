/*
 * CPU oracle for Miller-Hagberg-style sampling of the maximum-entropy
 * configuration models (UBCM, Sec. 2.2/2.4; UECM, Sec. 2.5 and Alg. 1).
 *
 * TEST INFRASTRUCTURE ONLY -- see mh_oracle.h.  Written for a reader holding
 * the paper: each function names the passage it follows.  Parameters are the
 * multiplicative ones, x_i = exp(-alpha_i) and y_i = exp(-beta_i), so that
 *   UBCM  p_ij = x_i x_j / (1 + x_i x_j)                         (Sec. 2.2)
 *   UECM  p_ij = t / (1 - y_i y_j + t),  t = x_i y_i x_j y_j      (Sec. 2.5)
 *         P(w | w > 0) = b^(w-1) (1 - b),  b = y_i y_j             (Sec. 2.5)
 *   bound p^_ij = t / (1 - Y + t),  Y = exp(-beta_min)            (Sec. 2.5)
 * Sorting ascending alpha (or alpha + beta) is sorting descending x (or x*y).
 */
#include "mh_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ Philox */
/* Philox4x32 with 10 rounds, from its published definition (Salmon et al.,
   SC'11, Sec. 3.3): each round multiplies counter words 0 and 2 by two fixed
   odd constants, swaps the halves of the 64-bit products into place and xors
   in the other two counter words and the round key; the key is bumped by two
   Weyl constants (golden ratio and sqrt(3) - 1, in 32-bit fixed point)
   between rounds. */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u;
static const uint32_t PHILOX_W1 = 0xBB67AE85u;

void mho_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t prod0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double mho_u53(uint32_t a, uint32_t b) {
    uint64_t m = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
    return (double)(m + 1u) * 0x1.0p-53;
}

/* ------------------------------------------------------------------ order */
/* Step (i) of Sec. 2.4 and the first line of Alg. 1: visit nodes in ascending
   alpha (UBCM) or ascending alpha + beta (UECM), i.e. descending x or x*y.
   Ties, which the paper leaves open, go by ascending node id. */
static const double* g_sort_key;

static int cmp_desc_then_id(const void* pa, const void* pb) {
    int32_t a = *(const int32_t*)pa, b = *(const int32_t*)pb;
    double za = g_sort_key[a], zb = g_sort_key[b];
    if (za > zb) return -1;
    if (za < zb) return 1;
    return (a > b) - (a < b);
}

int mho_order(const double* z, int64_t n, int32_t* perm) {
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    g_sort_key = z;
    qsort(perm, (size_t)n, sizeof(int32_t), cmp_desc_then_id);
    return MHO_OK;
}

/* ------------------------------------------------------------------ bound */
/* beta_min over the unprocessed nodes (Sec. 2.5): the smallest sum of two
   betas among ranks r..n-1, i.e. Y_r = exp(-beta_min) = product of the two
   largest y there.  The focal node r is one of the unprocessed nodes. */
int mho_bound(const double* ys, int64_t n, double* c) {
    double y1 = -1.0, y2 = -1.0; /* largest, second largest so far (from the end) */
    for (int64_t r = n - 1; r >= 0; --r) {
        double v = ys[r];
        if (v > y1) { y2 = y1; y1 = v; }
        else if (v > y2) { y2 = v; }
        double Y = (y2 < 0.0) ? 0.0 : y1 * y2;
        c[r] = 1.0 - Y;
    }
    return MHO_OK;
}

/* ------------------------------------------------------------------ plan */
/* Segmentation of a row into column ranges (not in the paper; a restart of the
   chain at column a with proposal probability taken at column a-1 is exact
   because that probability bounds every later column of the row).
   Rule, for row r with s = zs[r] and c = c[r] (c = 1 unweighted):
     J      = first column j > r with s*zs[j] < c (or n): proposals are likely
              on (r, J), so that range is cut every seg_work columns;
     mass   Q(z) = floor(z * 2^32) (2^32 if z >= 1), prefix sums P over ranks;
     m      = floor((seg_work * c / s) * 2^32), clamped to [1, 2^62];
     [J, n) is cut where the prefix mass from J crosses multiples of m. */
static uint64_t mass_q(double z) {
    if (z >= 1.0) return (uint64_t)1 << 32;
    return (uint64_t)(z * 4294967296.0);
}

typedef struct {
    int64_t n;
    const double* zs;
    const double* c; /* NULL: all ones */
    int32_t seg_work;
    uint64_t* P;     /* n + 1 prefix masses (NULL if seg_work == 0) */
} plan_ctx;

static double cval(const plan_ctx* pc, int64_t r) { return pc->c ? pc->c[r] : 1.0; }

static int plan_init(plan_ctx* pc, const double* zs, const double* c, int64_t n, int32_t seg_work) {
    pc->n = n; pc->zs = zs; pc->c = c; pc->seg_work = seg_work; pc->P = NULL;
    if (seg_work > 0) {
        pc->P = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n + 1));
        if (!pc->P) return MHO_EINVAL;
        pc->P[0] = 0;
        for (int64_t j = 0; j < n; ++j) pc->P[j + 1] = pc->P[j] + mass_q(zs[j]);
    }
    return MHO_OK;
}

static void plan_free(plan_ctx* pc) { free(pc->P); pc->P = NULL; }

/* first j in [lo, hi] with pred(j) true, pred monotone false..true */
static int64_t first_below(const plan_ctx* pc, double s, double c, int64_t lo, int64_t hi) {
    /* pred(j) = (j == n) || s*zs[j] < c */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int pred = (mid == pc->n) || (s * pc->zs[mid] < c);
        if (pred) hi = mid; else lo = mid + 1;
    }
    return lo;
}

static int64_t lower_bound_mass(const plan_ctx* pc, int64_t lo, int64_t hi, uint64_t v) {
    /* first j in [lo, hi] with P[j] >= v (hi if none) */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (pc->P[mid] >= v) hi = mid; else lo = mid + 1;
    }
    return lo;
}

typedef struct { int64_t J, nd, ns; uint64_t m; } row_plan;

static row_plan plan_row_info(const plan_ctx* pc, int64_t r) {
    row_plan rp = {0, 0, 0, 0};
    int64_t n = pc->n;
    double s = pc->zs[r];
    if (r >= n - 1 || s == 0.0) return rp;
    if (pc->seg_work <= 0) { rp.J = n; rp.nd = 1; return rp; }
    double c = cval(pc, r);
    int64_t T = pc->seg_work;
    rp.J = first_below(pc, s, c, r + 1, n);
    rp.nd = (rp.J - r - 1 + T - 1) / T;
    if (rp.J < n) {
        double md = ((double)T * c / s) * 4294967296.0;
        uint64_t m;
        if (!(md < 4611686018427387904.0)) m = (uint64_t)1 << 62;
        else if (md < 1.0) m = 1;
        else m = (uint64_t)md;
        uint64_t mass = pc->P[n] - pc->P[rp.J];
        rp.m = m;
        rp.ns = (mass == 0) ? 1 : (int64_t)((mass + m - 1) / m);
    }
    return rp;
}

static void plan_segment(const plan_ctx* pc, int64_t r, const row_plan* rp, int64_t k, int64_t* a, int64_t* b) {
    int64_t n = pc->n;
    if (pc->seg_work <= 0) { *a = r + 1; *b = n; return; }
    int64_t T = pc->seg_work;
    if (k < rp->nd) {
        *a = r + 1 + k * T;
        int64_t e = r + 1 + (k + 1) * T;
        *b = e < rp->J ? e : rp->J;
        return;
    }
    int64_t kk = k - rp->nd;
    uint64_t base = pc->P[rp->J];
    *a = (kk == 0) ? rp->J : lower_bound_mass(pc, rp->J, n, base + (uint64_t)kk * rp->m);
    *b = (kk == rp->ns - 1) ? n : lower_bound_mass(pc, rp->J, n, base + (uint64_t)(kk + 1) * rp->m);
}

int mho_plan_counts(const double* zs, const double* c, int64_t n, int32_t seg_work, int32_t* nseg) {
    plan_ctx pc;
    if (plan_init(&pc, zs, c, n, seg_work) != MHO_OK) return MHO_EINVAL;
    for (int64_t r = 0; r < n; ++r) {
        row_plan rp = plan_row_info(&pc, r);
        nseg[r] = (int32_t)(rp.nd + rp.ns);
    }
    plan_free(&pc);
    return MHO_OK;
}

int64_t mho_plan_row(const double* zs, const double* c, int64_t n, int32_t seg_work, int64_t r,
                     int64_t* a, int64_t* b, int64_t cap) {
    plan_ctx pc;
    if (plan_init(&pc, zs, c, n, seg_work) != MHO_OK) return MHO_EINVAL;
    row_plan rp = plan_row_info(&pc, r);
    int64_t cnt = rp.nd + rp.ns;
    for (int64_t k = 0; k < cnt && k < cap; ++k) plan_segment(&pc, r, &rp, k, &a[k], &b[k]);
    plan_free(&pc);
    return cnt;
}

/* ------------------------------------------------------------------ checks */
static int valid_params(const double* x, const double* y, int64_t n) {
    if (n < 0 || n > 2147483647LL) return 0;
    double zmax = 0.0, y1 = 0.0, y2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double xi = x[i];
        if (!(xi >= 0.0) || !isfinite(xi)) return 0;
        double z = xi;
        if (y) {
            double yi = y[i];
            if (!(yi >= 0.0) || !isfinite(yi)) return 0;
            z = xi * yi;
            if (!isfinite(z)) return 0;
            if (yi > y1) { y2 = y1; y1 = yi; } else if (yi > y2) { y2 = yi; }
        }
        if (z > zmax) zmax = z;
    }
    if (!isfinite(zmax * zmax)) return 0;
    if (y && !(y1 * y2 < 1.0)) return 0;
    return 1;
}

static int near_int(double d) {
    double f = floor(d + 0.5);
    double tol = 1e-12 * (d > 1.0 ? d : 1.0);
    return fabs(d - f) <= tol;
}

/* The skip of Sec. 2.3 before it is floored: the next candidate lies
   L = floor(d) columns past the chain's position, where L is geometric with
   P(L = l) = (1 - q)^l q, drawn by inversion as d = log U / log(1 - q).
   The proposal probability is q = t_q / (c + t_q) (c = 1 unweighted: q is the
   true p; c = 1 - Y weighted: q is the bound), so 1 - q = c / (c + t_q) and
   -log(1 - q) = log1p(t_q / c), which stays accurate when q is near 0 or 1. */
static double skip_real(double u1, double tq, double c) {
    return -log(u1) / log1p(tq / c);
}

/* The skip of the Chung-Lu chain (Sec. 2.3): the proposal probability is
   q = min(t_q, 1) itself, so -log(1 - q) = -log1p(-t_q) for t_q < 1; at
   q = 1 every column is a candidate (L = 0). */
static double skip_real_chung_lu(double u1, double tq) {
    if (tq >= 1.0) return 0.0;
    return -log(u1) / -log1p(-tq);
}

double mho_skip_real(double u1, double tq, double c) { return skip_real(u1, tq, c); }

void mho_skip_reals(const double* u1, int64_t n, double tq, double c, double* d) {
    for (int64_t i = 0; i < n; ++i) d[i] = skip_real(u1[i], tq, c);
}

/* Weight given an edge: geometric on {1, 2, ...} with P(w) = b^(w-1)(1-b)
   (Sec. 2.5), by inversion: w = 1 + floor(log U / log b). */
static int32_t draw_weight(double u, double b, int64_t* saturated, int* tie) {
    if (b == 0.0) return 1;
    double ratio = log(u) / log(b);
    if (near_int(ratio)) *tie = 1;
    if (ratio >= 2147483646.0) { ++*saturated; return INT32_MAX; }
    return 1 + (int32_t)ratio;
}

/* ------------------------------------------------------------------ MH sampler */
/* Sequential rejection sampling (Sec. 2.3, steps (i)-(iv) of Sec. 2.4, Alg. 1).
   Per row r (descending z) and per segment [a, b) of its columns:
     the chain sits at column pos = a - 1 with proposal probability q taken there
     (q = p_rr / p^_rr at a row start);
     it skips L ~ Geometric(q) columns, L >= 0, to candidate j = pos + 1 + L, and
     stops once j passes the end of the segment;
     it accepts j with probability p_rj / q, then sets q to the probability at j
     (the true p for UBCM, the bound p^ for UECM) whether or not j was accepted.
   Randomness: one Philox block per step, counter (step, rank r, replica,
   2*segment + 0); U1 drives the skip, U2 the acceptance; a second block with
   kind 1 gives the weight.  Key = seed.
   Floating point:  L = floor(-log U1 / log1p(t_q))          (UBCM, 1-q = 1/(1+t_q))
                    L = floor(-log U1 / log1p(t_q / c))      (UECM, 1-q = c/(c+t_q))
                    accept iff U2 * t_q * (1 + t) < t * (1 + t_q)          (U2 < p/q)
                           or  U2 * t_q * (e + t) < t * (c + t_q),  e = 1 - y_r y_j. */
typedef struct {
    int32_t* src; int32_t* dst; int32_t* w; int64_t capacity; int64_t count;
} edge_sink;

static void emit(edge_sink* es, int32_t a, int32_t b, int32_t wt) {
    if (es->count < es->capacity) {
        es->src[es->count] = a;
        es->dst[es->count] = b;
        if (es->w) es->w[es->count] = wt;
    }
    ++es->count;
}

/* One node set.  chung_lu != 0 (x holds the Chung-Lu weights w_i, y NULL):
   the target is p = min(t, 1) and the proposal q = min(t_q, 1), the chain of
   the Miller-Hagberg algorithm for the Chung-Lu model (Sec. 2.3); accept iff
   U2 * q < p. */
static int64_t sample_one_set(const double* x, const double* y, int chung_lu, int64_t n, uint64_t seed,
                              uint32_t replica, int32_t seg_work, int32_t* src, int32_t* dst, int32_t* w,
                              int64_t capacity, mho_stats* stats, int32_t* tie_rows, int64_t tie_cap,
                              int64_t* n_tie_rows) {
    mho_stats st;
    memset(&st, 0, sizeof(st));
    int64_t ntr = 0;
    if (!x || !valid_params(x, y, n) || seg_work < 0) return MHO_EINVAL;
    edge_sink es = {src, dst, w, capacity, 0};
    if (n < 2) goto done;

    double* z = (double*)malloc(sizeof(double) * (size_t)n);
    int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    double* zs = (double*)malloc(sizeof(double) * (size_t)n);
    double* ys = y ? (double*)malloc(sizeof(double) * (size_t)n) : NULL;
    double* c = y ? (double*)malloc(sizeof(double) * (size_t)n) : NULL;
    for (int64_t i = 0; i < n; ++i) z[i] = y ? x[i] * y[i] : x[i];
    mho_order(z, n, perm);
    for (int64_t r = 0; r < n; ++r) {
        zs[r] = z[perm[r]];
        if (y) ys[r] = y[perm[r]];
    }
    if (y) mho_bound(ys, n, c);

    plan_ctx pc;
    plan_init(&pc, zs, c, n, seg_work);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};

    for (int64_t r = 0; r + 1 < n; ++r) {
        row_plan rp = plan_row_info(&pc, r);
        int64_t nseg = rp.nd + rp.ns;
        double s = zs[r];
        double cr = y ? c[r] : 1.0;
        int32_t id_r = perm[r];
        int row_tie = 0;
        for (int64_t g = 0; g < nseg; ++g) {
            int64_t a, b;
            plan_segment(&pc, r, &rp, g, &a, &b);
            if (a >= b) continue;
            ++st.segments;
            int64_t pos = a - 1;
            double tq = s * zs[pos];
            uint32_t step = 0;
            for (;;) {
                if (tq == 0.0) break;
                uint32_t ctr[4] = {step, (uint32_t)r, replica, (uint32_t)(g << 1)};
                uint32_t u[4];
                mho_philox4x32_10(ctr, key, u);
                ++st.steps;
                double U1 = mho_u53(u[0], u[1]);
                double U2 = mho_u53(u[2], u[3]);
                double d = chung_lu ? skip_real_chung_lu(U1, tq) : skip_real(U1, tq, cr);
                double room = (double)(b - 1 - pos);
                /* a skip of exactly 0 at q = 1 is no rounding decision */
                if (!(chung_lu && tq >= 1.0) &&
                    (near_int(d) || fabs(d - room) <= 1e-12 * (room > 1.0 ? room : 1.0)))
                    row_tie = 1;
                if (d >= room) break;
                int64_t j = pos + 1 + (int64_t)d;
                double t = s * zs[j];
                double lhs, rhs;
                if (chung_lu) {
                    lhs = U2 * (tq < 1.0 ? tq : 1.0);
                    rhs = t < 1.0 ? t : 1.0;
                } else if (y) {
                    double e = 1.0 - ys[r] * ys[j];
                    lhs = (U2 * tq) * (e + t);
                    rhs = t * (cr + tq);
                } else {
                    lhs = (U2 * tq) * (1.0 + t);
                    rhs = t * (1.0 + tq);
                }
                ++st.proposals;
                if (fabs(lhs - rhs) <= 1e-12 * rhs) row_tie = 1;
                if (lhs < rhs) {
                    int32_t wt = 0;
                    if (y) {
                        uint32_t ctr2[4] = {step, (uint32_t)r, replica, (uint32_t)((g << 1) | 1)};
                        uint32_t v[4];
                        mho_philox4x32_10(ctr2, key, v);
                        double U3 = mho_u53(v[0], v[1]);
                        wt = draw_weight(U3, ys[r] * ys[j], &st.saturated_w, &row_tie);
                    }
                    ++st.accepts;
                    emit(&es, id_r, perm[j], wt);
                }
                tq = t;
                pos = j;
                ++step;
            }
        }
        if (row_tie) {
            ++st.near_ties;
            if (tie_rows && ntr < tie_cap) tie_rows[ntr] = id_r;
            ++ntr;
        }
    }
    plan_free(&pc);
    free(z); free(perm); free(zs); free(ys); free(c);
done:
    if (stats) *stats = st;
    if (n_tie_rows) *n_tie_rows = ntr;
    return es.count;
}

int64_t mho_sample_mh(const double* x, const double* y, int64_t n, uint64_t seed, uint32_t replica,
                      int32_t seg_work, int32_t* src, int32_t* dst, int32_t* w, int64_t capacity,
                      mho_stats* stats, int32_t* tie_rows, int64_t tie_cap, int64_t* n_tie_rows) {
    return sample_one_set(x, y, 0, n, seed, replica, seg_work, src, dst, w, capacity, stats, tie_rows, tie_cap,
                          n_tie_rows);
}

int64_t mho_sample_chung_lu(const double* wgt, int64_t n, uint64_t seed, uint32_t replica, int32_t seg_work,
                            int32_t* src, int32_t* dst, int64_t capacity, mho_stats* stats, int32_t* tie_rows,
                            int64_t tie_cap, int64_t* n_tie_rows) {
    return sample_one_set(wgt, NULL, 1, n, seed, replica, seg_work, src, dst, NULL, capacity, stats, tie_rows,
                          tie_cap, n_tie_rows);
}

/* ------------------------------------------------------------------ bipartite */
/* Bipartite and directed networks (Sec. 2.6): the "+" nodes (rows) and the "-"
   nodes (columns) are sorted by their own parameters, and every "+" node sweeps
   the whole "-" list with the same skip / accept / update rule.  Readings:
   the chain of a column range [a, b) starts before column a with the proposal
   probability of column a itself (it bounds every later column); the weighted
   bound of row r is Y_r = y_r * (largest column y) (the smallest beta_+ + beta_-
   that row r can meet); the same segment rule cuts a row's column range, with
   first column 0 instead of r + 1. */
static row_plan bip_row_info(const plan_ctx* cols, double s, double c) {
    row_plan rp = {0, 0, 0, 0};
    int64_t nc = cols->n;
    if (nc == 0 || s == 0.0) return rp;
    if (cols->seg_work <= 0) { rp.J = nc; rp.nd = 1; return rp; }
    int64_t T = cols->seg_work;
    rp.J = first_below(cols, s, c, 0, nc);
    rp.nd = (rp.J + T - 1) / T;
    if (rp.J < nc) {
        double md = ((double)T * c / s) * 4294967296.0;
        uint64_t m;
        if (!(md < 4611686018427387904.0)) m = (uint64_t)1 << 62;
        else if (md < 1.0) m = 1;
        else m = (uint64_t)md;
        uint64_t mass = cols->P[nc] - cols->P[rp.J];
        rp.m = m;
        rp.ns = (mass == 0) ? 1 : (int64_t)((mass + m - 1) / m);
    }
    return rp;
}

static void bip_segment(const plan_ctx* cols, const row_plan* rp, int64_t k, int64_t* a, int64_t* b) {
    int64_t nc = cols->n;
    if (cols->seg_work <= 0) { *a = 0; *b = nc; return; }
    int64_t T = cols->seg_work;
    if (k < rp->nd) {
        *a = k * T;
        int64_t e = (k + 1) * T;
        *b = e < rp->J ? e : rp->J;
        return;
    }
    int64_t kk = k - rp->nd;
    uint64_t base = cols->P[rp->J];
    *a = (kk == 0) ? rp->J : lower_bound_mass(cols, rp->J, nc, base + (uint64_t)kk * rp->m);
    *b = (kk == rp->ns - 1) ? nc : lower_bound_mass(cols, rp->J, nc, base + (uint64_t)(kk + 1) * rp->m);
}

int64_t mho_plan_row_bipartite(const double* zcs, int64_t nc, double s, double c, int32_t seg_work,
                               int64_t* a, int64_t* b, int64_t cap) {
    plan_ctx cols;
    if (plan_init(&cols, zcs, NULL, nc, seg_work) != MHO_OK) return MHO_EINVAL;
    row_plan rp = bip_row_info(&cols, s, c);
    int64_t cnt = rp.nd + rp.ns;
    for (int64_t k = 0; k < cnt && k < cap; ++k) bip_segment(&cols, &rp, k, &a[k], &b[k]);
    plan_free(&cols);
    return cnt;
}

static int finite_nonneg(const double* v, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!(v[i] >= 0.0) || !isfinite(v[i])) return 0;
    return 1;
}

static int valid_bip(const double* xr, const double* yr, int64_t nr, const double* xc, const double* yc, int64_t nc) {
    if (nr < 0 || nc < 0 || nr > 2147483647LL || nc > 2147483647LL) return 0;
    if (!finite_nonneg(xr, nr) || !finite_nonneg(xc, nc)) return 0;
    if (yr && (!finite_nonneg(yr, nr) || !finite_nonneg(yc, nc))) return 0;
    double zr = 0.0, zc = 0.0, yrm = 0.0, ycm = 0.0;
    for (int64_t i = 0; i < nr; ++i) {
        double z = yr ? xr[i] * yr[i] : xr[i];
        if (!isfinite(z)) return 0;
        if (z > zr) zr = z;
        if (yr && yr[i] > yrm) yrm = yr[i];
    }
    for (int64_t j = 0; j < nc; ++j) {
        double z = yr ? xc[j] * yc[j] : xc[j];
        if (!isfinite(z)) return 0;
        if (z > zc) zc = z;
        if (yr && yc[j] > ycm) ycm = yc[j];
    }
    if (!isfinite(zr * zc)) return 0;
    if (yr && nr > 0 && nc > 0 && !(yrm * ycm < 1.0)) return 0;
    return 1;
}

int64_t mho_sample_bipartite(const double* xr, const double* yr, int64_t nr, const double* xc, const double* yc,
                             int64_t nc, int exclude_self, uint64_t seed, uint32_t replica, int32_t seg_work,
                             int32_t* src, int32_t* dst, int32_t* w, int64_t capacity, mho_stats* stats,
                             int32_t* tie_rows, int64_t tie_cap, int64_t* n_tie_rows) {
    mho_stats st;
    memset(&st, 0, sizeof(st));
    int64_t ntr = 0;
    if (!xr || !xc || seg_work < 0 || (yr && !yc)) return MHO_EINVAL;
    if (!valid_bip(xr, yr, nr, xc, yc, nc)) return MHO_EINVAL;
    edge_sink es = {src, dst, w, capacity, 0};
    if (nr > 0 && nc > 0) {
        double* zr = (double*)malloc(sizeof(double) * (size_t)nr);
        double* zc = (double*)malloc(sizeof(double) * (size_t)nc);
        int32_t* pr = (int32_t*)malloc(sizeof(int32_t) * (size_t)nr);
        int32_t* pcn = (int32_t*)malloc(sizeof(int32_t) * (size_t)nc);
        double* zrs = (double*)malloc(sizeof(double) * (size_t)nr);
        double* zcs = (double*)malloc(sizeof(double) * (size_t)nc);
        for (int64_t i = 0; i < nr; ++i) zr[i] = yr ? xr[i] * yr[i] : xr[i];
        for (int64_t j = 0; j < nc; ++j) zc[j] = yr ? xc[j] * yc[j] : xc[j];
        mho_order(zr, nr, pr);
        mho_order(zc, nc, pcn);
        double ymax_c = 0.0;
        for (int64_t i = 0; i < nr; ++i) zrs[i] = zr[pr[i]];
        for (int64_t j = 0; j < nc; ++j) {
            zcs[j] = zc[pcn[j]];
            if (yr && yc[j] > ymax_c) ymax_c = yc[j];
        }
        plan_ctx cols;
        plan_init(&cols, zcs, NULL, nc, seg_work);
        uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
        for (int64_t r = 0; r < nr; ++r) {
            double s = zrs[r];
            int32_t id_r = pr[r];
            double yrr = yr ? yr[id_r] : 0.0;
            double cr = yr ? 1.0 - yrr * ymax_c : 1.0;
            row_plan rp = bip_row_info(&cols, s, cr);
            int64_t nseg = rp.nd + rp.ns;
            int row_tie = 0;
            for (int64_t g = 0; g < nseg; ++g) {
                int64_t a, b;
                bip_segment(&cols, &rp, g, &a, &b);
                if (a >= b) continue;
                ++st.segments;
                int64_t pos = a - 1;
                double tq = s * zcs[a];
                uint32_t step = 0;
                for (;;) {
                    if (tq == 0.0) break;
                    uint32_t ctr[4] = {step, (uint32_t)r, replica, (uint32_t)(g << 1)};
                    uint32_t u[4];
                    mho_philox4x32_10(ctr, key, u);
                    ++st.steps;
                    double U1 = mho_u53(u[0], u[1]);
                    double U2 = mho_u53(u[2], u[3]);
                    double d = skip_real(U1, tq, cr);
                    double room = (double)(b - 1 - pos);
                    if (near_int(d) || fabs(d - room) <= 1e-12 * (room > 1.0 ? room : 1.0)) row_tie = 1;
                    if (d >= room) break;
                    int64_t j = pos + 1 + (int64_t)d;
                    double t = s * zcs[j];
                    int32_t id_j = pcn[j];
                    double lhs, rhs, bb = 0.0;
                    if (yr) {
                        bb = yrr * yc[id_j];
                        double e = 1.0 - bb;
                        lhs = (U2 * tq) * (e + t);
                        rhs = t * (cr + tq);
                    } else {
                        lhs = (U2 * tq) * (1.0 + t);
                        rhs = t * (1.0 + tq);
                    }
                    ++st.proposals;
                    if (fabs(lhs - rhs) <= 1e-12 * rhs) row_tie = 1;
                    if (lhs < rhs && !(exclude_self && id_j == id_r)) {
                        int32_t wt = 0;
                        if (yr) {
                            uint32_t ctr2[4] = {step, (uint32_t)r, replica, (uint32_t)((g << 1) | 1)};
                            uint32_t v[4];
                            mho_philox4x32_10(ctr2, key, v);
                            wt = draw_weight(mho_u53(v[0], v[1]), bb, &st.saturated_w, &row_tie);
                        }
                        ++st.accepts;
                        emit(&es, id_r, id_j, wt);
                    }
                    tq = t;
                    pos = j;
                    ++step;
                }
            }
            if (row_tie) {
                ++st.near_ties;
                if (tie_rows && ntr < tie_cap) tie_rows[ntr] = id_r;
                ++ntr;
            }
        }
        plan_free(&cols);
        free(zr); free(zc); free(pr); free(pcn); free(zrs); free(zcs);
    }
    if (stats) *stats = st;
    if (n_tie_rows) *n_tie_rows = ntr;
    return es.count;
}

int64_t mho_sample_bipartite_bf(const double* xr, const double* yr, int64_t nr, const double* xc,
                                const double* yc, int64_t nc, int exclude_self, uint64_t seed, uint32_t replica,
                                int32_t* src, int32_t* dst, int32_t* w, int64_t capacity) {
    if (!xr || !xc || (yr && !yc) || !valid_bip(xr, yr, nr, xc, yc, nc)) return MHO_EINVAL;
    edge_sink es = {src, dst, w, capacity, 0};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int64_t sat = 0;
    for (int64_t i = 0; i < nr; ++i) {
        double zi = yr ? xr[i] * yr[i] : xr[i];
        for (int64_t j = 0; j < nc; ++j) {
            if (exclude_self && i == j) continue;
            double zj = yr ? xc[j] * yc[j] : xc[j];
            double t = zi * zj;
            uint32_t ctr[4] = {(uint32_t)j, (uint32_t)i, replica, 0xFFFFFFFEu};
            uint32_t u[4];
            mho_philox4x32_10(ctr, key, u);
            double e = yr ? 1.0 - yr[i] * yc[j] : 1.0;
            if (mho_u53(u[0], u[1]) * (e + t) < t) {
                int32_t wt = 0;
                if (yr) {
                    int tie = 0;
                    wt = draw_weight(mho_u53(u[2], u[3]), yr[i] * yc[j], &sat, &tie);
                }
                emit(&es, (int32_t)i, (int32_t)j, wt);
            }
        }
    }
    return es.count;
}

/* ------------------------------------------------------------------ brute force */
/* The brute-force sampler (Sec. 2.2): every pair i < j is an edge with
   probability p_ij, independently.  One Philox block per pair, counter
   (j, i, replica, 0xFFFFFFFF): U from words 0-1 decides the edge
   (U < p_ij, written U * (1 + t) < t, or U * (e + t) < t weighted), words 2-3
   give the weight. */
int64_t mho_sample_bf(const double* x, const double* y, int64_t n, uint64_t seed, uint32_t replica,
                      int64_t row_begin, int64_t row_end, int32_t* src, int32_t* dst, int32_t* w,
                      int64_t capacity, int64_t* n_near_ties) {
    if (!x || !valid_params(x, y, n)) return MHO_EINVAL;
    if (row_begin < 0) row_begin = 0;
    if (row_end > n) row_end = n;
    edge_sink es = {src, dst, w, capacity, 0};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int64_t ties = 0, sat = 0;
    for (int64_t i = row_begin; i < row_end; ++i) {
        double zi = y ? x[i] * y[i] : x[i];
        for (int64_t j = i + 1; j < n; ++j) {
            double zj = y ? x[j] * y[j] : x[j];
            double t = zi * zj;
            uint32_t ctr[4] = {(uint32_t)j, (uint32_t)i, replica, 0xFFFFFFFFu};
            uint32_t u[4];
            mho_philox4x32_10(ctr, key, u);
            double U = mho_u53(u[0], u[1]);
            double e = y ? 1.0 - y[i] * y[j] : 1.0;
            double lhs = U * (e + t);
            if (fabs(lhs - t) <= 1e-12 * t) ++ties;
            if (lhs < t) {
                int32_t wt = 0;
                if (y) {
                    int tie = 0;
                    wt = draw_weight(mho_u53(u[2], u[3]), y[i] * y[j], &sat, &tie);
                    ties += tie;
                }
                emit(&es, (int32_t)i, (int32_t)j, wt);
            }
        }
    }
    if (n_near_ties) *n_near_ties = ties;
    return es.count;
}

/* ------------------------------------------------------------------ expected degree */
/* k_i = sum_{j != i} p_ij is the degree constraint of the maximum-likelihood
   fit (Sec. 2.2); s_i = sum_{j != i} p_ij / (1 - b_ij) is the expected strength,
   since the conditional weight law of Sec. 2.5 has mean 1/(1 - b).
   With class multiplicities m: k_c = sum_{c' != c} m_c' p_cc' + (m_c - 1) p_cc.
   Neumaier's compensated summation in binary64. */
typedef struct { double sum, comp; } nsum;

static void nsum_add(nsum* a, double v) {
    double t = a->sum + v;
    if (fabs(a->sum) >= fabs(v)) a->comp += (a->sum - t) + v;
    else a->comp += (v - t) + a->sum;
    a->sum = t;
}

static double nsum_get(const nsum* a) { return a->sum + a->comp; }

static void pair_terms(double xi, double xj, const double* y, int64_t i, int64_t j, double* p, double* e) {
    double a = xi * xj;
    if (!y) {
        *p = a / (1.0 + a);
        *e = *p;
        return;
    }
    double b = y[i] * y[j];
    double ab = a * b;
    *p = ab / (1.0 - b + ab);
    *e = *p / (1.0 - b);
}

int mho_expected_degree(const double* x, const double* y, const double* mult, int64_t n,
                        const int64_t* rows, int64_t n_rows, double* k, double* s) {
    if (!x || n < 0) return MHO_EINVAL;
    int64_t cnt = rows ? n_rows : n;
    for (int64_t q = 0; q < cnt; ++q) {
        int64_t i = rows ? rows[q] : q;
        nsum sk = {0.0, 0.0}, ss = {0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            double mj = mult ? mult[j] : 1.0;
            double wgt = (j == i) ? mj - 1.0 : mj;
            if (wgt == 0.0) continue;
            double p, e;
            pair_terms(x[i], x[j], y, i, j, &p, &e);
            nsum_add(&sk, wgt * p);
            if (y) nsum_add(&ss, wgt * e);
        }
        k[q] = nsum_get(&sk);
        if (y && s) s[q] = nsum_get(&ss);
    }
    return MHO_OK;
}

/* Gradient of L = sum_c gk_c k_c + gs_c s_c.  With a = x_i x_j, b = y_i y_j,
   D = 1 - b + ab:  dp/da = b(1-b)/D^2, dp/db = a/D^2, and for e = p/(1-b):
   de/da = b/D^2, de/db = a/(D^2 (1-b)) + ab/(D (1-b)^2).  UBCM: dp/da = 1/(1+a)^2.
   dL/dx_d = sum_{c != d} [(gk_d m_c + m_d gk_c) dp/da + (gs_d m_c + m_d gs_c) de/da] x_c
           + 2 (m_d - 1) [gk_d dp/da + gs_d de/da]_(d,d) x_d,   and likewise for y. */
int mho_expected_degree_grad(const double* x, const double* y, const double* mult, int64_t n,
                             const double* gk, const double* gs, double* gx, double* gy) {
    if (!x || !gk || !gx || n < 0) return MHO_EINVAL;
    for (int64_t d = 0; d < n; ++d) {
        double md = mult ? mult[d] : 1.0;
        nsum sx = {0.0, 0.0}, sy = {0.0, 0.0};
        for (int64_t c = 0; c < n; ++c) {
            double mc = mult ? mult[c] : 1.0;
            double a = x[d] * x[c];
            double fk, fs; /* weights of dp and de */
            if (c == d) {
                fk = 2.0 * (md - 1.0) * gk[d];
                fs = y ? 2.0 * (md - 1.0) * gs[d] : 0.0;
            } else {
                fk = gk[d] * mc + md * gk[c];
                fs = y ? gs[d] * mc + md * gs[c] : 0.0;
            }
            if (fk == 0.0 && fs == 0.0) continue;
            if (!y) {
                double dpa = 1.0 / ((1.0 + a) * (1.0 + a));
                nsum_add(&sx, fk * dpa * x[c]);
            } else {
                double b = y[d] * y[c];
                double D = 1.0 - b + a * b;
                double D2 = D * D;
                double dpa = b * (1.0 - b) / D2;
                double dpb = a / D2;
                double dea = b / D2;
                double deb = a / (D2 * (1.0 - b)) + a * b / (D * (1.0 - b) * (1.0 - b));
                nsum_add(&sx, (fk * dpa + fs * dea) * x[c]);
                nsum_add(&sy, (fk * dpb + fs * deb) * y[c]);
            }
        }
        gx[d] = nsum_get(&sx);
        if (y && gy) gy[d] = nsum_get(&sy);
    }
    return MHO_OK;
}

/* ------------------------------------------------------------------ triangles */
/* Number of triangles of a simple undirected graph given as an edge list (each
   edge once, either orientation, no self-loops), by the definition: unordered
   triples {a, b, c} whose three pairs are all edges.  Each triangle is counted
   once, at its two smallest ids a < b: the common neighbours c > b of a and b.
   Used for the triangle statistics of sampled networks (Sec. 2.1, Fig. 1B). */
static int cmp_i32(const void* pa, const void* pb) {
    int32_t a = *(const int32_t*)pa, b = *(const int32_t*)pb;
    return (a > b) - (a < b);
}

int64_t mho_count_triangles(const int32_t* src, const int32_t* dst, int64_t m, int64_t n) {
    if (m < 0 || n < 0) return -1;
    int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t* adj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    int64_t* fill = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t e = 0; e < m; ++e) {
        ++deg[src[e] + 1];
        ++deg[dst[e] + 1];
    }
    for (int64_t i = 0; i < n; ++i) deg[i + 1] += deg[i];  /* deg[i] = start of i's list */
    for (int64_t e = 0; e < m; ++e) {
        adj[deg[src[e]] + fill[src[e]]++] = dst[e];
        adj[deg[dst[e]] + fill[dst[e]]++] = src[e];
    }
    for (int64_t i = 0; i < n; ++i) qsort(adj + deg[i], (size_t)(deg[i + 1] - deg[i]), sizeof(int32_t), cmp_i32);
    int64_t tri = 0;
    for (int64_t a = 0; a < n; ++a) {
        for (int64_t p = deg[a]; p < deg[a + 1]; ++p) {
            int32_t b = adj[p];
            if (b <= a) continue;
            /* common neighbours c > b of a and b: merge the two sorted lists */
            int64_t i = deg[a], j = deg[b];
            while (i < deg[a + 1] && j < deg[b + 1]) {
                if (adj[i] < adj[j]) ++i;
                else if (adj[i] > adj[j]) ++j;
                else {
                    if (adj[i] > b) ++tri;
                    ++i;
                    ++j;
                }
            }
        }
    }
    free(deg); free(adj); free(fill);
    return tri;
}

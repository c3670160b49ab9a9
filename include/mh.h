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
 *     allocates no memory.  Its only state: per-device facts it caches (the
 *     number of CUs, kernels' occupancy) and the scratch array of
 *     mh_sample_unweighted_noalloc.
 *   - Concurrency: the order step of a network of at most 256 tiles of 4096
 *     nodes (and no more tiles than the GPU has CUs: n <= 1,048,576 on an
 *     MI355X) exchanges digit counts between all of its tiles, which must be
 *     resident at once.  Run such calls alone on the GPU: a kernel running
 *     beside them (another stream, another process) can keep a tile from
 *     starting, and the sort then waits until its spin limit and returns
 *     MH_EHIP.  Larger networks use a look-back that tolerates it.  Calls
 *     must not share a workspace unless they are ordered on one stream.
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
    int32_t grid_blocks; /* sweep grid in blocks of 256 threads; 0 = every resident block */
    int32_t pad;
    /* Optional stage timing: NULL, or an array of MH_STAGE_EVENTS events made
     * by the caller (hipEventCreate).  The samplers record them on `stream` at
     * the start, after the order step, after the bound and plan steps, and after
     * the sweep; NULL entries are skipped.  Recording adds no synchronisation. */
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

/* Bytes of workspace the sampler needs for n nodes (weighted != 0: UECM):
 * about 200-220 bytes per node with segments (plan->seg_work > 0), most of it room
 * for the records of up to 8 n + 4096 segments of heavy rows; a sample with
 * more locates the others in its sweep, correctly but more slowly. */
size_t mh_workspace_bytes(int64_t n, int weighted, const mh_plan_params* plan);

/* Sample one network from the unweighted model (Sec. 2.4).
 *   x[n]          parameters, device, float64.
 *   seed, replica Philox key and counter word: different replicas are
 *                 independent samples.
 *   plan          NULL = {seg_work = 8, grid_blocks = 0}.
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

/* Asynchronous samplers: the same work as mh_sample_unweighted /
 * mh_sample_weighted, enqueued on `stream` without waiting for it, so that
 * samples can follow one another on a stream with no host round trip between
 * them.  Argument errors are returned at once; the sample's edge count and
 * status stay in the workspace until mh_sample_result() reads them (it waits
 * for the stream).  A later call on the same workspace replaces them, in
 * stream order; the output buffers and the workspace must not be touched by
 * other work on other streams before the sample completes.  No statistics. */
mh_status mh_sample_unweighted_async(const double* x, int64_t n, uint64_t seed, uint32_t replica,
                                     const mh_plan_params* plan, int32_t* src, int32_t* dst,
                                     int64_t capacity, void* workspace, size_t ws_bytes,
                                     hipStream_t stream);
mh_status mh_sample_weighted_async(const double* x, const double* y, int64_t n, uint64_t seed,
                                   uint32_t replica, const mh_plan_params* plan, int32_t* src,
                                   int32_t* dst, int32_t* w, int64_t capacity, void* workspace,
                                   size_t ws_bytes, hipStream_t stream);
/* Waits for `stream` and reads the last asynchronous sample of `workspace`:
 * *n_edges_host = its edge count; MH_ECAPACITY if that exceeds capacity (the
 * capacity the sample was given); MH_EINVAL / MH_EHIP if the device found
 * invalid parameters or a stalled step. */
mh_status mh_sample_result(const void* workspace, size_t ws_bytes, int64_t capacity,
                           int64_t* n_edges_host, hipStream_t stream);

/* Allocation-free sampler, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): mh_sample_unweighted without the workspace argument.  Its
 * scratch is a device array of the library itself, MH_NOALLOC_SCRATCH_BYTES
 * on each GPU the library runs on, held until the process ends; the call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine).
 * The caller still owns x and the outputs.
 *   n <= MH_NOALLOC_MAX_NODES (else MH_EINVAL); a plan whose workspace would
 *   exceed the scratch returns MH_EWORKSPACE (never at n <= MH_NOALLOC_MAX_NODES).
 * Every call on a GPU uses that GPU's one scratch array, which keeps the
 * last call's contents (each call clears what must start at zero), so calls
 * that overlap on one GPU (other host threads, other streams) race: callers
 * serialise them.  Otherwise as mh_sample_unweighted: synchronous, same
 * edges, same statistics. */
#define MH_NOALLOC_SCRATCH_BYTES (64u << 20)
#define MH_NOALLOC_MAX_NODES 262144
mh_status mh_sample_unweighted_noalloc(const double* x, int64_t n, uint64_t seed, uint32_t replica,
                                       const mh_plan_params* plan, int32_t* src, int32_t* dst,
                                       int64_t capacity, int64_t* n_edges_host, mh_stats* stats_host,
                                       hipStream_t stream);

/* Two node sets: bipartite and directed networks (Sec. 2.6).  Rows are the
 * "+" set (x_rows, y_rows, n_rows), columns the "-" set (x_cols, y_cols,
 * n_cols); p_ij is the model's formula with z_i from the row set and z_j from
 * the column set.  Each set is sorted by its own z (descending, ties by id)
 * and every row sweeps all columns with the same skip / accept / update rule;
 * a chain over the column range [a, b) starts with the proposal probability of
 * column a itself, and the weighted bound of row r is
 * Y_r = y_r * max_j y_cols[j] (the smallest beta+_r + beta-_j row r can meet).
 * The plan rule above applies with first column 0 and n = n_cols.
 *   y_rows, y_cols  both NULL (unweighted) or both device float64 (weighted;
 *                   w receives the weights, and every y_i y_j must be < 1).
 *   flags           0, or MH_BIP_NO_SELF: the two sets index the same nodes
 *                   (rows = out-parameters, columns = in-parameters of a
 *                   directed network) and the pair (i, i) is never an edge.
 *   src, dst        edge = (row id, column id); order unspecified.
 *   workspace       >= mh_bipartite_workspace_bytes(n_rows, n_cols, weighted, plan).
 * The other arguments, the outputs and the errors are those of the one-set
 * samplers; (max row z)(max column z) must be finite.  An empty set gives an
 * empty sample without reading the other set. */
#define MH_BIP_NO_SELF 1u
size_t mh_bipartite_workspace_bytes(int64_t n_rows, int64_t n_cols, int weighted, const mh_plan_params* plan);
mh_status mh_sample_bipartite(const double* x_rows, const double* y_rows, int64_t n_rows,
                              const double* x_cols, const double* y_cols, int64_t n_cols, uint32_t flags,
                              uint64_t seed, uint32_t replica, const mh_plan_params* plan, int32_t* src,
                              int32_t* dst, int32_t* w, int64_t capacity, int64_t* n_edges_host,
                              void* workspace, size_t ws_bytes, mh_stats* stats_host, hipStream_t stream);

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

/* ---- Batched ensembles: many networks x many replicas in one persistent launch ----
 * Ensembles of hundreds or thousands of samples per null-model test motivate
 * the method (Sec. 2.2); here every network is ordered, bounded and planned
 * once, and all requested (network, replica) samples are swept by one resident
 * grid.  A sample (network i, replica r) is identical, edge for edge, to
 * mh_sample_unweighted/mh_sample_weighted(x_i[, y_i], seed, r) with the same
 * seg_work. */
typedef struct {
    int64_t n;        /* nodes */
    const double* x;  /* device float64[n] */
    const double* y;  /* device float64[n]; NULL = unweighted (every network of a batch uses the same model) */
    int32_t seg_work; /* plan parameter of this network (0 = one segment per row) */
    int32_t pad;
} mh_network;

#define MH_BATCH_EDGES 0   /* edges (src, dst[, w]) and optionally the sample index per edge (sid) */
#define MH_BATCH_DEGREES 1 /* per-sample degree sequences: degrees[deg_off[s] + node id] */
#define MH_BATCH_DEGREES_STAGED 2
#define MH_BATCH_OUT_CHUNK 4096                /* edge output: slots a wave reserves at a time */
#define MH_BATCH_EDGE_SLACK (4096ll * 4096ll)  /* edge output: room beyond the edges that always suffices */ /* the same sequences, columns counted through a slot buffer (src) */

typedef struct {
    int32_t seg_work;    /* chosen plan parameter */
    int32_t grid_blocks; /* chosen persistent grid (0 = all resident blocks) */
    float ms;            /* median probe time */
} mh_tuning;

/* Workspace for a batch of these networks and at most max_samples samples per call. */
size_t mh_batch_workspace_bytes(const mh_network* nets_host, int32_t n_networks, int32_t max_samples);

/* Order, bound and plan every network into the workspace (synchronous; MH_EINVAL
 * if any network's parameters are invalid).  Later calls on this workspace must
 * pass the same nets_host array. */
mh_status mh_batch_prepare(const mh_network* nets_host, int32_t n_networks, int32_t max_samples,
                           void* workspace, size_t ws_bytes, hipStream_t stream);

/* Sample s = 0..n_samples-1 is (network sample_net[s], replica sample_rep[s])
 * (device int32/uint32 arrays; a network index outside [0, n_networks) fails
 * the call with MH_EINVAL, reported by mh_batch_result).  MH_BATCH_EDGES: up to `capacity` edges into
 * src/dst (w for weighted networks; sid[k] = sample of edge k, may be NULL),
 * order unspecified.  Each wave of the launch reserves output slots
 * MH_BATCH_OUT_CHUNK at a time and the unused tails of the waves' last chunks
 * are filled afterwards, so the call needs room for the edges plus one chunk
 * per wave (4 waves per block, at most 4096 waves: MH_BATCH_EDGE_SLACK slots
 * always suffice); otherwise mh_batch_result returns MH_ECAPACITY with a
 * capacity that suffices (the edge count plus a chunk per wave).  MH_BATCH_DEGREES: degrees[deg_off[s] + v] (device int32,
 * offsets device int64; the caller's array must hold deg_off[s] + n of every
 * listed sample) is overwritten with node v's degree in sample s, every
 * accepted edge adding to its endpoints by a device atomic (the rate of random
 * atomic adds bounds it).  MH_BATCH_DEGREES_STAGED: the same degrees, the same
 * samples, counted through src (capacity int32 words, scratch owned by the
 * caller, contents undefined afterwards): each sample's node ids fall in
 * windows of 32768; the front of src holds 144 bytes of bookkeeping per
 * (sample, window) key, the rest the keys' slot regions, sized from a bound on
 * each window's expected column hits and cut at the capacity.  The sweep
 * writes each accepted edge's column into its key's region (one device atomic
 * per key and wave flush, not per edge) and a counting kernel adds every
 * region up in LDS, one block per key.  Columns beyond their region's end are
 * added by atomics; with less room than the bookkeeping, or a network of more
 * than 128 windows (4,194,304 nodes), the call counts by atomics throughout:
 * any capacity (0 included) gives the same degrees.
 * grid_blocks = 0 uses every resident block.  Asynchronous, kernels only: it
 * may be captured in a hipGraph.  mh_batch_result reads the edge count back. */
mh_status mh_batch_sample_async(const mh_network* nets_host, int32_t n_networks, int32_t max_samples,
                                void* workspace, size_t ws_bytes, const int32_t* sample_net,
                                const uint32_t* sample_rep, int32_t n_samples, uint64_t seed,
                                int32_t mode, int32_t* src, int32_t* dst, int32_t* w, int32_t* sid,
                                int64_t capacity, int32_t* degrees, const int64_t* deg_off,
                                int32_t grid_blocks, hipStream_t stream);

/* Edge count of the last batch call (synchronises the stream); MH_ECAPACITY if
 * it exceeds capacity (pass capacity < 0 to skip that check). */
mh_status mh_batch_result(const mh_network* nets_host, int32_t n_networks, int32_t max_samples,
                          void* workspace, size_t ws_bytes, int64_t* n_edges_host, int64_t capacity,
                          hipStream_t stream);

/* Capture mh_batch_sample_async with these arguments into an executable graph
 * (*exec_out, owned by the caller: hipGraphExecDestroy).  Replays sample the
 * same (network, replica) list, read from the same device arrays. */
mh_status mh_batch_capture(const mh_network* nets_host, int32_t n_networks, int32_t max_samples,
                           void* workspace, size_t ws_bytes, const int32_t* sample_net,
                           const uint32_t* sample_rep, int32_t n_samples, uint64_t seed, int32_t mode,
                           int32_t* src, int32_t* dst, int32_t* w, int32_t* sid, int64_t capacity,
                           int32_t* degrees, const int64_t* deg_off, int32_t grid_blocks,
                           hipStream_t stream, hipGraphExec_t* exec_out);

/* Time the degree-sink sweep of a probe batch for every (seg_work, grid) pair
 * of the candidates (median of 3), set every network's seg_work to the
 * fastest, prepare the workspace with it, and report it in *best.  The
 * workspace must fit the layout of every candidate. */
mh_status mh_batch_autotune(mh_network* nets_host, int32_t n_networks, int32_t max_samples,
                            void* workspace, size_t ws_bytes, const int32_t* sample_net,
                            const uint32_t* sample_rep, int32_t n_samples, int32_t* degrees,
                            const int64_t* deg_off, const int32_t* seg_candidates, int32_t n_seg,
                            const int32_t* grid_candidates, int32_t n_grid, mh_tuning* best,
                            hipStream_t stream);

/* Launch / destroy a graph made by mh_batch_capture (thin wrappers of the HIP calls). */
mh_status mh_graph_launch(hipGraphExec_t exec, hipStream_t stream);
mh_status mh_graph_destroy(hipGraphExec_t exec);

/* Canonical order of an edge list (a convenience: the method's output, the
 * edge list E of Alg. 1, is a set; its order leaves the sweep depending on the
 * schedule).  Sorts src[0..n_edges), dst[...] and, if w is not NULL, w[...] in
 * place by (src, dst) ascending, comparing node ids as integers; every pair
 * appears once in a sample, so the order is total and a sample's sorted list is
 * a function of its inputs alone.  Ids must be non-negative.  Device pointers on
 * `stream`; workspace: mh_sort_edges_workspace_bytes(n_edges) bytes, owned by
 * the caller.  Synchronous (reads the sort's status back): MH_EINVAL for
 * n_edges < 0 or above INT32_MAX or missing arrays, MH_EWORKSPACE, MH_EHIP. */
size_t mh_sort_edges_workspace_bytes(int64_t n_edges);
mh_status mh_sort_edges(int32_t* src, int32_t* dst, int32_t* w, int64_t n_edges, void* workspace,
                        size_t ws_bytes, hipStream_t stream);

/* ---- The Chung-Lu comparison model and the statistics of its bias ----
 * The Chung-Lu model read as edge probabilities, p_ij = min(w_i w_j, 1) with
 * w_i = k_i / sqrt(2M) (Sec. 2.1), is what the Miller-Hagberg algorithm samples
 * (Sec. 2.3); the paper contrasts it with the unbiased model on the density of
 * edges among the largest-degree nodes (Fig. 1A) and on triangle counts
 * (Fig. 1B). */
#define MH_MODEL_UBCM 0
#define MH_MODEL_CHUNG_LU 1

/* One Chung-Lu sample: as mh_sample_unweighted with w in place of x (device
 * float64 [n], finite, >= 0, (max w)^2 finite) and the chain of Sec. 2.3:
 * proposal q = min(t_q, 1), skip L = floor(-log U1 / -log1p(-t_q)) (0 when
 * t_q >= 1), accept iff U2 q < min(t, 1).  Same order, plan, counters,
 * workspace (mh_workspace_bytes(n, 0, plan)) and errors. */
mh_status mh_sample_chung_lu(const double* w, int64_t n, uint64_t seed, uint32_t replica,
                             const mh_plan_params* plan, int32_t* src, int32_t* dst, int64_t capacity,
                             int64_t* n_edges_host, void* workspace, size_t ws_bytes, mh_stats* stats_host,
                             hipStream_t stream);

/* One unweighted sample (model MH_MODEL_UBCM: x as mh_sample_unweighted;
 * MH_MODEL_CHUNG_LU: x as w above) reduced in the sweep to counts by rank, no
 * edge list: rank_counts[j] (device int32 [n], cleared by the call) = number
 * of edges whose endpoint of larger rank has rank j, ranks being positions in
 * the node order (descending x, ties by ascending id; mh_order gives it).  The
 * edges among the K nodes of largest x number rank_counts[0] + ... +
 * rank_counts[K-1], the numerator of the rich-club density of Fig. 1A.
 * *n_edges_host = the sample's edge count.  Same sample as the edge-list call
 * with the same arguments.  Synchronous; workspace mh_workspace_bytes(n, 0, plan). */
mh_status mh_sample_rank_counts(const double* x, int64_t n, int32_t model, uint64_t seed, uint32_t replica,
                                const mh_plan_params* plan, int32_t* rank_counts, int64_t* n_edges_host,
                                void* workspace, size_t ws_bytes, mh_stats* stats_host, hipStream_t stream);

/* Number of triangles of a simple undirected graph: src, dst device int32
 * [n_edges], each edge once in either orientation, ids in [0, n), no loops
 * (MH_EINVAL otherwise; a pair listed twice is counted as two edges).  Each
 * triangle is counted once, at its two smallest ids.  *triangles_host
 * receives the count.  Synchronous; workspace mh_triangles_workspace_bytes(n,
 * n_edges) bytes (about 40 bytes per edge and 8 per node), owned by the caller. */
size_t mh_triangles_workspace_bytes(int64_t n, int64_t n_edges);
mh_status mh_count_triangles(const int32_t* src, const int32_t* dst, int64_t n_edges, int64_t n,
                             uint64_t* triangles_host, void* workspace, size_t ws_bytes, hipStream_t stream);

const char* mh_status_string(mh_status s);

#ifdef __cplusplus
}
#endif
#endif

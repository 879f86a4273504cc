/*
 * sg.h -- C ABI of the MI355X (gfx950) shard-graph build library.
 *
 * The library builds the per-shard graph index of ScaleGANN's divide-and-merge
 * workflow (Sec. IV, "Workflow": partition the data with k-means into
 * overlapping shards, build every shard's graph independently on a GPU, merge
 * the shard graphs by edge union over the replicated vectors) and queries it.
 *
 * Conventions shared by every call
 * --------------------------------
 *  * Pointers are DEVICE pointers unless the name ends in `_h` (host).
 *  * Matrices are row-major; `ld` is the row stride in elements (>= d).
 *  * Ids are int32; SG_NONE (-1) pads lists that have fewer valid entries.
 *  * The caller owns every input, output and workspace buffer; the library
 *    never frees caller memory.  `ws` is a device workspace of at least the
 *    size returned by the matching *_workspace_size call (NULL allowed when
 *    that size is 0); it must stay untouched until the stream reaches the
 *    call's last kernel.
 *  * `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *    asynchronous on it unless stated otherwise.
 *  * Arguments are validated on the host before any launch; a bad argument
 *    returns SG_ERR_ARG (or SG_ERR_WORKSPACE) and launches nothing.  Launch
 *    and runtime failures return SG_ERR_HIP.  Outputs are undefined after an
 *    error.  sg_last_error() gives the calling thread's last error text.
 *  * Calls are re-entrant and thread-safe; calls that share output or
 *    workspace memory must be ordered by the caller.
 *  * Every kernel is deterministic: the same call on the same inputs writes
 *    the same bytes.
 *  * One call takes at most 2^26 - 1024 rows (n, nq, n_global, the rows of a
 *    batch with each shard padded to 256): kernels that give every row a
 *    wavefront launch 64 work-items per row, and a dispatch holds fewer than
 *    2^32 work-items.  Larger counts return SG_ERR_ARG.
 */
#ifndef SG_H
#define SG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sg_status;
enum {
    SG_OK = 0,
    SG_ERR_ARG = -1,          /* invalid argument (checked on the host)         */
    SG_ERR_HIP = -2,          /* HIP runtime or launch failure                  */
    SG_ERR_WORKSPACE = -3,    /* workspace missing or too small                 */
    SG_ERR_UNSUPPORTED = -4,  /* valid but not implemented shape / type combo   */
    SG_ERR_INTERNAL = -5      /* unexpected internal failure                    */
};
#define SG_NONE (-1)

typedef enum { SG_L2 = 0, SG_IP = 1 } sg_metric;
typedef enum { SG_F32 = 0, SG_F16 = 1, SG_BF16 = 2, SG_U8 = 3 } sg_dtype;

/* Arithmetic of the distance contraction in sg_knn_graph.
 *  SG_PREC_FP32 : FP32 inputs to FP32 MFMA, FP32 accumulation (the plain build).
 *  SG_PREC_F16  : FP16 inputs to FP16 MFMA, FP32 accumulation.  Exact for U8
 *                 data with d <= 128 (every product and partial sum is an
 *                 integer below 2^24), and the native type of FP16 data.
 *  SG_PREC_BF16 : rows rounded to BF16 (nearest even), BF16 MFMA, FP32
 *                 accumulation; a reduced-precision key followed by an FP32
 *                 re-rank when rerank > k.
 *  SG_PREC_FP8  : rows scaled per row by a power of two and rounded to OCP FP8
 *                 E4M3 (nearest even, saturating), FP8 MFMA, FP32
 *                 accumulation; followed by an FP32 re-rank when rerank > k.
 *  SG_PREC_I8   : U8 input only, d <= 256: rows shifted by -128 to INT8, INT8
 *                 MFMA with exact INT32 sums; the keys (L2: ||c'||^2 -
 *                 2 q'.c', IP: -q'.c' - 128 sum(c'), with x' = x - 128) are
 *                 integers below 2^24, so the result equals the FP32 build and
 *                 the exact kNN bit for bit, at twice the FP16 MFMA rate.
 *  With BF16 / FP8 and the IP metric the candidate key is the L2 key of the
 *  rounded rows with the candidate's exact squared norm put back,
 *  ||c~||^2 - ||c||^2 - 2 q~.c~: the same ranking as -q.c up to rounding, with
 *  a rounding error that scales with ||q - c||. */
typedef enum { SG_PREC_FP32 = 0, SG_PREC_F16 = 1, SG_PREC_BF16 = 2, SG_PREC_FP8 = 3, SG_PREC_I8 = 4 } sg_prec;

const char* sg_status_str(sg_status s);   /* static text for a status code            */
const char* sg_last_error(void);          /* detail of this thread's last failing call */
const char* sg_version(void);

/* ------------------------------------------------------------------------
 * sg_partition -- k-means partition with selective replication
 *
 * Follows Sec. IV step 1 and Sec. V (Algorithm 1) for one in-memory block:
 *  1. Lloyd k-means: centroids start at rows init_idx_h[0..S-1]; `iters`
 *     iterations of (assign each row to the nearest centroid by squared L2,
 *     ties to the lower index; replace each centroid by the FP64 mean of its
 *     members, an empty cluster keeping its centroid).  Distances are FP32;
 *     centroid sums are FP64 in a fixed-order two-level reduction.
 *  2. primary[i] = nearest centroid under the final centroids.
 *  3. Replicas (Sec. V-B): radius r[c] = largest Euclidean distance of c's
 *     primary members.  Row i with primary c at distance d visits the other
 *     centroids in ascending distance d' (ties to the lower index) and joins
 *     c' when d' < epsilon*d and d' < epsilon*tau*r[c'], until it is in omega
 *     shards.  epsilon = +inf accepts every visited centroid, i.e. each row
 *     joins its omega nearest centroids (the replicate-to-nearest policy).
 *  4. Membership: shard s holds member_ids[shard_offsets_h[s] ..
 *     shard_offsets_h[s+1]), ascending global row ids.
 *
 *  X        : n x d rows (stride ld) of `dtype`.
 *  S        : number of shards, 1..64;  omega: 1..min(S, 8);  iters >= 0.
 *  d        : 1..4096.
 *  centroids: out, S x d FP64.   primary: out, n int32.
 *  shard_offsets_h: out (host), S+1 int64.
 *  member_ids: out, `capacity` int32 (capacity >= n*omega always suffices).
 *  Synchronises `stream` (the membership sizes are data dependent).  Returns
 *  SG_ERR_ARG if the membership does not fit in `capacity`.
 * ---------------------------------------------------------------------- */
sg_status sg_partition_workspace_size(int64_t n, int32_t d, int32_t S, int32_t omega,
                                      size_t* bytes);
sg_status sg_partition(const void* X, sg_dtype dtype, int64_t n, int32_t d, int64_t ld,
                       int32_t S, int32_t omega, int32_t iters, float epsilon, float tau,
                       const int64_t* init_idx_h, double* centroids, int32_t* primary,
                       int64_t* shard_offsets_h, int32_t* member_ids, int64_t capacity,
                       void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * sg_partition_blockwise -- k-means partition with blockwise-adaptive
 * assignment and selective replication
 *
 * Follows Sec. V-A (blockwise-adaptive assignment) and Sec. V-B with
 * Algorithm 1, for rows streamed in blocks of block_rows in row order (the
 * order a disk-resident dataset is read in).  k-means as in sg_partition;
 * then, with the final centroids, for block t = 1, 2, ...:
 *  1. Original vectors first: each row of the block, in row order, joins its
 *     nearest AVAILABLE cluster (size < shard_cap; if every cluster is full,
 *     its nearest) as its primary.
 *  2. Statistics: R2[c] = largest squared distance of c's primaries so far;
 *     replica threshold theta[c] = max(0, shard_cap - ceil(prim[c] * n /
 *     seen)), the room left once the primaries expected from c's share so far
 *     are reserved (dense clusters get small thresholds; unlimited when
 *     shard_cap = 0 or adaptive = 0); tau_t = 1 + (tau0 - 1) / t, a radius
 *     factor that starts at tau0 and falls towards 1.
 *  3. Algorithm 1: each row, in row order, visits the other clusters by
 *     ascending distance and joins c' when size[c'] < shard_cap and
 *     rep[c'] < theta[c'] (checkSizeLimit) and d'^2 < eps^2 d^2 and
 *     d'^2 < eps^2 tau_t^2 R2[c'] (the distance and radius constraints,
 *     squared), until it is in omega clusters; epsilon = +inf skips the
 *     constraints.
 * Decisions use FP32 squared distances (FP32 centroids, fma sums over
 * ascending dimensions), visiting order by (squared distance, index) and
 * FP32 products.  One block of all rows with shard_cap = 0 and tau0 = 1 is the
 * single-block rule of sg_partition (in squared form).
 *  block_rows: >= 1;  shard_cap: >= 0 (0 = no limit);  tau0 >= 1;
 *  adaptive: 0 or 1.  primary: out, n int32, each row's primary cluster (its
 *  nearest available one).  Other arguments and outputs as sg_partition;
 *  the workspace size depends on block_rows.  Synchronises `stream`.
 * ---------------------------------------------------------------------- */
sg_status sg_partition_blockwise_workspace_size(int64_t n, int32_t d, int32_t S, int32_t omega,
                                                int64_t block_rows, size_t* bytes);
sg_status sg_partition_blockwise(const void* X, sg_dtype dtype, int64_t n, int32_t d, int64_t ld,
                                 int32_t S, int32_t omega, int32_t iters, float epsilon, float tau0,
                                 int64_t block_rows, int64_t shard_cap, int32_t adaptive,
                                 const int64_t* init_idx_h, double* centroids, int32_t* primary,
                                 int64_t* shard_offsets_h, int32_t* member_ids, int64_t capacity,
                                 void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * sg_knn_graph -- exact (or reduced-precision + re-ranked) kNN graph of one shard
 *
 * The per-shard index build of Sec. IV step 2, done as a tiled all-pairs
 * distance contraction (the dense-product formulation of Sec. II-A) fused
 * with a per-row top-k.  For rows i != j of the shard:
 *    L2: delta(i,j) = ||x_i - x_j||^2,   IP: delta(i,j) = -x_i . x_j.
 * Row i's list holds the k ids j != i (self excluded by index) with the
 * smallest (delta, j), ascending; fewer than k candidates pad with SG_NONE /
 * +inf.  dist[i][t] is delta(i, nbr[i][t]) in FP32.
 *  X      : n x d rows (stride ld) of `dtype`; ids are row indices 0..n-1.
 *  k      : 1..256.   prec: see sg_prec (FP32 needs F32/U8/F16/BF16 input,
 *           F16 needs F16 or U8 input, BF16 / FP8 need F32, F16 or U8 input).
 *  rerank : 0 for none, else c with k <= c <= 256: the top c by the `prec` key
 *           are re-scored with the exact FP32 difference-form distance and
 *           the best k by (delta, id) kept.
 *  nbr    : out, n x k int32.   dist: out, n x k FP32, may be NULL.
 *  order  : out, n int32, may be NULL: the rows in the order the build
 *           visited them (its locality order: rows grouped by nearest of
 *           about n/256 pivot rows, ascending row order within a pivot; the
 *           identity for small n), a permutation of 0..n-1 to pass to
 *           sg_prune.  The same call writes the same order.
 *  d      : 1..1024 for FP32 and FP8, 1..768 for FP16 / BF16 (larger d returns
 *           SG_ERR_UNSUPPORTED).  Queries are register resident up to FP32
 *           d <= 128 and 16-bit / FP8 d <= 768 / 1024; wider FP32 rows use a
 *           k-streamed kernel.
 * ---------------------------------------------------------------------- */
sg_status sg_knn_graph_workspace_size(int64_t n, int32_t d, int32_t k, sg_prec prec,
                                      int32_t rerank, size_t* bytes);
sg_status sg_knn_graph(const void* X, sg_dtype dtype, int64_t n, int32_t d, int64_t ld,
                       sg_metric metric, int32_t k, sg_prec prec, int32_t rerank, int32_t* nbr,
                       float* dist, int32_t* order, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * sg_quantize_rows -- the operand rows the distance contraction consumes
 *
 * The preparation step of the shard build: each row converted to the
 * arithmetic type of `prec`, exactly as sg_knn_graph prepares it (the
 * reduced-precision form of the precision study; the rounding and the
 * per-row scale are a reading -- the paper fixes no compute precision):
 *   SG_PREC_FP32 : FP32 values (exact for every input type);
 *   SG_PREC_F16  : FP16 (F16 or U8 input: exact);
 *   SG_PREC_BF16 : BF16 bits, round to nearest even (a NaN stays a quiet NaN);
 *   SG_PREC_FP8  : OCP FP8 E4M3 codes of x / 2^e (round to nearest even,
 *                  saturating at +-448, NaN -> 0x7f), with the per-row scale
 *                  exponent e = the smallest integer such that max|x| / 2^e
 *                  <= 448 (0 for an all-zero row), written to scale_exp.
 *  out      : n x ldo elements of the operand type (4, 2, 2 or 1 bytes),
 *             columns d..ldo-1 set to zero.  ldo: d..2^20.
 *  scale_exp: n int32 (FP8 only; NULL otherwise allowed).
 *  sqnorm   : n FP32, may be NULL: the squared L2 norm of the rounded row,
 *             the norm term the distance kernel adds (FP32 sum, each lane
 *             summing every 64th element, then a fixed butterfly).
 * Same input rules as sg_knn_graph (k and rerank aside).  No workspace.
 * ---------------------------------------------------------------------- */
sg_status sg_quantize_rows(const void* X, sg_dtype dtype, int64_t n, int32_t d, int64_t ld, sg_prec prec,
                           void* out, int64_t ldo, int32_t* scale_exp, float* sqnorm, void* stream);

/* ------------------------------------------------------------------------
 * sg_knn_rows -- exact (or re-ranked) kNN of listed rows against all rows
 *
 * The same computation as sg_knn_graph restricted to the query rows
 * rows[0..nq) (device int64 row indices of X): row r of nbr / dist is the
 * list of X row rows[r] over all n rows of X, itself excluded by index.  Used
 * to judge a build on a sample of rows.  Listed rows outside [0, n) give
 * empty lists.
 * ---------------------------------------------------------------------- */
sg_status sg_knn_rows_workspace_size(int64_t n, int32_t d, int64_t nq, int32_t k, sg_prec prec,
                                     int32_t rerank, size_t* bytes);
sg_status sg_knn_rows(const void* X, sg_dtype dtype, int64_t n, int32_t d, int64_t ld,
                      sg_metric metric, const int64_t* rows, int64_t nq, int32_t k, sg_prec prec,
                      int32_t rerank, int32_t* nbr, float* dist, void* ws, size_t ws_bytes,
                      void* stream);

/* ------------------------------------------------------------------------
 * sg_knn_graph_batched -- kNN graphs and pruned graphs of many shards at once
 *
 * The per-shard build of Sec. IV step 2 for all S shards of one GPU in a
 * single pass (the batching form): shard s is rows [offsets_h[s],
 * offsets_h[s+1]) of X (offsets_h[0] = 0, non-decreasing, S <= 64).  For each
 * shard the result equals sg_knn_graph on that shard alone (ids local to the
 * shard), followed by sg_prune to degree R:
 *    graphs[offsets_h[s] + i][0..R)  pruned list of local row i of shard s,
 *    knn   [offsets_h[s] + i][0..k)  its kNN list (knn may be NULL).
 * k in 1..256, R in 1..min(k, 128); rows need a register-resident distance
 * kernel (FP32 d <= 128, 16-bit d <= 768, FP8 d <= 1024).  rerank: 0, or a
 * candidate width c in k..256 as in sg_knn_graph (the c best by the prec
 * key, re-ranked by exact FP32 distance to the k lists).  The distance work
 * of all shards is one persistent launch (largest shards first); the launch
 * shape is the one sg_knn_autotune recorded for the largest shard, else the
 * default.
 *
 * plan: NULL runs the sequence eagerly on `stream`.  Otherwise the stream must
 * not be the default stream: if *plan is NULL the call captures the sequence
 * into a HIP graph, instantiates it, stores the new plan in *plan and launches
 * it; if *plan is a plan from an earlier call with identical arguments
 * (pointers, sizes, stream, device, launch shape) the call replays it with one
 * graph launch; other arguments give SG_ERR_ARG.  The plan is owned by the
 * caller and freed with sg_batch_plan_destroy (NULL is accepted).
 * ---------------------------------------------------------------------- */
typedef struct sg_batch_plan sg_batch_plan;
sg_status sg_knn_graph_batched_workspace_size(const int64_t* offsets_h, int32_t S, int32_t d, int32_t k,
                                              int32_t R, sg_prec prec, int32_t rerank, size_t* bytes);
sg_status sg_knn_graph_batched(const void* X, sg_dtype dtype, int32_t d, int64_t ld,
                               const int64_t* offsets_h, int32_t S, sg_metric metric, int32_t k,
                               int32_t R, sg_prec prec, int32_t rerank, int32_t* graphs, int32_t* knn,
                               void* ws, size_t ws_bytes, void* stream, sg_batch_plan** plan);
void sg_batch_plan_destroy(sg_batch_plan* plan);

/* sg_knn_graph_batched_autotune -- times the whole batched pass (arguments as
 * sg_knn_graph_batched without a plan; the outputs are written) once per
 * launch shape of the distance kernel and records the fastest for batched
 * calls of this precision, padded row length, selection width and
 * power-of-two bucket of the largest shard; without such a record a batched
 * call takes the shape recorded by sg_knn_autotune for its largest shard.  A
 * persistent launch over many shards can favour another shape than one
 * launch of its largest shard.  Synchronises `stream`.  chosen / times_ms as
 * sg_knn_autotune. */
sg_status sg_knn_graph_batched_autotune(const void* X, sg_dtype dtype, int32_t d, int64_t ld,
                                        const int64_t* offsets_h, int32_t S, sg_metric metric, int32_t k,
                                        int32_t R, sg_prec prec, int32_t rerank, int32_t* graphs, int32_t* knn,
                                        void* ws, size_t ws_bytes, void* stream, int32_t* chosen, float* times_ms,
                                        int32_t max_times);

/* ------------------------------------------------------------------------
 * Distance-kernel variants and autotuning
 *
 * Each (precision, padded row length) has a default distance kernel and may
 * have alternatives with other launch shapes (workgroup size, candidate rows
 * per LDS tile); all give identical results.  sg_knn_variant_count reports
 * how many exist for (prec, d, k).
 *
 * sg_knn_autotune times every variant on the given rows (the same arguments
 * and workspace as sg_knn_graph; no lists are written) and records the
 * fastest, process-wide, for calls of that precision, padded row length, k
 * and power-of-two bucket of n; later sg_knn_graph / sg_knn_rows calls of that
 * shape use it.  Synchronises `stream`.  chosen (nullable) receives the
 * winning index; times_ms (nullable when max_times == 0) receives up to
 * max_times per-variant milliseconds.
 *
 * sg_knn_force_variant makes the calling thread's later calls use variant
 * `variant` (an index past the end means the default), or, for -1, the
 * recorded choice again.  Meant for tests that check every variant.
 * ---------------------------------------------------------------------- */
sg_status sg_knn_variant_count(sg_prec prec, int32_t d, int32_t k, int32_t* count);
sg_status sg_knn_autotune(const void* X, sg_dtype dtype, int64_t n, int32_t d, int64_t ld,
                          sg_metric metric, int32_t k, sg_prec prec, int32_t rerank, void* ws,
                          size_t ws_bytes, void* stream, int32_t* chosen, float* times_ms,
                          int32_t max_times);
sg_status sg_knn_force_variant(int32_t variant);

/* ------------------------------------------------------------------------
 * sg_rerank -- exact re-rank of given candidate lists
 *
 * For each row i of X: the ids cand[i][0..c) (SG_NONE, out-of-range ids,
 * repeats and i itself skipped) are re-scored with the FP32 difference-form
 * distance (L2: sum_t (x_it - x_jt)^2; IP: -sum_t x_it x_jt) and the best k by
 * (delta, id) kept, padded with SG_NONE / +inf.  Summation order: ascending t
 * for d <= 128; for wider rows each of 64 lanes sums the elements 4l..4l+3 of
 * every 256-element chunk in ascending order and the 64 partial sums are
 * combined by a fixed butterfly (deterministic).  Used by the learned form:
 * candidates proposed on projected rows are re-ranked on the original rows.
 * k <= c <= 256; d <= 1024.  No workspace.
 * ---------------------------------------------------------------------- */
sg_status sg_rerank(const void* X, sg_dtype dtype, int64_t n, int32_t d, int64_t ld, sg_metric metric,
                    const int32_t* cand, int32_t c, int32_t k, int32_t* nbr, float* dist, void* stream);

/* ------------------------------------------------------------------------
 * sg_knn_graph_learned -- kNN graph from proposals on projected rows
 *
 * The learned form of the shard build: each row's candidates come from
 * low-dimensional projections P (n x e FP32 rows, stride ldp; e.g. the unit
 * projections of sg_mlp_project) instead of all-pairs distances on X.  Row
 * i's c candidates are the rows j != i with the largest P_i . P_j, ranked by
 * the FP8 key of sg_knn_graph (prec FP8, metric IP) on P; they are then
 * re-scored on X with the FP32 difference-form distance of `metric` (as
 * sg_rerank) and the best k by (delta, id) kept.  nbr / dist as sg_knn_graph.
 * With c >= n - 1 every row is a candidate and the result is the exact kNN
 * graph under the FP32 re-rank distance.  k <= c <= 256, e <= 1024,
 * d <= 1024.
 * ---------------------------------------------------------------------- */
sg_status sg_knn_graph_learned_workspace_size(int64_t n, int32_t e, int32_t c, size_t* bytes);
sg_status sg_knn_graph_learned(const void* X, sg_dtype dtype, int32_t d, int64_t ld, sg_metric metric,
                               const float* P, int64_t n, int32_t e, int64_t ldp, int32_t c, int32_t k,
                               int32_t* nbr, float* dist, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * sg_prune -- rank-based edge prune + reverse-edge pass to out-degree R
 *
 * The graph-optimisation step of the CAGRA shard build the paper uses
 * (Sec. II-A, Sec. IV step 2), in this reading:
 *  1. detour(x,j) = #{ i < j : y_j occurs in N(y_i) at a position < j },
 *     N(x) = [y_0 .. y_{K-1}] = knn row x.  Valid positions are ordered by
 *     (detour ascending, j ascending); the first R are P(x), in that order.
 *  2. Every x and p < R with y = P(x)[p] valid puts x into Rev(y) with key
 *     (p, x); Rev(y) is ordered by that key.  With h = ceil(R/2):
 *     F(y) = P(y)[0:h] ++ (Rev(y) entries not yet present)
 *            ++ (P(y)[h:R] entries not yet present), cut at R.
 *  knn : n x K int32, each row's valid ids distinct, in [0, n), != the row,
 *        followed by any SG_NONE padding (as sg_knn_graph writes it).
 *  K   : 1..256;  R: 1..min(K, 128).  out: n x R int32 (SG_NONE padded).
 *  Ids outside [0, n) in knn are treated as SG_NONE.
 *  order: NULL, or n device int32 giving the order in which rows are
 *        processed, e.g. the order sg_knn_graph returns, so that rows
 *        processed together share neighbour lists in cache.  The result never
 *        depends on it: an array that is not a permutation of 0..n-1 (an
 *        entry out of range or repeated) is detected on the device and the
 *        rows are then processed in row order.
 * ---------------------------------------------------------------------- */
sg_status sg_prune_workspace_size(int64_t n, int32_t K, int32_t R, size_t* bytes);
sg_status sg_prune(const int32_t* knn, int64_t n, int32_t K, int32_t R, const int32_t* order,
                   int32_t* out, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * sg_prune_noalloc -- sg_prune without a workspace argument and without
 * allocating
 *
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation).  Computes
 * exactly what sg_prune computes, with the same arguments minus the
 * workspace: the kernels use a static scratch array of
 * SG_PRUNE_NOALLOC_SCRATCH_BYTES in the library (one per GPU, held until the
 * process ends; its device address is looked up on the first call on each
 * GPU).  The call makes no allocation of any kind.
 *  Limit: sg_prune_workspace_size(n, K, R) must not exceed
 *  SG_PRUNE_NOALLOC_SCRATCH_BYTES (128 MiB: about 200 000 rows at R = 32,
 *  102 000 at R = 64, 32 000 at R = 128); larger calls return SG_ERR_ARG
 *  before any launch.
 *  Every call on one GPU shares that GPU's scratch (it keeps the last call's
 *  contents; the call clears what must start at zero): calls that may overlap
 *  on one GPU (different streams, or different host threads) race, and the
 *  caller must order them.
 * ---------------------------------------------------------------------- */
#define SG_PRUNE_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
sg_status sg_prune_noalloc(const int32_t* knn, int64_t n, int32_t K, int32_t R, const int32_t* order,
                           int32_t* out, void* stream);

/* ------------------------------------------------------------------------
 * sg_merge -- edge-union merge of shard graphs (Sec. II-A, Sec. IV step 3)
 *
 * graphs holds shards 0..S-1's R-wide lists (local ids) back to back, shard
 * s's rows at [shard_offsets_h[s], shard_offsets_h[s+1]); member_ids maps a
 * local row of shard s to its global id (ascending within each shard, as
 * sg_partition writes it; ids outside [0, n_global) are skipped, as are
 * local ids outside their shard).  For a global id g present in shards s_1 < .. <
 * s_m with lists L_1..L_m translated to global ids:
 *   for pos = 0..R-1, for t = 1..m: append L_t[pos] if valid, not yet in the
 *   list and != g; stop at max_degree.
 * max_degree = omega*R keeps the plain union; a smaller value caps it.
 *  out: n_global x max_degree int32 (SG_NONE padded);  degree: n_global int32.
 *  S: 1..65536;  R: 1..256;  max_degree: 1..1024.
 * ---------------------------------------------------------------------- */
sg_status sg_merge_workspace_size(int32_t S, const int64_t* shard_offsets_h, int64_t n_global,
                                  size_t* bytes);
sg_status sg_merge(int32_t S, const int64_t* shard_offsets_h, const int32_t* member_ids,
                   const int32_t* graphs, int32_t R, int64_t n_global, int32_t max_degree,
                   int32_t* out, int32_t* degree, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * sg_search -- greedy best-first beam search on the merged graph
 *
 * The DiskANN-style search used to query the merged index (Sec. VI).  A beam
 * of capacity L ordered by (delta, id) starts at `entry` (entry < 0: the
 * medoid, the row nearest to the mean of X, computed on the GPU).  Repeat:
 * expand the first unexpanded beam entry, visiting its neighbours in list
 * order, each id evaluated once per query, inserting those that beat the
 * L-th entry; stop when every beam entry is expanded.  The first topk entries
 * are returned.
 *  X: n x d (stride ld);  Q: nq x d (stride ldq), same dtype as X.
 *  graph: n x max_degree int32 (SG_NONE padded).
 *  topk <= L <= 512;  max_degree <= 256.
 *  out_ids: nq x topk;  out_dist: nq x topk FP32, may be NULL.
 * ---------------------------------------------------------------------- */
sg_status sg_search_workspace_size(int64_t n, int32_t d, int64_t nq, size_t* bytes);
sg_status sg_search(const void* X, sg_dtype dtype, int64_t n, int32_t d, int64_t ld,
                    sg_metric metric, const int32_t* graph, int32_t max_degree, const void* Q,
                    int64_t nq, int64_t ldq, int32_t topk, int32_t L, int64_t entry,
                    int32_t* out_ids, float* out_dist, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Learned candidate proposer (a small MLP trained on the GPU)
 *
 *   z = (x - mu) / sigma,  h1 = W1 z + b1,  a1 = GELU(h1) (erf form),
 *   h2 = W2 a1 + b2,  f = h2 / ||h2||          W1: H x D, W2: E x H (row-major)
 *
 * Rows are FP32 (n x D, stride ld).  Layer products use BF16-rounded operands
 * with FP32 accumulation; masters, biases, Adam moments and outputs are FP32.
 * sg_mlp_stats: mu = per-dimension mean, sigma = one global standard
 *   deviation, over the listed rows (ws: >= 2048 bytes).
 * sg_mlp_loss_grad: one forward + backward on B anchors and B positives
 *   (device row lists): in-batch softmax cross-entropy of the logits
 *   f(a_i).f(p_j)/T, target j = i; writes the mean loss (device float) and
 *   the gradients of W1, b1, W2, b2.
 * sg_mlp_train: `steps` Adam steps (bias corrected); step t uses anchors /
 *   positives [t*B, (t+1)*B) of the given device lists (the sampling is the
 *   caller's, seeded); adam_m / adam_v hold H*D + H + E*H + E floats each, in
 *   the order W1, b1, W2, b2, zero before the first step; losses (nullable)
 *   receives one loss per step.  use_graph != 0 captures one step in a
 *   hipGraph and replays it.
 * sg_mlp_project: f for every row into F (n x E).
 * ---------------------------------------------------------------------- */
sg_status sg_mlp_workspace_size(int32_t B, int32_t D, int32_t H, int32_t E, size_t* bytes);
sg_status sg_mlp_stats(const float* X, int64_t n, int32_t D, int64_t ld, const int64_t* rows,
                       int64_t nrows, float* mu, float* sigma, void* ws, size_t ws_bytes, void* stream);
sg_status sg_mlp_loss_grad(const float* X, int64_t n, int32_t D, int64_t ld, const int64_t* anchors,
                           const int64_t* positives, int32_t B, int32_t H, int32_t E, const float* W1,
                           const float* b1, const float* W2, const float* b2, const float* mu,
                           const float* sigma, float T, float* loss, float* gW1, float* gb1,
                           float* gW2, float* gb2, void* ws, size_t ws_bytes, void* stream);
sg_status sg_mlp_train(const float* X, int64_t n, int32_t D, int64_t ld, const int64_t* anchors,
                       const int64_t* positives, int32_t B, int32_t steps, int32_t H, int32_t E,
                       float* W1, float* b1, float* W2, float* b2, float* adam_m, float* adam_v,
                       const float* mu, const float* sigma, float T, float lr, float beta1,
                       float beta2, float eps, float* losses, int32_t use_graph, void* ws,
                       size_t ws_bytes, void* stream);
sg_status sg_mlp_project(const float* X, int64_t n, int32_t D, int64_t ld, int32_t H, int32_t E,
                         const float* W1, const float* b1, const float* W2, const float* b2,
                         const float* mu, const float* sigma, float* F, void* ws, size_t ws_bytes,
                         void* stream);
sg_status sg_mlp_project_workspace_size(int32_t D, int32_t H, int32_t E, size_t* bytes);

/* ------------------------------------------------------------------------
 * Profiling of the distance kernel (host-side, per process)
 *
 * sg_profile_begin() starts recording a pair of HIP events around every
 * launch of the fused distance + top-k kernel made by sg_knn_graph, on the
 * stream that launch uses.  sg_profile_end() waits for those events and
 * returns the summed kernel time (ms) and the number of launches since the
 * matching begin, then stops recording.  Not meant to be called concurrently
 * from several threads.
 * ---------------------------------------------------------------------- */
sg_status sg_profile_begin(void);
sg_status sg_profile_end(double* kernel_ms, int64_t* launches);

/* ------------------------------------------------------------------------
 * Scheduling shard builds on cloud GPU instances, and their cost
 * (Sec. IV, "Cloud Instance Task Scheduler" and "Spot instance cost
 * analysis").  Host-only calls: pointers ending in _h are host memory, no
 * device is touched.
 *
 * sg_cost_model: cost = (overall_time + transfer_time) * cpu_price
 *                      + (gpu_active_time + transfer_time) * gpu_price.
 *
 * sg_sched_fit_linear: least-squares line time = a + b * size through m >= 1
 * sampled builds (the paper estimates a shard's build time from small sampled
 * builds, build time being linear in shard size).
 *
 * sg_sched_simulate: T shard-build tasks (est_h: the scheduler's estimate,
 * actual_h > 0: the real time) on G instances.  Instance g is active in
 * [ready, end) (end = +inf: never terminated); its end becomes known to the
 * scheduler at `notice` (<= ready: known from the start, e.g. a guaranteed
 * duration; +inf: never told).  Availability-based policy: a task goes only
 * to an idle active instance.  Time-based policy (time_based = 1): an
 * instance whose end is known takes only tasks with transfer + est <= its
 * remaining lifetime.  A task occupies its instance for transfer + actual;
 * one whose instance terminates first returns to the head of the task list
 * and runs again.  At one time, terminations, then completions, then one
 * assignment pass over idle instances in index order, each taking the first
 * task in the list that fits (none: it stays idle).
 *  Outputs (nullable except summary_h): task_instance_h[T] (the instance that
 *  completed the task, -1 if it never did), task_start_h / task_end_h[T] (of
 *  the completing run, NaN if none), attempts_h[T] (runs started);
 *  summary_h[4] = { makespan, GPU active time (every occupation, lost work
 *  included), preemptions, tasks completed }.
 * ---------------------------------------------------------------------- */
typedef struct {
    double ready;    /* activation time, >= 0                                  */
    double end;      /* termination time (> ready; +inf: never)                */
    double notice;   /* time from which `end` is known (+inf: never)           */
} sg_instance;
sg_status sg_cost_model(double overall_time, double gpu_active_time, double transfer_time, double cpu_price,
                        double gpu_price, double* cost);
sg_status sg_sched_fit_linear(const double* sizes_h, const double* times_h, int32_t m, double* a, double* b);
sg_status sg_sched_simulate(const double* est_h, const double* actual_h, int32_t T, const sg_instance* inst_h,
                            int32_t G, int32_t time_based, double transfer, int32_t* task_instance_h,
                            double* task_start_h, double* task_end_h, int32_t* attempts_h, double* summary_h);

#ifdef __cplusplus
}
#endif
#endif /* SG_H */

/*
 * oracle.h -- plain, slow, obviously-correct FP64 CPU oracle for the per-shard
 * kNN-graph build of ScaleGANN (divide-and-merge graph ANN indexing).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant with the
 * GPU library.
 *
 * Every function states the passage of the paper (or the documented reading of
 * it) that it follows.  Floating point is FP64, except where a floating-point
 * comparison decides an integer outcome that the kernel decides too (the
 * blockwise assignment): that decision is taken in the kernel's FP32
 * arithmetic, written out step by step.  Inputs are the same stored arrays
 * (FP32 / FP16 / BF16 / U8) the GPU consumes, widened to FP64.
 *
 * Return value convention: 0 on success, negative on a bad argument.
 */
#ifndef SG_ORACLE_H
#define SG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_F32 = 0, ORC_F16 = 1, ORC_BF16 = 2, ORC_U8 = 3 };
enum { ORC_L2 = 0, ORC_IP = 1 };
#define ORC_NONE (-1)

/* Threads the OpenMP loops of this library use. */
int orc_num_threads(void);

/* Widen an n x d row-major array (row stride ld elements) of the given dtype to FP64. */
int orc_widen(const void* X, int dtype, int64_t n, int d, int64_t ld, double* out);

/* Exact kNN of the given query rows against all n rows (Sec. II-A: kNN graph,
 * distances by dense products; Sec. IV step 2: per-shard index build).
 * delta(i,j) = sum_t (x_it - x_jt)^2 (L2) or -sum_t x_it x_jt (IP), summed in
 * FP64 in the fixed order t = 0..d-1.  Row i's list is the first K of
 * {j != i} ordered by (delta ascending, j ascending); padded with ORC_NONE /
 * +inf when fewer than K exist.  rows == NULL means all rows 0..n-1 (nrows
 * must then equal n).  nbr, dist: nrows x K. */
int orc_knn(const double* X, int64_t n, int d, int metric, int K,
            const int64_t* rows, int64_t nrows, int32_t* nbr, double* dist);

/* delta(pairs[2p], pairs[2p+1]) for npairs (row, row) pairs, FP64 as in orc_knn;
 * ORC_NONE in either slot gives +inf. */
int orc_pair_dist(const double* X, int64_t n, int d, int metric, const int64_t* pairs,
                  int64_t npairs, double* out);

/* Rank-based (detour-count) prune of a kNN graph down to out-degree R.
 * detour(x,j) = #{ i < j : y_j occurs in N(y_i) at a position < j }, with
 * N(x) = [y_0 .. y_{K-1}].  Valid positions are ordered by (detour, j); the
 * first R form P(x) in that order.  ORC_NONE entries are skipped and pad the
 * tail. */
int orc_detour_prune(const int32_t* knn, int64_t n, int K, int R, int32_t* P);

/* Reverse-edge pass and combine.  For every x and p < R with y = P(x)[p]
 * valid, x joins Rev(y) with key (p, x); Rev(y) is ordered by that key.
 * With h = ceil(R/2):  F(y) = P(y)[0:h] ++ (Rev(y) not yet present)
 * ++ (P(y)[h:R] not yet present), cut at R, padded with ORC_NONE. */
int orc_reverse_combine(const int32_t* P, int64_t n, int R, int32_t* F);

/* Merge of shard graphs by edge union over replicated vectors (Sec. II-A,
 * Sec. IV step 3).  graphs holds the per-shard R-wide lists (local ids) for
 * shards 0..S-1 back to back; member_ids maps local row to global id.
 * For a global id present in shards s_1 < ... < s_m with lists L_1..L_m
 * (translated to global ids): for pos = 0..R-1, for t = 1..m, append L_t[pos]
 * if valid, not yet present and not the id itself; stop at max_degree.
 * out: n_global x max_degree (ORC_NONE padded), degree: n_global. */
int orc_merge(int S, const int64_t* shard_offsets, const int32_t* member_ids,
              const int32_t* graphs, int R, int64_t n_global, int max_degree,
              int32_t* out, int32_t* degree);

/* Lloyd k-means (Sec. IV step 1, Sec. V): centroids start at the rows
 * init_idx[0..S-1]; each of `iters` iterations assigns every row to the
 * nearest centroid (squared L2, ties to the lower index) and replaces every
 * centroid by the FP64 mean of its members (an empty cluster keeps its
 * centroid).  centroids (in/out not needed): S x d.  labels: final nearest
 * centroid of each row under the returned centroids. */
int orc_kmeans(const double* X, int64_t n, int d, int S, int iters,
               const int64_t* init_idx, double* centroids, int32_t* labels);

/* Selective replica assignment (Sec. V-B, Algorithm 1) for one in-memory
 * block (tau given, capacity unlimited).  d, d', r' are unsquared Euclidean
 * distances; r[c] = max distance of c's primary members.  For each vector v
 * with primary c (its nearest centroid), centroids are visited in ascending
 * distance (ties to the lower index); c' != c joins v's shards when
 * d' < eps*d and d' < eps*tau*r[c'], until omega shards are reached.
 * eps = +inf accepts every visited centroid (the replicate-to-nearest-others
 * policy).  assign: n x omega shard ids (primary first, ORC_NONE padded).
 * counts: S shard sizes. */
int orc_assign_replicas(const double* X, int64_t n, int d, const double* centroids,
                        int S, const int32_t* primary, int omega, double eps, double tau,
                        int32_t* assign, int64_t* counts);

/* Blockwise-adaptive assignment with selective replication (Sec. V-A, V-B,
 * Algorithm 1) over rows streamed in blocks of block_rows (row order):
 * per block, primaries to the nearest available cluster (size < cap), then
 * radius, replica thresholds theta[c] = max(0, cap - ceil(prim[c] n / seen))
 * (unlimited when cap = 0 or adaptive = 0) and tau_t = 1 + (tau0 - 1)/t, then
 * replicas by Algorithm 1 with the size check size < cap and rep < theta and
 * the constraints in squared form, d'^2 < eps^2 d^2, d'^2 < eps^2 tau_t^2 R2.
 * Decisions are taken in FP32 (the kernel's precision): FP32 centroids,
 * fma-summed squared distances over ascending t, FP32 products.
 * assign: n x omega (primary first, ORC_NONE padded); counts: S sizes. */
int orc_assign_blockwise(const double* X, int64_t n, int d, const double* C, int S, int omega,
                         double eps, double tau0, int64_t block_rows, int64_t cap, int adaptive,
                         int32_t* assign, int64_t* counts);

/* Shard membership in CSR form, each shard's member list ascending by global
 * id (so the order of vectors inside a shard is deterministic). */
int orc_membership(const int32_t* assign, int64_t n, int omega, int S,
                   int64_t* shard_offsets, int32_t* member_ids);

/* Medoid: argmin_i ||x_i - mean(X)||^2 in FP64, ties to the lower id. */
int64_t orc_medoid(const double* X, int64_t n, int d);

/* Greedy beam search on a graph (the DiskANN-style best-first search used to
 * query the merged index, Sec. VI).  Beam of capacity L ordered by
 * (delta, id); repeatedly expand the first unexpanded beam entry, visiting its
 * neighbours in list order (each id evaluated once), inserting those that
 * beat the L-th entry; stop when every beam entry is expanded.  entry < 0
 * means the medoid.  out_ids / out_dist: nq x topk. */
int orc_search(const double* X, int64_t n, int d, int metric, const int32_t* graph,
               int max_degree, const double* Q, int64_t nq, int topk, int L,
               int64_t entry, int32_t* out_ids, double* out_dist);

/* Re-rank: each row's c candidate ids (ORC_NONE, repeats and the row itself
 * skipped) re-scored with the exact FP64 delta; the first K by (delta, id)
 * are kept. */
int orc_rerank(const double* X, int64_t n, int d, int metric, const int32_t* cand,
               int c, int K, int32_t* nbr, double* dist);

/* Rounding of FP32 values to BF16 (round to nearest, ties to even). */
int orc_to_bf16(const float* x, int64_t n, uint16_t* out);
/* Rounding of FP32 values to OCP FP8 E4M3 (bias 7, largest finite 448, no
 * infinity), round to nearest even, saturating to +-448. */
int orc_to_fp8e4m3(const float* x, int64_t n, uint8_t* out);
/* Decoders (exact). */
int orc_from_bf16(const uint16_t* x, int64_t n, double* out);
int orc_from_fp8e4m3(const uint8_t* x, int64_t n, double* out);
/* Per-row power-of-two FP8 scaling: s_i = 2^ceil(log2(amax_i / 448)) (1 for an
 * all-zero row); q_ij = fp8(x_ij / s_i). */
int orc_quant_rows_fp8(const float* X, int64_t n, int d, uint8_t* q, float* scale);

/* Learned proposer (a small MLP, not in the paper):
 *   z = (x - mu) / sigma,  h1 = W1 z + b1,  a1 = GELU(h1) (erf form),
 *   h2 = W2 a1 + b2,  f = h2 / ||h2||.
 * W1: H x D, W2: E x H (row-major), biases FP64 copies of the caller's. */
int orc_mlp_forward(const double* X, int64_t n, int D, int H, int E,
                    const double* W1, const double* b1, const double* W2, const double* b2,
                    const double* mu, double sigma, double* F);
/* In-batch softmax cross-entropy over logits l_ij = f(a_i) . f(p_j) / T,
 * loss = mean_i CE(l_i, i), and its exact gradients with respect to
 * W1, b1, W2, b2 (anchors and positives share the network). */
int orc_mlp_loss_grad(const double* Xa, const double* Xp, int64_t B, int D, int H, int E,
                      const double* W1, const double* b1, const double* W2, const double* b2,
                      const double* mu, double sigma, double T, double* loss,
                      double* gW1, double* gb1, double* gW2, double* gb2);
/* One Adam step (bias-corrected), in place on w, m, v. */
int orc_adam(double* w, const double* g, double* m, double* v, int64_t n, double lr,
             double beta1, double beta2, double eps, int64_t step);

#ifdef __cplusplus
}
#endif
#endif

/*
 * oracle.c -- plain FP64 CPU oracle for the per-shard kNN-graph build.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Written for
 * obviousness, not speed: no blocking, no fusion, full sorts where the
 * definition is a sort.  Each function cites the passage it follows; the
 * prune / reverse / merge rules are readings of the paper (which names CAGRA's
 * graph optimisation and DiskANN's edge-union merge without defining them),
 * documented beside their definitions in oracle.h.
 *
 * Parity status (what pins each function) is listed at the top of the test
 * files under tests/ that exercise it.
 */
#include "oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

int orc_num_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ */
/* element decoding                                                    */
/* ------------------------------------------------------------------ */

static double half_to_double(uint16_t h) {
    int sign = (h >> 15) & 1;
    int e = (h >> 10) & 0x1f;
    int m = h & 0x3ff;
    double v;
    if (e == 0) {
        v = ldexp((double)m, -24);               /* subnormal: m * 2^-24 */
    } else if (e == 31) {
        v = m ? NAN : INFINITY;
    } else {
        v = ldexp(1.0 + m / 1024.0, e - 15);
    }
    return sign ? -v : v;
}

static double bf16_to_double(uint16_t b) {
    uint32_t bits = ((uint32_t)b) << 16;
    float f;
    memcpy(&f, &bits, 4);
    return (double)f;
}

int orc_widen(const void* X, int dtype, int64_t n, int d, int64_t ld, double* out) {
    if (n < 0 || d <= 0 || ld < d) return -1;
    for (int64_t i = 0; i < n; ++i) {
        for (int t = 0; t < d; ++t) {
            int64_t k = i * ld + t;
            double v;
            switch (dtype) {
                case ORC_F32: v = ((const float*)X)[k]; break;
                case ORC_F16: v = half_to_double(((const uint16_t*)X)[k]); break;
                case ORC_BF16: v = bf16_to_double(((const uint16_t*)X)[k]); break;
                case ORC_U8: v = ((const uint8_t*)X)[k]; break;
                default: return -1;
            }
            out[i * (int64_t)d + t] = v;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* distances                                                           */
/* ------------------------------------------------------------------ */

/* delta(a, b): squared Euclidean or negated inner product, FP64, t ascending. */
static double delta(const double* a, const double* b, int d, int metric) {
    double s = 0.0;
    if (metric == ORC_L2) {
        for (int t = 0; t < d; ++t) {
            double u = a[t] - b[t];
            s += u * u;
        }
        return s;
    }
    for (int t = 0; t < d; ++t) s += a[t] * b[t];
    return -s;
}

typedef struct {
    double dist;
    int64_t id;
} cand_t;

/* total order: distance ascending, then id ascending */
static int cand_cmp(const void* pa, const void* pb) {
    const cand_t* a = (const cand_t*)pa;
    const cand_t* b = (const cand_t*)pb;
    if (a->dist < b->dist) return -1;
    if (a->dist > b->dist) return 1;
    if (a->id < b->id) return -1;
    if (a->id > b->id) return 1;
    return 0;
}

/* ------------------------------------------------------------------ */
/* exact kNN                                                           */
/* ------------------------------------------------------------------ */

int orc_knn(const double* X, int64_t n, int d, int metric, int K,
            const int64_t* rows, int64_t nrows, int32_t* nbr, double* dist) {
    if (n < 0 || d <= 0 || K <= 0 || (metric != ORC_L2 && metric != ORC_IP)) return -1;
    if (!rows && nrows != n) return -1;
    int bad = 0;
#pragma omp parallel
    {
        cand_t* all = (cand_t*)malloc(sizeof(cand_t) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 16)
        for (int64_t r = 0; r < nrows; ++r) {
            int64_t i = rows ? rows[r] : r;
            if (i < 0 || i >= n) {
                bad = 1;
                continue;
            }
            int64_t m = 0;
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;                 /* self excluded by index */
                all[m].dist = delta(X + i * d, X + j * d, d, metric);
                all[m].id = j;
                ++m;
            }
            qsort(all, (size_t)m, sizeof(cand_t), cand_cmp);
            for (int k = 0; k < K; ++k) {
                if (k < m) {
                    nbr[r * K + k] = (int32_t)all[k].id;
                    if (dist) dist[r * K + k] = all[k].dist;
                } else {
                    nbr[r * K + k] = ORC_NONE;
                    if (dist) dist[r * K + k] = INFINITY;
                }
            }
        }
        free(all);
    }
    return bad ? -1 : 0;
}

int orc_pair_dist(const double* X, int64_t n, int d, int metric, const int64_t* pairs,
                  int64_t npairs, double* out) {
    if (n < 0 || d <= 0 || (metric != ORC_L2 && metric != ORC_IP)) return -1;
    for (int64_t p = 0; p < npairs; ++p) {
        int64_t a = pairs[2 * p], b = pairs[2 * p + 1];
        if (a == ORC_NONE || b == ORC_NONE) {
            out[p] = INFINITY;
            continue;
        }
        if (a < 0 || a >= n || b < 0 || b >= n) return -1;
        out[p] = delta(X + a * d, X + b * d, d, metric);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* detour-count prune                                                  */
/* ------------------------------------------------------------------ */

int orc_detour_prune(const int32_t* knn, int64_t n, int K, int R, int32_t* P) {
    if (n < 0 || K <= 0 || R <= 0 || R > K) return -1;
    for (int64_t k = 0; k < n * K; ++k)
        if (knn[k] != ORC_NONE && (knn[k] < 0 || knn[k] >= n)) return -1;
    int bad = 0;
#pragma omp parallel
    {
        int* det = (int*)malloc(sizeof(int) * K);
        int* order = (int*)malloc(sizeof(int) * K);
#pragma omp for schedule(dynamic, 64)
        for (int64_t x = 0; x < n; ++x) {
            const int32_t* Nx = knn + x * K;
            int nvalid = 0;
            for (int j = 0; j < K; ++j) {
                det[j] = 0;
                if (Nx[j] == ORC_NONE) continue;
                /* count i < j whose list holds y_j before position j */
                for (int i = 0; i < j; ++i) {
                    if (Nx[i] == ORC_NONE) continue;
                    const int32_t* Ny = knn + (int64_t)Nx[i] * K;
                    for (int p = 0; p < j; ++p) {
                        if (Ny[p] == Nx[j]) {
                            det[j] += 1;
                            break;
                        }
                    }
                }
                order[nvalid++] = j;
            }
            /* stable insertion sort of valid positions by detour count
             * (positions enter in ascending j, so equal counts keep j order) */
            for (int a = 1; a < nvalid; ++a) {
                int v = order[a];
                int b = a - 1;
                while (b >= 0 && det[order[b]] > det[v]) {
                    order[b + 1] = order[b];
                    --b;
                }
                order[b + 1] = v;
            }
            for (int r = 0; r < R; ++r)
                P[x * R + r] = (r < nvalid) ? Nx[order[r]] : ORC_NONE;
        }
        free(det);
        free(order);
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* reverse edges + combine                                             */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t p;
    int32_t x;
} rev_t;

static int rev_cmp(const void* pa, const void* pb) {
    const rev_t* a = (const rev_t*)pa;
    const rev_t* b = (const rev_t*)pb;
    if (a->p != b->p) return a->p < b->p ? -1 : 1;
    if (a->x != b->x) return a->x < b->x ? -1 : 1;
    return 0;
}

static int present(const int32_t* list, int len, int32_t v) {
    for (int i = 0; i < len; ++i)
        if (list[i] == v) return 1;
    return 0;
}

int orc_reverse_combine(const int32_t* P, int64_t n, int R, int32_t* F) {
    if (n < 0 || R <= 0) return -1;
    for (int64_t k = 0; k < n * R; ++k)
        if (P[k] != ORC_NONE && (P[k] < 0 || P[k] >= n)) return -1;
    /* collect Rev(y) */
    int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t k = 0; k < n * R; ++k)
        if (P[k] != ORC_NONE) cnt[P[k] + 1] += 1;
    for (int64_t y = 0; y < n; ++y) cnt[y + 1] += cnt[y];
    int64_t total = cnt[n];
    rev_t* rev = (rev_t*)malloc(sizeof(rev_t) * (size_t)(total > 0 ? total : 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t y = 0; y < n; ++y) fill[y] = cnt[y];
    for (int64_t x = 0; x < n; ++x)
        for (int p = 0; p < R; ++p) {
            int32_t y = P[x * R + p];
            if (y == ORC_NONE) continue;
            rev[fill[y]].p = p;
            rev[fill[y]].x = (int32_t)x;
            fill[y] += 1;
        }
    int h = (R + 1) / 2;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t y = 0; y < n; ++y) {
        rev_t* ry = rev + cnt[y];
        int64_t ny = cnt[y + 1] - cnt[y];
        qsort(ry, (size_t)ny, sizeof(rev_t), rev_cmp);
        int32_t* out = F + y * R;
        int len = 0;
        for (int q = 0; q < h && len < R; ++q) {
            int32_t v = P[y * R + q];
            if (v != ORC_NONE && !present(out, len, v)) out[len++] = v;
        }
        for (int64_t e = 0; e < ny && len < R; ++e) {
            int32_t v = ry[e].x;
            if (!present(out, len, v)) out[len++] = v;
        }
        for (int q = h; q < R && len < R; ++q) {
            int32_t v = P[y * R + q];
            if (v != ORC_NONE && !present(out, len, v)) out[len++] = v;
        }
        for (int q = len; q < R; ++q) out[q] = ORC_NONE;
    }
    free(cnt);
    free(rev);
    free(fill);
    return 0;
}

/* ------------------------------------------------------------------ */
/* merge                                                               */
/* ------------------------------------------------------------------ */

int orc_merge(int S, const int64_t* off, const int32_t* member_ids, const int32_t* graphs,
              int R, int64_t n_global, int max_degree, int32_t* out, int32_t* degree) {
    if (S <= 0 || R <= 0 || max_degree <= 0 || n_global < 0) return -1;
    if (off[0] != 0) return -1;
    for (int s = 0; s < S; ++s)
        if (off[s + 1] < off[s]) return -1;
    int64_t total = off[S];
    for (int64_t r = 0; r < total; ++r)
        if (member_ids[r] < 0 || member_ids[r] >= n_global) return -1;
    /* occurrences of each global id as (shard, row), gathered shard by shard
     * so each id's occurrences come out in ascending shard order */
    int64_t* cnt = (int64_t*)calloc((size_t)n_global + 1, sizeof(int64_t));
    for (int64_t r = 0; r < total; ++r) cnt[member_ids[r] + 1] += 1;
    for (int64_t g = 0; g < n_global; ++g) cnt[g + 1] += cnt[g];
    int64_t* occ = (int64_t*)malloc(sizeof(int64_t) * (size_t)(total > 0 ? total : 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_global > 0 ? n_global : 1));
    for (int64_t g = 0; g < n_global; ++g) fill[g] = cnt[g];
    for (int s = 0; s < S; ++s)
        for (int64_t r = off[s]; r < off[s + 1]; ++r) occ[fill[member_ids[r]]++] = r;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t g = 0; g < n_global; ++g) {
        int32_t* o = out + g * (int64_t)max_degree;
        int len = 0;
        for (int pos = 0; pos < R && len < max_degree; ++pos) {
            for (int64_t t = cnt[g]; t < cnt[g + 1] && len < max_degree; ++t) {
                int64_t row = occ[t];
                int s = 0;
                while (!(row >= off[s] && row < off[s + 1])) ++s;
                int32_t v = graphs[row * R + pos];
                if (v == ORC_NONE) continue;
                if (v < 0 || v >= off[s + 1] - off[s]) {
                    bad = 1;
                    continue;
                }
                int32_t gv = member_ids[off[s] + v];
                if (gv == g || present(o, len, gv)) continue;
                o[len++] = gv;
            }
        }
        degree[g] = len;
        for (int q = len; q < max_degree; ++q) o[q] = ORC_NONE;
    }
    free(cnt);
    free(occ);
    free(fill);
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* k-means partition + selective replication                           */
/* ------------------------------------------------------------------ */

static int32_t nearest_centroid(const double* x, const double* C, int S, int d) {
    int32_t best = 0;
    double bd = delta(x, C, d, ORC_L2);
    for (int c = 1; c < S; ++c) {
        double v = delta(x, C + (int64_t)c * d, d, ORC_L2);
        if (v < bd) {                           /* strict: ties stay at lower index */
            bd = v;
            best = c;
        }
    }
    return best;
}

int orc_kmeans(const double* X, int64_t n, int d, int S, int iters, const int64_t* init_idx,
               double* C, int32_t* labels) {
    if (n <= 0 || d <= 0 || S <= 0 || iters < 0) return -1;
    for (int c = 0; c < S; ++c) {
        if (init_idx[c] < 0 || init_idx[c] >= n) return -1;
        memcpy(C + (int64_t)c * d, X + init_idx[c] * d, sizeof(double) * d);
    }
    double* sum = (double*)malloc(sizeof(double) * (size_t)S * d);
    int64_t* count = (int64_t*)malloc(sizeof(int64_t) * S);
    for (int it = 0; it < iters; ++it) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) labels[i] = nearest_centroid(X + i * d, C, S, d);
        memset(sum, 0, sizeof(double) * (size_t)S * d);
        memset(count, 0, sizeof(int64_t) * S);
        for (int64_t i = 0; i < n; ++i) {       /* members summed in ascending row order */
            int c = labels[i];
            count[c] += 1;
            for (int t = 0; t < d; ++t) sum[(int64_t)c * d + t] += X[i * d + t];
        }
        for (int c = 0; c < S; ++c) {
            if (count[c] == 0) continue;         /* empty cluster keeps its centroid */
            for (int t = 0; t < d; ++t)
                C[(int64_t)c * d + t] = sum[(int64_t)c * d + t] / (double)count[c];
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) labels[i] = nearest_centroid(X + i * d, C, S, d);
    free(sum);
    free(count);
    return 0;
}

int orc_assign_replicas(const double* X, int64_t n, int d, const double* C, int S,
                        const int32_t* primary, int omega, double eps, double tau,
                        int32_t* assign, int64_t* counts) {
    if (n < 0 || d <= 0 || S <= 0 || omega <= 0) return -1;
    /* radius of each cluster: largest unsquared distance of a primary member */
    double* radius = (double*)calloc((size_t)S, sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        int c = primary[i];
        if (c < 0 || c >= S) {
            free(radius);
            return -1;
        }
        double r = sqrt(delta(X + i * d, C + (int64_t)c * d, d, ORC_L2));
        if (r > radius[c]) radius[c] = r;
    }
    int accept_all = isinf(eps) && eps > 0;
#pragma omp parallel
    {
        cand_t* cs = (cand_t*)malloc(sizeof(cand_t) * S);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            const double* x = X + i * d;
            int c = primary[i];
            for (int k = 0; k < S; ++k) {
                cs[k].dist = sqrt(delta(x, C + (int64_t)k * d, d, ORC_L2));
                cs[k].id = k;
            }
            qsort(cs, (size_t)S, sizeof(cand_t), cand_cmp);   /* ascending, ties lower index */
            double dc = sqrt(delta(x, C + (int64_t)c * d, d, ORC_L2));
            int32_t* a = assign + i * omega;
            int assigned = 1;
            a[0] = c;
            for (int k = 0; k < S; ++k) {
                if (assigned >= omega) break;
                int cc = (int)cs[k].id;
                if (cc == c) continue;
                double dp = cs[k].dist;
                if (accept_all || (dp < eps * dc && dp < eps * tau * radius[cc])) a[assigned++] = cc;
            }
            for (int k = assigned; k < omega; ++k) a[k] = ORC_NONE;
        }
        free(cs);
    }
    for (int c = 0; c < S; ++c) counts[c] = 0;
    for (int64_t k = 0; k < n * omega; ++k)
        if (assign[k] != ORC_NONE) counts[assign[k]] += 1;
    free(radius);
    return 0;
}

/* Blockwise-adaptive assignment (Sec. V-A) with selective replication
 * (Sec. V-B, Algorithm 1), rows streamed in blocks of `block_rows` in row
 * order.  For block t = 1, 2, ...:
 *   1. each row in order joins its nearest AVAILABLE cluster (size < cap;
 *      with every cluster full, its nearest) as its primary ("original
 *      vectors first");
 *   2. statistics: R2[c] = largest squared distance of c's primaries so far;
 *      the replica threshold theta[c] = cap - ceil(prim[c] * n / seen), at
 *      least 0 (space kept for the primaries still expected; dense clusters
 *      get small thresholds), unlimited when cap = 0 or adaptive = 0;
 *      tau_t = 1 + (tau0 - 1) / t (large early, tending to 1);
 *   3. each row in order visits the other clusters by ascending distance and
 *      joins c' when size[c'] < cap and rep[c'] < theta[c'] (checkSizeLimit)
 *      and d'^2 < eps^2 d^2 and d'^2 < eps^2 tau_t^2 R2[c'] (both constraints,
 *      squared), until it is in omega clusters (eps = +inf: every available
 *      cluster).
 * The decisions are integer outcomes of floating-point comparisons, taken
 * here in the FP32 arithmetic the GPU kernel uses: centroids rounded to FP32,
 * squared distances summed as s = fma(u, u, s) over ascending t with
 * u = x_t - c_t, visiting order by (squared distance, index), and the
 * products eps^2 * d^2 and (eps^2 * tau_t^2) * R2 rounded to FP32.
 * assign: n x omega (primary first, then replicas in the order taken,
 * ORC_NONE padded); counts: S cluster sizes. */
typedef struct {
    float d2;
    int id;
} fcand_t;

static int fcand_cmp(const void* pa, const void* pb) {
    const fcand_t* a = (const fcand_t*)pa;
    const fcand_t* b = (const fcand_t*)pb;
    if (a->d2 < b->d2) return -1;
    if (a->d2 > b->d2) return 1;
    return a->id < b->id ? -1 : (a->id > b->id ? 1 : 0);
}

static float sqdist_f32(const double* x, const float* c, int d) {
    float s = 0.0f;
    for (int t = 0; t < d; ++t) {
        float u = (float)x[t] - c[t];
        s = fmaf(u, u, s);
    }
    return s;
}

int orc_assign_blockwise(const double* X, int64_t n, int d, const double* C, int S, int omega,
                         double eps, double tau0, int64_t block_rows, int64_t cap, int adaptive,
                         int32_t* assign, int64_t* counts) {
    if (n < 0 || d <= 0 || S <= 0 || omega <= 0 || block_rows <= 0 || cap < 0 || tau0 < 1.0)
        return -1;
    float* Cf = (float*)malloc(sizeof(float) * (size_t)S * d);
    for (int64_t e = 0; e < (int64_t)S * d; ++e) Cf[e] = (float)C[e];
    int64_t* size = (int64_t*)calloc((size_t)S, sizeof(int64_t));
    int64_t* prim = (int64_t*)calloc((size_t)S, sizeof(int64_t));
    int64_t* rep = (int64_t*)calloc((size_t)S, sizeof(int64_t));
    int64_t* theta = (int64_t*)malloc(sizeof(int64_t) * S);
    float* R2 = (float*)calloc((size_t)S, sizeof(float));
    fcand_t* cs = (fcand_t*)malloc(sizeof(fcand_t) * (size_t)S * (size_t)(block_rows < n ? block_rows : (n > 0 ? n : 1)));
    int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * (size_t)(block_rows < n ? block_rows : (n > 0 ? n : 1)));
    const int accept_all = isinf(eps) && eps > 0;
    const float eps_f = (float)eps;
    const float eps2 = eps_f * eps_f;
    const float tau0_f = (float)tau0;
    for (int64_t b0 = 0, t = 1; b0 < n; b0 += block_rows, ++t) {
        const int64_t b1 = b0 + block_rows < n ? b0 + block_rows : n;
        /* visiting order of every row of the block */
        for (int64_t i = b0; i < b1; ++i) {
            fcand_t* ci = cs + (i - b0) * S;
            for (int c = 0; c < S; ++c) {
                ci[c].d2 = sqdist_f32(X + i * d, Cf + (int64_t)c * d, d);
                ci[c].id = c;
            }
            qsort(ci, (size_t)S, sizeof(fcand_t), fcand_cmp);
        }
        /* 1. primaries: nearest available cluster, in row order */
        for (int64_t i = b0; i < b1; ++i) {
            const fcand_t* ci = cs + (i - b0) * S;
            int k = 0;
            if (cap > 0) {
                while (k < S && size[ci[k].id] >= cap) ++k;
                if (k == S) k = 0;            /* every cluster full: the nearest */
            }
            const int c = ci[k].id;
            pos[i - b0] = k;
            size[c] += 1;
            prim[c] += 1;
            if (ci[k].d2 > R2[c]) R2[c] = ci[k].d2;
            int32_t* a = assign + i * omega;
            a[0] = c;
            for (int j = 1; j < omega; ++j) a[j] = ORC_NONE;
        }
        /* 2. thresholds and radius factor after the block's primaries */
        const int64_t seen = b1;
        for (int c = 0; c < S; ++c) {
            if (cap == 0 || !adaptive) {
                theta[c] = INT64_MAX;
            } else {
                const int64_t expect = (prim[c] * n + seen - 1) / seen;   /* ceil(prim * n / seen) */
                theta[c] = cap - expect > 0 ? cap - expect : 0;
            }
        }
        const float tau_t = 1.0f + (tau0_f - 1.0f) / (float)t;
        const float et2 = eps2 * (tau_t * tau_t);
        /* 3. replicas (Algorithm 1), in row order */
        for (int64_t i = b0; i < b1; ++i) {
            const fcand_t* ci = cs + (i - b0) * S;
            int32_t* a = assign + i * omega;
            const int c = a[0];
            const float dc2 = ci[pos[i - b0]].d2;
            int assigned = 1;
            for (int k = 0; k < S && assigned < omega; ++k) {
                const int cc = ci[k].id;
                if (cc == c) continue;
                if (cap > 0 && size[cc] >= cap) continue;          /* checkSizeLimit */
                if (rep[cc] >= theta[cc]) continue;
                const float dp2 = ci[k].d2;
                if (accept_all || (dp2 < eps2 * dc2 && dp2 < et2 * R2[cc])) {
                    a[assigned++] = cc;
                    size[cc] += 1;
                    rep[cc] += 1;
                }
            }
        }
    }
    for (int c = 0; c < S; ++c) counts[c] = size[c];
    free(Cf);
    free(size);
    free(prim);
    free(rep);
    free(theta);
    free(R2);
    free(cs);
    free(pos);
    return 0;
}

int orc_membership(const int32_t* assign, int64_t n, int omega, int S, int64_t* off,
                   int32_t* member_ids) {
    if (n < 0 || omega <= 0 || S <= 0) return -1;
    for (int s = 0; s <= S; ++s) off[s] = 0;
    for (int64_t k = 0; k < n * omega; ++k) {
        int32_t s = assign[k];
        if (s == ORC_NONE) continue;
        if (s < 0 || s >= S) return -1;
        off[s + 1] += 1;
    }
    for (int s = 0; s < S; ++s) off[s + 1] += off[s];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * S);
    for (int s = 0; s < S; ++s) fill[s] = off[s];
    for (int64_t i = 0; i < n; ++i)           /* ascending i gives ascending member lists */
        for (int k = 0; k < omega; ++k) {
            int32_t s = assign[i * omega + k];
            if (s != ORC_NONE) member_ids[fill[s]++] = (int32_t)i;
        }
    free(fill);
    return 0;
}

/* ------------------------------------------------------------------ */
/* greedy search                                                       */
/* ------------------------------------------------------------------ */

int64_t orc_medoid(const double* X, int64_t n, int d) {
    if (n <= 0) return -1;
    double* mean = (double*)calloc((size_t)d, sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        for (int t = 0; t < d; ++t) mean[t] += X[i * d + t];
    for (int t = 0; t < d; ++t) mean[t] /= (double)n;
    int64_t best = 0;
    double bd = delta(X, mean, d, ORC_L2);
    for (int64_t i = 1; i < n; ++i) {
        double v = delta(X + i * d, mean, d, ORC_L2);
        if (v < bd) {
            bd = v;
            best = i;
        }
    }
    free(mean);
    return best;
}

int orc_search(const double* X, int64_t n, int d, int metric, const int32_t* graph,
               int max_degree, const double* Q, int64_t nq, int topk, int L, int64_t entry,
               int32_t* out_ids, double* out_dist) {
    if (n <= 0 || d <= 0 || topk <= 0 || L < topk || max_degree <= 0) return -1;
    if (entry < 0) entry = orc_medoid(X, n, d);
    if (entry >= n) return -1;
#pragma omp parallel
    {
        cand_t* beam = (cand_t*)malloc(sizeof(cand_t) * (L + 1));
        char* expanded = (char*)malloc((size_t)L + 1);
        unsigned char* visited = (unsigned char*)malloc((size_t)n);
#pragma omp for schedule(dynamic, 4)
        for (int64_t qi = 0; qi < nq; ++qi) {
            const double* q = Q + qi * d;
            memset(visited, 0, (size_t)n);
            int size = 1;
            beam[0].dist = delta(q, X + entry * d, d, metric);
            beam[0].id = entry;
            expanded[0] = 0;
            visited[entry] = 1;
            for (;;) {
                int k = 0;
                while (k < size && expanded[k]) ++k;
                if (k == size) break;
                expanded[k] = 1;
                int64_t v = beam[k].id;
                for (int e = 0; e < max_degree; ++e) {
                    int32_t u = graph[v * max_degree + e];
                    if (u == ORC_NONE || u < 0 || u >= n) continue;
                    if (visited[u]) continue;
                    visited[u] = 1;
                    cand_t c;
                    c.dist = delta(q, X + (int64_t)u * d, d, metric);
                    c.id = u;
                    if (size == L && cand_cmp(&c, &beam[L - 1]) >= 0) continue;
                    /* sorted insertion; the last entry falls off when full */
                    int pos = size < L ? size : L - 1;
                    while (pos > 0 && cand_cmp(&c, &beam[pos - 1]) < 0) {
                        beam[pos] = beam[pos - 1];
                        expanded[pos] = expanded[pos - 1];
                        --pos;
                    }
                    beam[pos] = c;
                    expanded[pos] = 0;
                    if (size < L) ++size;
                }
            }
            for (int t = 0; t < topk; ++t) {
                out_ids[qi * topk + t] = t < size ? (int32_t)beam[t].id : ORC_NONE;
                if (out_dist) out_dist[qi * topk + t] = t < size ? beam[t].dist : INFINITY;
            }
        }
        free(beam);
        free(expanded);
        free(visited);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* re-rank                                                             */
/* ------------------------------------------------------------------ */

int orc_rerank(const double* X, int64_t n, int d, int metric, const int32_t* cand, int c, int K,
               int32_t* nbr, double* dist) {
    if (n < 0 || d <= 0 || c <= 0 || K <= 0) return -1;
    int bad = 0;
#pragma omp parallel
    {
        cand_t* cs = (cand_t*)malloc(sizeof(cand_t) * c);
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            int m = 0;
            for (int e = 0; e < c; ++e) {
                int32_t j = cand[i * c + e];
                if (j == ORC_NONE || j == i) continue;   /* self excluded by index */
                if (j < 0 || j >= n) {
                    bad = 1;
                    continue;
                }
                int dup = 0;
                for (int u = 0; u < m; ++u)
                    if (cs[u].id == j) dup = 1;
                if (dup) continue;
                cs[m].dist = delta(X + i * d, X + (int64_t)j * d, d, metric);
                cs[m].id = j;
                ++m;
            }
            qsort(cs, (size_t)m, sizeof(cand_t), cand_cmp);
            for (int k = 0; k < K; ++k) {
                nbr[i * K + k] = k < m ? (int32_t)cs[k].id : ORC_NONE;
                if (dist) dist[i * K + k] = k < m ? cs[k].dist : INFINITY;
            }
        }
        free(cs);
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* number formats                                                      */
/* ------------------------------------------------------------------ */

int orc_to_bf16(const float* x, int64_t n, uint16_t* out) {
    for (int64_t i = 0; i < n; ++i) {
        uint32_t b;
        memcpy(&b, &x[i], 4);
        if (isnan(x[i])) {
            out[i] = (uint16_t)((b >> 16) | 0x0040);
            continue;
        }
        /* keep the upper 16 bits, rounding the dropped 16 to nearest even */
        uint32_t lower = b & 0xffffu;
        uint32_t upper = b >> 16;
        if (lower > 0x8000u || (lower == 0x8000u && (upper & 1u))) upper += 1;
        out[i] = (uint16_t)upper;
    }
    return 0;
}

int orc_from_bf16(const uint16_t* x, int64_t n, double* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = bf16_to_double(x[i]);
    return 0;
}

/* round a non-negative value to the nearest integer, ties to even */
static double rne(double v) {
    double f = floor(v);
    double r = v - f;
    if (r > 0.5) return f + 1.0;
    if (r < 0.5) return f;
    return fmod(f, 2.0) == 0.0 ? f : f + 1.0;
}

static uint8_t fp8_encode(double v) {
    uint8_t sign = 0;
    if (isnan(v)) return 0x7f;
    if (v < 0 || (v == 0 && signbit(v))) {
        sign = 0x80;
        v = -v;
    }
    if (v >= 448.0) return sign | 0x7e;         /* saturate to the largest finite */
    /* E4M3: normal values 2^(e-7) * (1 + m/8), e in 1..15; subnormals m * 2^-9 */
    if (v < ldexp(1.0, -6)) {
        double q = rne(v / ldexp(1.0, -9));      /* 0..8; 8 is the smallest normal */
        return sign | (uint8_t)q;
    }
    int e;
    frexp(v, &e);                                /* v = f * 2^e, f in [0.5, 1) */
    int ex = e - 1;                              /* v in [2^ex, 2^(ex+1)) */
    double mant = v / ldexp(1.0, ex);            /* [1, 2) */
    double mq = rne((mant - 1.0) * 8.0);         /* 0..8 */
    if (mq == 8.0) {
        mq = 0.0;
        ex += 1;
    }
    int code = ((ex + 7) << 3) | (int)mq;
    if (code > 0x7e) code = 0x7e;
    return sign | (uint8_t)code;
}

static double fp8_decode(uint8_t c) {
    int sign = c >> 7;
    int e = (c >> 3) & 0xf;
    int m = c & 7;
    double v;
    if (e == 15 && m == 7) return NAN;
    if (e == 0)
        v = ldexp((double)m, -9);
    else
        v = ldexp(1.0 + m / 8.0, e - 7);
    return sign ? -v : v;
}

int orc_to_fp8e4m3(const float* x, int64_t n, uint8_t* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = fp8_encode((double)x[i]);
    return 0;
}

int orc_from_fp8e4m3(const uint8_t* x, int64_t n, double* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = fp8_decode(x[i]);
    return 0;
}

int orc_quant_rows_fp8(const float* X, int64_t n, int d, uint8_t* q, float* scale) {
    if (n < 0 || d <= 0) return -1;
    for (int64_t i = 0; i < n; ++i) {
        double amax = 0.0;
        for (int t = 0; t < d; ++t) {
            double a = fabs((double)X[i * d + t]);
            if (a > amax) amax = a;
        }
        double s = 1.0;
        if (amax > 0.0) s = ldexp(1.0, (int)ceil(log2(amax / 448.0)));
        /* the exponent must make amax/s <= 448 even when log2 rounds */
        while (amax / s > 448.0) s *= 2.0;
        scale[i] = (float)s;
        for (int t = 0; t < d; ++t) q[i * d + t] = fp8_encode((double)X[i * d + t] / s);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* learned proposer (MLP) forward / backward / Adam                    */
/* ------------------------------------------------------------------ */

static double gelu(double x) { return 0.5 * x * (1.0 + erf(x / sqrt(2.0))); }

static double gelu_grad(double x) {
    const double inv_sqrt_2pi = 0.39894228040143267794;
    return 0.5 * (1.0 + erf(x / sqrt(2.0))) + x * inv_sqrt_2pi * exp(-0.5 * x * x);
}

/* forward for one row, keeping intermediates: h1 (H), h2 (E), f (E) */
static void mlp_row(const double* x, int D, int H, int E, const double* W1, const double* b1,
                    const double* W2, const double* b2, const double* mu, double sigma,
                    double* z, double* h1, double* h2, double* f, double* nrm) {
    for (int t = 0; t < D; ++t) z[t] = (x[t] - mu[t]) / sigma;
    for (int u = 0; u < H; ++u) {
        double s = b1[u];
        for (int t = 0; t < D; ++t) s += W1[(int64_t)u * D + t] * z[t];
        h1[u] = s;
    }
    double nn = 0.0;
    for (int e = 0; e < E; ++e) {
        double s = b2[e];
        for (int u = 0; u < H; ++u) s += W2[(int64_t)e * H + u] * gelu(h1[u]);
        h2[e] = s;
        nn += s * s;
    }
    *nrm = sqrt(nn);
    for (int e = 0; e < E; ++e) f[e] = h2[e] / *nrm;
}

int orc_mlp_forward(const double* X, int64_t n, int D, int H, int E, const double* W1,
                    const double* b1, const double* W2, const double* b2, const double* mu,
                    double sigma, double* F) {
    if (n < 0 || D <= 0 || H <= 0 || E <= 0 || !(sigma > 0)) return -1;
#pragma omp parallel
    {
        double* z = (double*)malloc(sizeof(double) * D);
        double* h1 = (double*)malloc(sizeof(double) * H);
        double* h2 = (double*)malloc(sizeof(double) * E);
        double nrm;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            mlp_row(X + i * D, D, H, E, W1, b1, W2, b2, mu, sigma, z, h1, h2, F + i * E, &nrm);
        free(z);
        free(h1);
        free(h2);
    }
    return 0;
}

int orc_mlp_loss_grad(const double* Xa, const double* Xp, int64_t B, int D, int H, int E,
                      const double* W1, const double* b1, const double* W2, const double* b2,
                      const double* mu, double sigma, double T, double* loss, double* gW1,
                      double* gb1, double* gW2, double* gb2) {
    if (B <= 0 || D <= 0 || H <= 0 || E <= 0 || !(sigma > 0) || !(T > 0)) return -1;
    int64_t R2 = 2 * B;                          /* rows 0..B-1 anchors, B..2B-1 positives */
    double* Z = (double*)malloc(sizeof(double) * R2 * D);
    double* H1 = (double*)malloc(sizeof(double) * R2 * H);
    double* H2 = (double*)malloc(sizeof(double) * R2 * E);
    double* Fm = (double*)malloc(sizeof(double) * R2 * E);
    double* NR = (double*)malloc(sizeof(double) * R2);
    for (int64_t r = 0; r < R2; ++r) {
        const double* x = r < B ? Xa + r * D : Xp + (r - B) * D;
        mlp_row(x, D, H, E, W1, b1, W2, b2, mu, sigma, Z + r * D, H1 + r * H, H2 + r * E,
                Fm + r * E, &NR[r]);
    }
    /* logits and softmax cross-entropy, target of row i is column i */
    double* G = (double*)malloc(sizeof(double) * B * B);  /* dL/dlogit */
    double L = 0.0;
    for (int64_t i = 0; i < B; ++i) {
        double mx = -INFINITY;
        for (int64_t j = 0; j < B; ++j) {
            double s = 0.0;
            for (int e = 0; e < E; ++e) s += Fm[i * E + e] * Fm[(B + j) * E + e];
            G[i * B + j] = s / T;
            if (G[i * B + j] > mx) mx = G[i * B + j];
        }
        double se = 0.0;
        for (int64_t j = 0; j < B; ++j) se += exp(G[i * B + j] - mx);
        double lse = mx + log(se);
        L += lse - G[i * B + i];
        for (int64_t j = 0; j < B; ++j) {
            double p = exp(G[i * B + j] - lse);
            G[i * B + j] = (p - (i == j ? 1.0 : 0.0)) / (double)B;
        }
    }
    *loss = L / (double)B;
    /* dL/df for anchors and positives */
    double* dF = (double*)calloc((size_t)(R2 * E), sizeof(double));
    for (int64_t i = 0; i < B; ++i)
        for (int64_t j = 0; j < B; ++j) {
            double g = G[i * B + j] / T;
            for (int e = 0; e < E; ++e) {
                dF[i * E + e] += g * Fm[(B + j) * E + e];
                dF[(B + j) * E + e] += g * Fm[i * E + e];
            }
        }
    memset(gW1, 0, sizeof(double) * (size_t)H * D);
    memset(gb1, 0, sizeof(double) * H);
    memset(gW2, 0, sizeof(double) * (size_t)E * H);
    memset(gb2, 0, sizeof(double) * E);
    double* dh2 = (double*)malloc(sizeof(double) * E);
    double* dh1 = (double*)malloc(sizeof(double) * H);
    for (int64_t r = 0; r < R2; ++r) {
        const double* f = Fm + r * E;
        const double* df = dF + r * E;
        /* through f = h2 / ||h2||:  dh2 = (df - f (f . df)) / ||h2|| */
        double fd = 0.0;
        for (int e = 0; e < E; ++e) fd += f[e] * df[e];
        for (int e = 0; e < E; ++e) dh2[e] = (df[e] - f[e] * fd) / NR[r];
        for (int e = 0; e < E; ++e) {
            gb2[e] += dh2[e];
            for (int u = 0; u < H; ++u) gW2[(int64_t)e * H + u] += dh2[e] * gelu(H1[r * H + u]);
        }
        for (int u = 0; u < H; ++u) {
            double s = 0.0;
            for (int e = 0; e < E; ++e) s += W2[(int64_t)e * H + u] * dh2[e];
            dh1[u] = s * gelu_grad(H1[r * H + u]);
        }
        for (int u = 0; u < H; ++u) {
            gb1[u] += dh1[u];
            for (int t = 0; t < D; ++t) gW1[(int64_t)u * D + t] += dh1[u] * Z[r * D + t];
        }
    }
    free(Z);
    free(H1);
    free(H2);
    free(Fm);
    free(NR);
    free(G);
    free(dF);
    free(dh2);
    free(dh1);
    return 0;
}

int orc_adam(double* w, const double* g, double* m, double* v, int64_t n, double lr,
             double beta1, double beta2, double eps, int64_t step) {
    if (n < 0 || step <= 0) return -1;
    double c1 = 1.0 - pow(beta1, (double)step);
    double c2 = 1.0 - pow(beta2, (double)step);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        double mh = m[i] / c1;
        double vh = v[i] / c2;
        w[i] -= lr * mh / (sqrt(vh) + eps);
    }
    return 0;
}

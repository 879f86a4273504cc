// knn.hip -- exact (and reduced-precision) kNN graph of one shard.
//
// The shard build of Sec. IV step 2 as a tiled all-pairs distance contraction
// (the dense-product formulation named in Sec. II-A) fused with a per-row
// top-k selection, for gfx950:
//
//  * prep: rows -> MFMA operand rows (FP32 / FP16 / BF16 / FP8 with a
//    power-of-two per-row scale), zero-padded to the k granule, plus the
//    squared norms of the operand rows (NaN for padding rows, never admitted).
//  * locality order (shards of >= 4096 rows): rows grouped by their nearest of
//    about n/256 evenly spaced pivot rows (a stable sort: ascending row order
//    within a pivot, so the order returned is the same on every run).
//  * dist_topk: a workgroup (a launch shape: 8 waves x 32 queries, or 4 waves
//    with 64- or 32-row candidate tiles, chosen by the autotuner) owns a block
//    of query rows, each wave 32 of them held in registers, and streams every
//    candidate row of the shard through LDS in double-buffered tiles (the
//    next tile already loading into registers while the current one is
//    computed), first the tiles of its own pivot group, then all others in
//    one shared order.  Each 32x32 MFMA output tile holds candidates on its
//    rows and queries on its columns, so every lane sees 16 candidates of
//    ONE query and keeps that query's admission threshold in a register.  The
//    accumulator starts at ||c||^2 and the query operand is pre-scaled by -2
//    (exact), so the MFMA result is already the ranking key ||c||^2 - 2 q.c
//    (L2) or -q.c (IP).  Keys at or below the threshold go to a 16- or
//    32-entry LDS buffer per query; a full buffer is merged in registers (wave
//    bitonic sort + bitonic merge) into the query's sorted top-K list of
//    (distance, id) keys in the workspace, which lowers the threshold.
//    Admission is exact in any candidate order: a candidate farther than the
//    K-th distance of a subset already seen cannot be in the top K, and one
//    at exactly that distance is admitted (the comparison is <=) and ranked by
//    (distance, id) in the merge.  The query itself (by index) and padding
//    rows carry NaN keys, which no comparison admits.
//  * rerank: the top-c candidates of a reduced-precision key re-scored with
//    the exact FP32 difference-form distance, best k kept.
#include "knn_impl.hpp"

namespace sg {
namespace knn {

// ||c'||^2 = -2 (e >> 1) + (e & 1) from the INT8 L2 start word e.
__global__ void i8_norms_kernel(float* __restrict__ v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t e = __builtin_bit_cast(int32_t, v[i]);
        v[i] = (float)(-2 * (e >> 1) + (e & 1));
    }
}

std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;
thread_local int g_force_variant = -1;

int chosen_variant(int prec, int d, int ksel, int64_t n, int count) {
    int idx = 0;
    if (g_force_variant >= 0) {
        idx = g_force_variant < count ? g_force_variant : 0;
    } else {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune.find(tune_key(prec, d, ksel, n));
        if (it != g_tune.end() && it->second < count) idx = it->second;
    }
    return idx;
}

Kern choose_kernel(int prec, int d, int ksel, int64_t n) {
    const std::vector<Kern> v = kernel_variants(prec, d, ksel);
    if (v.empty()) return Kern();
    return v[chosen_variant(prec, d, ksel, n, (int)v.size())];
}

}  // namespace knn
}  // namespace sg

using namespace sg;

extern "C" sg_status sg_knn_graph_workspace_size(int64_t n, int32_t d, int32_t k, sg_prec prec,
                                                 int32_t rerank, size_t* bytes) {
    return guarded([&] {
        SG_REQUIRE(bytes != nullptr, "bytes is NULL");
        SG_REQUIRE(n >= 0 && d >= 1 && d <= 1024 && k >= 1 && k <= 256, "bad sizes");
        knn::Layout L = knn::layout_k(n, d, k, prec, rerank == k ? 0 : rerank);
        *bytes = n == 0 ? 0 : knn::total_bytes(L, n, -1, prec);
    });
}

namespace sg {
namespace knn {

// kNN of rows (nq >= 0: the listed rows; nq < 0: every row) against all n rows.
void run(const void* X, int dtype, int64_t n, int d, int64_t ld, int metric, int k, int prec,
         int rerank, const int64_t* rows, int64_t nq, int32_t* nbr, float* dist, void* ws,
         size_t ws_bytes, hipStream_t s, int32_t* order_out = nullptr) {
    if (rerank == k) rerank = 0;
    Layout L = layout_k(n, d, k, prec, rerank);
    const Kern kern = choose_kernel(prec, d, L.ksel, n);
    if (!kern.fn && !kern.ks) {
        set_error("sg_knn: no distance kernel for this precision at d = " + std::to_string(d));
        throw Fail{SG_ERR_UNSUPPORTED};
    }
    const bool subset = rows != nullptr;
    const size_t need = total_bytes(L, n, subset ? nq : -1, prec);
    if (ws_bytes < need || ws == nullptr) {
        set_error("sg_knn: workspace too small (need " + std::to_string(need) + " bytes)");
        throw Fail{SG_ERR_WORKSPACE};
    }
    const bool local = use_locality(n, subset) && kern.near != nullptr;
    const int64_t nq_rows = subset ? nq : n;
    const int64_t nq_pad = subset ? pad_rows(nq) : L.n_pad;
    Carver cv(ws);
    uint8_t* ops = cv.take<uint8_t>(L.ops_bytes);
    float* ninit = cv.take<float>(L.n_pad);
    float* nout = cv.take<float>(L.n_pad);
    int32_t* sexp = prec == SG_PREC_FP8 ? cv.take<int32_t>(L.n_pad) : nullptr;
    uint8_t* qops = ops;
    float* qninit = ninit;
    float* qnout = nout;
    int32_t* qsexp = sexp;
    const int64_t* qid = nullptr;
    if (subset) {
        qops = cv.take<uint8_t>((size_t)nq_pad * L.DP * elem_bytes(prec));
        qninit = cv.take<float>(nq_pad);
        qnout = cv.take<float>(nq_pad);
        qsexp = cv.take<int32_t>(nq_pad);
        int64_t* qid_w = cv.take<int64_t>(nq_pad);
        fill<int64_t>(qid_w, -1, nq_pad, s);
        SG_HIP(hipMemcpyAsync(qid_w, rows, nq * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
        qid = qid_w;
    }
    uint64_t* state = cv.take<uint64_t>((size_t)nq_pad * L.ksel);
    const bool plain_ip = metric == SG_IP && !norm_corrected_ip(metric, prec);
    const float qmul = plain_ip ? -1.0f : -2.0f;
    const float osc = norm_corrected_ip(metric, prec) ? 0.5f : 1.0f;

    int64_t* perm = nullptr;
    int32_t* pid = nullptr;
    if (local) {
        const int64_t P = n_pivots(n), Pp = pad_rows(P);
        perm = cv.take<int64_t>(L.n_pad);
        pid = cv.take<int32_t>(L.n_pad);
        int32_t* lab = cv.take<int32_t>(L.n_pad);
        void* sort_tmp = cv.take<char>(label_sort_tmp_bytes(n, bits_for(P)));
        uint8_t* pops = cv.take<uint8_t>((size_t)Pp * L.DP * elem_bytes(prec));
        float* pinit = cv.take<float>(Pp);
        float* pnout = cv.take<float>(Pp);
        int32_t* psexp = cv.take<int32_t>(Pp);
        int64_t* piv = cv.take<int64_t>(P);
        // nearest pivot of every row (queries: all rows in their own order)
        pivot_rows_kernel<<<(unsigned)cdiv(P, 256), 256, 0, s>>>(piv, P, n);
        SG_LAUNCH_CHECK();
        launch_prep(X, dtype, P, d, ld, piv, n, Pp, L.DP, prec, metric,
                    pops, pinit, pnout, prec == SG_PREC_FP8 ? psexp : nullptr, s);
        SG_LAUNCH_CHECK();
        launch_prep(X, dtype, n, d, ld, nullptr, n, L.n_pad, L.DP, prec, metric, ops,
                    ninit, nout, sexp, s);
        SG_LAUNCH_CHECK();
        kern.near<<<(unsigned)(L.n_pad / (32 * NEAR_WAVES)), NEAR_WAVES * 64, 0, s>>>(
            pops, pinit, prec == SG_PREC_FP8 ? psexp : nullptr, (int)P, ops, sexp, (int)n, qmul, lab);
        SG_LAUNCH_CHECK();
        // group the rows by pivot, ascending row order within a pivot (stable)
        label_sort(lab, n, bits_for(P), pid, sort_tmp, s);
        const unsigned eg = (unsigned)std::min<int64_t>(cdiv(L.n_pad, 256), 4096);
        rows_to_perm_kernel<<<eg, 256, 0, s>>>(pid, n, L.n_pad, perm, pid);
        SG_LAUNCH_CHECK();
    }

    launch_prep(X, dtype, n, d, ld, perm, n, L.n_pad, L.DP, prec, metric, ops, ninit,
                nout, sexp, s);
    SG_LAUNCH_CHECK();
    if (order_out && !subset) {   // the rows in the order the build visits them
        if (pid)
            SG_HIP(hipMemcpyAsync(order_out, pid, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        else
            iota32_kernel<<<(unsigned)std::min<int64_t>(cdiv(n, 256), 4096), 256, 0, s>>>(order_out, n);
        SG_LAUNCH_CHECK();
    }
    if (subset) {
        launch_prep(X, dtype, nq, d, ld, rows, n, nq_pad, L.DP, prec,
                    metric, qops, qninit, qnout, qsexp, s);
        SG_LAUNCH_CHECK();
    }
    // (the resident-query kernels write every list themselves)
    if (!kern.fn) fill<uint64_t>(state, EMPTY_KEY, nq_pad * L.ksel, s);
    const bool final_here = rerank == 0;
    TopkArgs A{};
    A.ops = ops; A.ninit = ninit; A.sexp = sexp; A.cpid = pid; A.n = (int)n;
    A.qops = qops; A.qid = qid; A.qnout = qnout; A.qsexp = qsexp; A.qout = perm; A.nq = (int)nq_rows;
    A.qmul = qmul; A.osc = osc; A.state = state;
    A.nbr = final_here ? nbr : nullptr; A.dist = final_here ? dist : nullptr; A.k_out = k;
    profile_record(s, true);
    launch_topk(kern, A, nq_pad, L.DP, s);
    profile_record(s, false);
    if (!final_here && nbr)   // (no lists wanted when only timing the distance kernel)
        launch_rerank<uint64_t>(X, dtype, nq_rows, d, ld, metric, subset ? rows : perm, n, state, L.ksel, rerank, k,
                                nbr, dist, perm, s);
}

}  // namespace knn
}  // namespace sg

extern "C" sg_status sg_knn_graph(const void* X, sg_dtype dtype, int64_t n, int32_t d, int64_t ld,
                                  sg_metric metric, int32_t k, sg_prec prec, int32_t rerank,
                                  int32_t* nbr, float* dist, int32_t* order, void* ws, size_t ws_bytes,
                                  void* stream) {
    return guarded([&] {
        knn::check_args(X, dtype, n, d, ld, metric, k, prec, rerank);
        SG_REQUIRE(nbr != nullptr || n == 0, "nbr is NULL");
        if (n == 0) return;
        knn::run(X, dtype, n, d, ld, metric, k, prec, rerank, nullptr, -1, nbr, dist, ws, ws_bytes,
                 as_stream(stream), order);
    });
}

extern "C" sg_status sg_knn_rows_workspace_size(int64_t n, int32_t d, int64_t nq, int32_t k, sg_prec prec,
                                                int32_t rerank, size_t* bytes) {
    return guarded([&] {
        SG_REQUIRE(bytes != nullptr, "bytes is NULL");
        SG_REQUIRE(n >= 0 && nq >= 0 && d >= 1 && d <= 1024 && k >= 1 && k <= 256, "bad sizes");
        if (rerank == k) rerank = 0;
        knn::Layout L = knn::layout_k(n, d, k, prec, rerank);
        *bytes = (n == 0 || nq == 0) ? 0 : knn::total_bytes(L, n, nq, prec);
    });
}

extern "C" sg_status sg_knn_rows(const void* X, sg_dtype dtype, int64_t n, int32_t d, int64_t ld,
                                 sg_metric metric, const int64_t* rows, int64_t nq, int32_t k,
                                 sg_prec prec, int32_t rerank, int32_t* nbr, float* dist, void* ws,
                                 size_t ws_bytes, void* stream) {
    return guarded([&] {
        knn::check_args(X, dtype, n, d, ld, metric, k, prec, rerank);
        SG_REQUIRE(nq >= 0 && nq <= MAX_ROWS, "nq out of range (at most 2^26 - 1024 rows)");
        if (n == 0 || nq == 0) return;
        SG_REQUIRE(rows != nullptr && nbr != nullptr, "NULL pointer");
        knn::run(X, dtype, n, d, ld, metric, k, prec, rerank, rows, nq, nbr, dist, ws, ws_bytes,
                 as_stream(stream));
    });
}

extern "C" sg_status sg_rerank(const void* X, sg_dtype dtype, int64_t n, int32_t d, int64_t ld, sg_metric metric,
                               const int32_t* cand, int32_t c, int32_t k, int32_t* nbr, float* dist,
                               void* stream) {
    return guarded([&] {
        SG_REQUIRE(n >= 0 && n <= MAX_ROWS, "n out of range (at most 2^26 - 1024 rows)");
        SG_REQUIRE(d >= 1 && d <= 1024 && ld >= d, "bad d / ld (d <= 1024)");
        SG_REQUIRE(c >= 1 && c <= 256 && k >= 1 && k <= c, "need 1 <= k <= c <= 256");
        SG_REQUIRE(metric == SG_L2 || metric == SG_IP, "unknown metric");
        SG_REQUIRE(dtype >= SG_F32 && dtype <= SG_U8, "unknown dtype");
        if (n == 0) return;
        SG_REQUIRE(X && cand && nbr, "NULL pointer");
        knn::launch_rerank<int32_t>(X, dtype, n, d, ld, metric, nullptr, n, cand, c, c, k, nbr, dist, nullptr,
                                    as_stream(stream));
    });
}

extern "C" sg_status sg_knn_variant_count(sg_prec prec, int32_t d, int32_t k, int32_t* count) {
    return guarded([&] {
        SG_REQUIRE(count != nullptr, "count is NULL");
        SG_REQUIRE(d >= 1 && d <= 1024 && k >= 1 && k <= 256, "bad sizes");
        SG_REQUIRE(prec >= SG_PREC_FP32 && prec <= SG_PREC_I8, "unknown precision");
        *count = (int32_t)knn::kernel_variants(prec, d, knn::ksel_for(k)).size();
    });
}

extern "C" sg_status sg_knn_force_variant(int32_t variant) {
    return guarded([&] {
        SG_REQUIRE(variant >= -1, "variant must be -1 (off) or a variant index");
        knn::g_force_variant = variant;
    });
}

extern "C" sg_status sg_knn_autotune(const void* X, sg_dtype dtype, int64_t n, int32_t d, int64_t ld,
                                     sg_metric metric, int32_t k, sg_prec prec, int32_t rerank, void* ws,
                                     size_t ws_bytes, void* stream, int32_t* chosen, float* times_ms,
                                     int32_t max_times) {
    return guarded([&] {
        knn::check_args(X, dtype, n, d, ld, metric, k, prec, rerank);
        SG_REQUIRE(n > 0, "autotuning needs rows");
        SG_REQUIRE(max_times >= 0 && (max_times == 0 || times_ms != nullptr), "bad times_ms / max_times");
        hipStream_t s = as_stream(stream);
        const int ksel = knn::layout_k(n, d, k, prec, rerank == k ? 0 : rerank).ksel;
        const int nv = (int)knn::kernel_variants(prec, d, ksel).size();
        SG_REQUIRE(nv > 0, "no distance kernel for this precision and d");
        const int saved = knn::g_force_variant;
        std::vector<float> ms(nv, 0.f);
        hipEvent_t e0, e1;
        SG_HIP(hipEventCreate(&e0));
        SG_HIP(hipEventCreate(&e1));
        struct Restore {
            int v;
            hipEvent_t a, b;
            ~Restore() {
                knn::g_force_variant = v;
                (void)hipEventDestroy(a);
                (void)hipEventDestroy(b);
            }
        } restore{saved, e0, e1};
        // nbr / dist scratch inside the caller's workspace is not available,
        // so the timed runs keep only the state (no final lists)
        for (int v = 0; v < nv; ++v) {
            knn::g_force_variant = v;
            knn::run(X, dtype, n, d, ld, metric, k, prec, rerank, nullptr, -1, nullptr, nullptr, ws, ws_bytes, s);
            SG_HIP(hipEventRecord(e0, s));
            knn::run(X, dtype, n, d, ld, metric, k, prec, rerank, nullptr, -1, nullptr, nullptr, ws, ws_bytes, s);
            SG_HIP(hipEventRecord(e1, s));
            SG_HIP(hipEventSynchronize(e1));
            SG_HIP(hipEventElapsedTime(&ms[v], e0, e1));
        }
        int best = 0;
        for (int v = 1; v < nv; ++v)
            if (ms[v] < ms[best]) best = v;
        {
            std::lock_guard<std::mutex> g(knn::g_tune_mu);
            knn::g_tune[knn::tune_key(prec, d, ksel, n)] = best;
        }
        if (chosen) *chosen = best;
        for (int v = 0; v < nv && v < max_times; ++v) times_ms[v] = ms[v];
    });
}

extern "C" sg_status sg_knn_graph_learned_workspace_size(int64_t n, int32_t e, int32_t c, size_t* bytes) {
    return guarded([&] {
        SG_REQUIRE(bytes != nullptr, "bytes is NULL");
        SG_REQUIRE(n >= 0 && e >= 1 && e <= 1024 && c >= 1 && c <= 256, "bad sizes");
        if (n == 0) {
            *bytes = 0;
            return;
        }
        const knn::Layout L = knn::layout_k(n, e, c, SG_PREC_FP8, 0);
        *bytes = align_up((size_t)n * c * 4, 256) + knn::total_bytes(L, n, -1, SG_PREC_FP8);
    });
}

extern "C" sg_status sg_knn_graph_learned(const void* X, sg_dtype dtype, int32_t d, int64_t ld, sg_metric metric,
                                          const float* P, int64_t n, int32_t e, int64_t ldp, int32_t c, int32_t k,
                                          int32_t* nbr, float* dist, void* ws, size_t ws_bytes, void* stream) {
    return guarded([&] {
        knn::check_args(X, dtype, n, d, ld, metric, k, SG_PREC_FP32, 0);
        SG_REQUIRE(e >= 1 && e <= 1024 && ldp >= e, "bad e / ldp");
        SG_REQUIRE(c >= k && c <= 256, "need k <= c <= 256");
        SG_REQUIRE(n == 0 || (P != nullptr && nbr != nullptr), "NULL pointer");
        if (n == 0) return;
        const size_t cbytes = align_up((size_t)n * c * 4, 256);
        SG_REQUIRE(ws != nullptr && ws_bytes >= cbytes, "workspace too small");
        hipStream_t s = as_stream(stream);
        int32_t* cand = static_cast<int32_t*>(ws);
        knn::run(P, SG_F32, n, e, ldp, SG_IP, c, SG_PREC_FP8, 0, nullptr, -1, cand, nullptr,
                 static_cast<char*>(ws) + cbytes, ws_bytes - cbytes, s);
        knn::launch_rerank<int32_t>(X, dtype, n, d, ld, metric, nullptr, n, cand, c, c, k, nbr, dist, nullptr, s);
    });
}

extern "C" sg_status sg_quantize_rows(const void* X, sg_dtype dtype, int64_t n, int32_t d, int64_t ld,
                                      sg_prec prec, void* out, int64_t ldo, int32_t* scale_exp, float* sqnorm,
                                      void* stream) {
    return guarded([&] {
        knn::check_args(X, dtype, n, d, ld, SG_L2, 1, prec, 0);
        SG_REQUIRE(ldo >= d && ldo <= (int64_t(1) << 20), "ldo must be in d..2^20");
        if (n == 0) return;
        SG_REQUIRE(out != nullptr, "out is NULL");
        SG_REQUIRE(prec != SG_PREC_FP8 || scale_exp != nullptr, "FP8 needs scale_exp");
        hipStream_t s = as_stream(stream);
        knn::launch_prep(X, dtype, n, d, ld, nullptr, n, n, (int)ldo, prec,
                         SG_L2, static_cast<uint8_t*>(out), sqnorm, nullptr,
                         prec == SG_PREC_FP8 ? scale_exp : nullptr, s);
        SG_LAUNCH_CHECK();
        if (prec == SG_PREC_I8 && sqnorm) {   // the INT8 start word back to the squared norm
            knn::i8_norms_kernel<<<(unsigned)std::min<int64_t>(cdiv(n, 256), 4096), 256, 0, s>>>(sqnorm, n);
            SG_LAUNCH_CHECK();
        }
    });
}

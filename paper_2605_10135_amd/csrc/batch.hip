// batch.hip -- shard graphs of many shards in one pass (the batching form).
//
// The per-shard build of Sec. IV step 2 for all shards of one GPU at once:
// every step runs as one launch over all shards (operand preparation, the
// locality order, the distance + top-k kernel, the prune), so that small
// shards do not leave the GPU idle.  The distance kernel is persistent: a grid
// sized to the GPU's resident capacity takes (shard, query block) items from
// a device counter, largest shards first (longest-processing-time order, so
// that the tail is made of short items).  With a plan, the whole sequence is
// captured once into a HIP graph and later calls replay it with one launch.
#include <cstring>

#include "batch_impl.hpp"

struct sg_batch_plan {
    hipGraphExec_t exec = nullptr;
    std::vector<uint8_t> sig;   // the arguments the graph was captured with
    int device = -1;
};

namespace sg {
namespace batch {

using namespace knn;

// Row maps of the identity operand layout and of the pivots; the locality
// permutation starts empty (padding = -1).
__global__ void maps_kernel(Shards sh, int64_t* __restrict__ idmap, int64_t* __restrict__ perm,
                            int32_t* __restrict__ pid, int64_t* __restrict__ pivmap) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < sh.pad0[sh.S]; j += stride) {
        const int s = shard_of(sh.pad0, sh.S, j);
        const int64_t loc = j - sh.pad0[s], ns = sh.row0[s + 1] - sh.row0[s];
        idmap[j] = loc < ns ? sh.row0[s] + loc : -1;
        perm[j] = -1;
        pid[j] = -1;
    }
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < sh.ppad0[sh.S]; p += stride) {
        const int s = shard_of(sh.ppad0, sh.S, p);
        const int64_t lp = p - sh.ppad0[s], P = sh.piv0[s + 1] - sh.piv0[s];
        const int64_t ns = sh.row0[s + 1] - sh.row0[s];
        pivmap[p] = lp < P ? sh.row0[s] + lp * ns / P : -1;
    }
}

// Labels of the batch's rows in compact row order (row r of shard s is
// operand row pad0[s] + r - row0[s]); a label outside the shard's range is
// taken as the shard's first.
__global__ void compact_labels_kernel(Shards sh, const int32_t* __restrict__ lab, int32_t* __restrict__ labc) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < sh.row0[sh.S];
         r += (int64_t)gridDim.x * blockDim.x) {
        const int s = shard_of(sh.row0, sh.S, r);
        int64_t c = lab[sh.pad0[s] + r - sh.row0[s]];
        if (c < sh.piv0[s] || c >= sh.piv0[s + 1]) c = sh.piv0[s];
        labc[r] = (int32_t)c;
    }
}

// From the locality order over all rows (position -> row, sorted by global
// label, so the positions of shard s are row0[s]..row0[s+1]-1 because shard
// s's labels follow shard s-1's): the operand-layout maps of each shard.
__global__ void place_batched_kernel(Shards sh, const int32_t* __restrict__ order, int64_t* __restrict__ perm,
                                     int32_t* __restrict__ pid) {
    for (int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pos < sh.row0[sh.S];
         pos += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = order[pos];
        const int s = shard_of(sh.row0, sh.S, pos);
        const int64_t o = pos - sh.row0[s] + sh.pad0[s];
        perm[o] = r;
        pid[o] = r;
    }
}

// Batch-row ids -> shard-local ids, in place (SG_NONE stays).  A block's
// entries are consecutive, so their rows nearly always lie in one shard: it is
// found once per block, and per entry only where the block straddles a shard
// boundary.
__global__ void localize_kernel(Shards sh, int32_t* __restrict__ lists, int width) {
    const int64_t total = sh.row0[sh.S] * width;
    // four entries per work-item (one 16-byte load and store, all four in one
    // row) when rows are a multiple of four entries wide and the lists 16-byte
    // aligned, else one
    const int per = (width % 4 == 0 && (reinterpret_cast<uintptr_t>(lists) & 15) == 0) ? 4 : 1;
    const int64_t chunk = (int64_t)blockDim.x * per;
    for (int64_t e0 = (int64_t)blockIdx.x * chunk; e0 < total; e0 += (int64_t)gridDim.x * chunk) {
        const int64_t e = e0 + (int64_t)threadIdx.x * per;
        const int64_t e1 = (e0 + chunk < total ? e0 + chunk : total) - 1;
        const int s0 = shard_of(sh.row0, sh.S, e0 / width);
        const bool one = e1 / width < sh.row0[s0 + 1];
        if (e >= total) continue;
        const int64_t base = one ? sh.row0[s0] : sh.row0[shard_of(sh.row0, sh.S, e / width)];
        if (per == 4) {
            int4 v = *reinterpret_cast<const int4*>(lists + e);
            v.x = v.x >= 0 ? (int32_t)(v.x - base) : v.x;
            v.y = v.y >= 0 ? (int32_t)(v.y - base) : v.y;
            v.z = v.z >= 0 ? (int32_t)(v.z - base) : v.z;
            v.w = v.w >= 0 ? (int32_t)(v.w - base) : v.w;
            *reinterpret_cast<int4*>(lists + e) = v;
        } else {
            const int32_t v = lists[e];
            if (v >= 0) lists[e] = (int32_t)(v - base);
        }
    }
}

// Everything a call needs, derived from its arguments.
struct Plan {
    Shards sh{};
    int S = 0, ksel = 0, DP = 0, eb = 0, nitems = 0;
    int rerank = 0;   // FP32 re-rank width (0: none)
    int64_t n_all = 0, n_max = 0;
    BKern kern;
    size_t prune_bytes = 0, scan_bytes = 0, total = 0;
};

Plan make_plan(const int64_t* off, int S, int d, int k, int R, int prec, int rerank) {
    SG_REQUIRE(S >= 1 && S <= MAXS, "S must be in 1..64");
    SG_REQUIRE(off != nullptr, "offsets_h is NULL");
    SG_REQUIRE(off[0] == 0, "offsets_h[0] must be 0");
    SG_REQUIRE(d >= 1 && d <= 1024, "d out of range");
    SG_REQUIRE(k >= 1 && k <= 256, "k must be in 1..256");
    SG_REQUIRE(rerank == 0 || (rerank >= k && rerank <= 256), "rerank must be 0 or in k..256");
    SG_REQUIRE(R >= 1 && R <= k && R <= 128, "R must be in 1..min(k, 128)");
    SG_REQUIRE(prec >= SG_PREC_FP32 && prec <= SG_PREC_I8, "unknown precision");
    Plan p;
    p.S = S;
    p.sh.S = S;
    p.rerank = rerank == k ? 0 : rerank;
    p.ksel = std::max(64, ksel_for(p.rerank > 0 ? p.rerank : k));
    for (int s = 0; s < S; ++s) {
        SG_REQUIRE(off[s + 1] >= off[s], "offsets_h must be non-decreasing");
        SG_REQUIRE(off[s + 1] - off[s] < (int64_t(1) << 31), "shard too large");
    }
    SG_REQUIRE(off[S] + (int64_t)S * PAD_ROWS <= MAX_ROWS, "too many rows in the batch (at most 2^26 - 1024 with padding)");
    std::vector<BKern> kv;
    SG_REQUIRE(batched_shapes(prec, d, p.ksel, kv), "no register-resident distance kernel for this precision and d");
    int64_t pad = 0, piv = 0, ppad = 0;
    for (int s = 0; s < S; ++s) {
        const int64_t ns = off[s + 1] - off[s];
        p.sh.row0[s] = off[s];
        p.sh.pad0[s] = pad;
        p.sh.piv0[s] = piv;
        p.sh.ppad0[s] = ppad;
        pad += pad_rows(ns);
        const int64_t P = ns > 0 ? n_pivots(ns) : 0;
        piv += P;
        ppad += pad_rows(P);
        p.n_max = std::max(p.n_max, ns);
    }
    p.sh.row0[S] = off[S];
    p.sh.pad0[S] = pad;
    p.sh.piv0[S] = piv;
    p.sh.ppad0[S] = ppad;
    p.n_all = off[S];
    // the launch shape: a forced one, else the choice recorded for batched
    // passes of this shape (sg_knn_graph_batched_autotune), else the choice
    // recorded for single-shard builds of the largest shard's size
    int idx = -1;
    if (g_force_variant >= 0) {
        idx = g_force_variant < (int)kv.size() ? g_force_variant : 0;
    } else {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune.find(batched_tune_key(prec, d, p.ksel, p.n_max));
        if (it != g_tune.end() && it->second < (int)kv.size()) idx = it->second;
    }
    if (idx < 0) idx = chosen_variant(prec, d, p.ksel, p.n_max, (int)kv.size());
    p.kern = kv[idx];
    p.DP = p.kern.DP;
    p.eb = elem_bytes(prec);
    // work items: shards by descending size (ties by index), blocks of nq_block rows
    std::vector<int> ord(S);
    for (int s = 0; s < S; ++s) ord[s] = s;
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int a, int b) { return off[a + 1] - off[a] > off[b + 1] - off[b]; });
    int64_t items = 0;
    for (int k2 = 0; k2 < S; ++k2) {
        p.sh.order[k2] = ord[k2];
        p.sh.item0[k2] = (int32_t)items;
        items += (p.sh.pad0[ord[k2] + 1] - p.sh.pad0[ord[k2]]) / p.kern.nq_block;
    }
    p.sh.item0[S] = (int32_t)items;
    SG_REQUIRE(items < (int64_t(1) << 31), "too many work items");
    p.nitems = (int)items;
    size_t pb = 0;
    if (sg_prune_workspace_size(p.n_all, k, R, &pb) != SG_OK) throw Fail{SG_ERR_INTERNAL};
    p.prune_bytes = pb;
    p.scan_bytes = label_sort_tmp_bytes(p.n_all, bits_for(std::max<int64_t>(piv, 1)));
    const size_t P8 = align_up((size_t)pad * 8, 256), P4 = align_up((size_t)pad * 4, 256);
    const size_t Q8 = align_up((size_t)ppad * 8, 256), Q4 = align_up((size_t)ppad * 4, 256);
    p.total = align_up((size_t)pad * p.DP * p.eb, 256) + 3 * P4        // ops, ninit, nout, sexp
              + 2 * P8 + 2 * P4                                       // idmap, perm, pid, lab
              + Q8 + align_up((size_t)ppad * p.DP * p.eb, 256) + 3 * Q4   // pivots
              + align_up((size_t)p.n_all * 4, 256) + align_up(p.scan_bytes, 256)   // compact labels, label sort
              + align_up((size_t)pad * p.ksel * 8, 256)               // state
              + 256                                                   // counter
              + align_up((size_t)p.n_all * k * 4, 256)                // kNN lists (when not returned)
              + align_up((size_t)p.n_all * 4, 256)                    // locality order of the rows
              + align_up(p.prune_bytes, 256) + 1024;
    return p;
}

// Enqueue the whole build on s (no host synchronisation, no memset: valid
// inside a stream capture; the profiling events only when eager).
void enqueue(const Plan& p, const void* X, int dtype, int d, int64_t ld, int metric, int k, int R, int prec,
             int32_t* graphs, int32_t* knn_out, void* ws, hipStream_t s, bool eager) {
    const int64_t pad = p.sh.pad0[p.S], ppad = p.sh.ppad0[p.S], piv = p.sh.piv0[p.S];
    Carver cv(ws);
    uint8_t* ops = cv.take<uint8_t>((size_t)pad * p.DP * p.eb);
    float* ninit = cv.take<float>(pad);
    float* nout = cv.take<float>(pad);
    int32_t* sexp = cv.take<int32_t>(pad);
    int64_t* idmap = cv.take<int64_t>(pad);
    int64_t* perm = cv.take<int64_t>(pad);
    int32_t* pid = cv.take<int32_t>(pad);
    int32_t* lab = cv.take<int32_t>(pad);
    int64_t* pivmap = cv.take<int64_t>(ppad);
    uint8_t* pops = cv.take<uint8_t>((size_t)ppad * p.DP * p.eb);
    float* pinit = cv.take<float>(ppad);
    float* pnout = cv.take<float>(ppad);
    int32_t* psexp = cv.take<int32_t>(ppad);
    int32_t* labc = cv.take<int32_t>(p.n_all);
    void* sort_tmp = cv.take<char>(p.scan_bytes);
    uint64_t* state = cv.take<uint64_t>((size_t)pad * p.ksel);
    unsigned int* counter = cv.take<unsigned int>(64);
    int32_t* knn_ws = cv.take<int32_t>((size_t)p.n_all * k);
    int32_t* order = cv.take<int32_t>(p.n_all);
    void* prune_ws = cv.take<char>(p.prune_bytes);
    int32_t* knn = knn_out ? knn_out : knn_ws;
    const bool fp8 = prec == SG_PREC_FP8;
    const bool plain_ip = metric == SG_IP && !norm_corrected_ip(metric, prec);
    const float qmul = plain_ip ? -1.0f : -2.0f;
    const float osc = norm_corrected_ip(metric, prec) ? 0.5f : 1.0f;
    const unsigned eg = (unsigned)std::min<int64_t>(cdiv(std::max(pad, ppad), 256), 8192);

    maps_kernel<<<eg, 256, 0, s>>>(p.sh, idmap, perm, pid, pivmap);
    SG_LAUNCH_CHECK();
    launch_prep(X, dtype, ppad, d, ld, pivmap, p.n_all, ppad, p.DP, prec,
                metric, pops, pinit, pnout, fp8 ? psexp : nullptr, s);
    SG_LAUNCH_CHECK();
    launch_prep(X, dtype, pad, d, ld, idmap, p.n_all, pad, p.DP, prec, metric,
                ops, ninit, nout, fp8 ? sexp : nullptr, s);
    SG_LAUNCH_CHECK();
    p.kern.near<<<(unsigned)(pad / (NEAR_WAVES * 32)), NEAR_WAVES * 64, 0, s>>>(
        p.sh, pops, pinit, fp8 ? psexp : nullptr, ops, fp8 ? sexp : nullptr, qmul, lab);
    SG_LAUNCH_CHECK();
    // the locality order: rows sorted by (global label, row), stable
    compact_labels_kernel<<<eg, 256, 0, s>>>(p.sh, lab, labc);
    SG_LAUNCH_CHECK();
    label_sort(labc, p.n_all, bits_for(std::max<int64_t>(piv, 1)), order, sort_tmp, s);
    place_batched_kernel<<<eg, 256, 0, s>>>(p.sh, order, perm, pid);
    SG_LAUNCH_CHECK();
    launch_prep(X, dtype, pad, d, ld, perm, p.n_all, pad, p.DP, prec, metric,
                ops, ninit, nout, fp8 ? sexp : nullptr, s);
    SG_LAUNCH_CHECK();
    // (the distance kernel writes every list itself: no initialisation)
    fill<unsigned int>(counter, 0u, 1, s);

    TopkArgs A{};
    A.ops = ops;
    A.ninit = ninit;
    A.sexp = fp8 ? sexp : nullptr;
    A.cpid = pid;
    A.qnout = nout;
    A.qout = perm;
    A.qmul = qmul;
    A.osc = osc;
    A.state = state;
    A.nbr = p.rerank > 0 ? nullptr : knn;   // with a re-rank the lists come from the FP32 pass
    A.dist = nullptr;
    A.k_out = k;
    int dev = 0, cus = 0, per_cu = 0;
    SG_HIP(hipGetDevice(&dev));
    SG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    SG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(p.kern.fn),
                                                        p.kern.threads, 0));
    const int grid = std::max(1, std::min(p.nitems, cus * std::max(per_cu, 1)));
    if (eager) profile_record(s, true);
    p.kern.fn<<<grid, p.kern.threads, 0, s>>>(A, p.sh, counter, p.nitems);
    SG_LAUNCH_CHECK();
    if (eager) profile_record(s, false);
    if (p.rerank > 0)   // exact FP32 distances of every row's rerank candidates; padding slots are skipped
        launch_rerank<uint64_t>(X, dtype, pad, d, ld, metric, perm, p.n_all, state, p.ksel, p.rerank, k, knn, nullptr,
                                perm, s);

    const sg_status pr = sg_prune(knn, p.n_all, k, R, order, graphs, prune_ws, p.prune_bytes, s);
    if (pr != SG_OK) throw Fail{pr};
    const unsigned lg = (unsigned)std::min<int64_t>(cdiv(p.n_all * R, 256), 8192);
    localize_kernel<<<lg, 256, 0, s>>>(p.sh, graphs, R);
    SG_LAUNCH_CHECK();
    if (knn_out) {
        localize_kernel<<<(unsigned)std::min<int64_t>(cdiv(p.n_all * k, 256), 8192), 256, 0, s>>>(p.sh, knn_out, k);
        SG_LAUNCH_CHECK();
    }
}

std::vector<uint8_t> signature(const void* X, int dtype, int d, int64_t ld, const int64_t* off, int S, int metric,
                               int k, int R, int prec, const int32_t* graphs, const int32_t* knn, const void* ws,
                               size_t ws_bytes, hipStream_t s, const Plan& p) {
    std::vector<uint8_t> v;
    auto put = [&](const void* a, size_t n) {
        const uint8_t* b = static_cast<const uint8_t*>(a);
        v.insert(v.end(), b, b + n);
    };
    put(&X, sizeof X);
    put(&dtype, sizeof dtype);
    put(&d, sizeof d);
    put(&ld, sizeof ld);
    put(off, sizeof(int64_t) * (S + 1));
    put(&S, sizeof S);
    put(&metric, sizeof metric);
    put(&k, sizeof k);
    put(&R, sizeof R);
    put(&prec, sizeof prec);
    put(&graphs, sizeof graphs);
    put(&knn, sizeof knn);
    put(&ws, sizeof ws);
    put(&ws_bytes, sizeof ws_bytes);
    put(&s, sizeof s);
    put(&p.kern.fn, sizeof p.kern.fn);
    put(&p.rerank, sizeof p.rerank);
    return v;
}

}  // namespace batch
}  // namespace sg

using namespace sg;

extern "C" sg_status sg_knn_graph_batched_workspace_size(const int64_t* offsets_h, int32_t S, int32_t d, int32_t k,
                                                         int32_t R, sg_prec prec, int32_t rerank, size_t* bytes) {
    return guarded([&] {
        SG_REQUIRE(bytes != nullptr, "bytes is NULL");
        *bytes = batch::make_plan(offsets_h, S, d, k, R, prec, rerank).total;
    });
}

extern "C" sg_status sg_knn_graph_batched(const void* X, sg_dtype dtype, int32_t d, int64_t ld,
                                          const int64_t* offsets_h, int32_t S, sg_metric metric, int32_t k,
                                          int32_t R, sg_prec prec, int32_t rerank, int32_t* graphs, int32_t* knn,
                                          void* ws, size_t ws_bytes, void* stream, sg_batch_plan** plan) {
    return guarded([&] {
        const batch::Plan p = batch::make_plan(offsets_h, S, d, k, R, prec, rerank);
        knn::check_args(X, dtype, p.n_all, d, ld, metric, k, prec, p.rerank);
        SG_REQUIRE(graphs != nullptr, "graphs is NULL");
        if (ws == nullptr || ws_bytes < p.total) {
            set_error("sg_knn_graph_batched: workspace too small (need " + std::to_string(p.total) + " bytes)");
            throw Fail{SG_ERR_WORKSPACE};
        }
        if (p.n_all == 0) return;
        hipStream_t s = as_stream(stream);
        if (plan == nullptr) {
            batch::enqueue(p, X, dtype, d, ld, metric, k, R, prec, graphs, knn, ws, s, true);
            return;
        }
        SG_REQUIRE(s != nullptr, "capturing a plan needs a non-default stream");
        const std::vector<uint8_t> sig =
            batch::signature(X, dtype, d, ld, offsets_h, S, metric, k, R, prec, graphs, knn, ws, ws_bytes, s, p);
        int dev = 0;
        SG_HIP(hipGetDevice(&dev));
        if (*plan != nullptr) {
            SG_REQUIRE((*plan)->sig == sig && (*plan)->device == dev,
                       "the plan was captured for other arguments (destroy it and pass a NULL plan)");
            SG_HIP(hipGraphLaunch((*plan)->exec, s));
            return;
        }
        SG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipGraph_t graph = nullptr;
        try {
            batch::enqueue(p, X, dtype, d, ld, metric, k, R, prec, graphs, knn, ws, s, false);
        } catch (...) {
            (void)hipStreamEndCapture(s, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        SG_HIP(hipStreamEndCapture(s, &graph));
        hipGraphExec_t exec = nullptr;
        const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        SG_HIP(e);
        sg_batch_plan* np = new sg_batch_plan;
        np->exec = exec;
        np->sig = sig;
        np->device = dev;
        *plan = np;
        SG_HIP(hipGraphLaunch(exec, s));
    });
}

extern "C" sg_status sg_knn_graph_batched_autotune(const void* X, sg_dtype dtype, int32_t d, int64_t ld,
                                                   const int64_t* offsets_h, int32_t S, sg_metric metric, int32_t k,
                                                   int32_t R, sg_prec prec, int32_t rerank, int32_t* graphs,
                                                   int32_t* knn, void* ws, size_t ws_bytes, void* stream,
                                                   int32_t* chosen, float* times_ms, int32_t max_times) {
    return guarded([&] {
        const batch::Plan p0 = batch::make_plan(offsets_h, S, d, k, R, prec, rerank);
        knn::check_args(X, dtype, p0.n_all, d, ld, metric, k, prec, p0.rerank);
        SG_REQUIRE(graphs != nullptr, "graphs is NULL");
        SG_REQUIRE(p0.n_all > 0, "autotuning needs rows");
        SG_REQUIRE(max_times >= 0 && (max_times == 0 || times_ms != nullptr), "bad times_ms / max_times");
        if (ws == nullptr || ws_bytes < p0.total) {
            set_error("sg_knn_graph_batched_autotune: workspace too small (need " + std::to_string(p0.total) +
                      " bytes)");
            throw Fail{SG_ERR_WORKSPACE};
        }
        std::vector<batch::BKern> kv;
        batch::batched_shapes(prec, d, p0.ksel, kv);
        const int nv = (int)kv.size();
        hipStream_t s = as_stream(stream);
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
        for (int v = 0; v < nv; ++v) {
            knn::g_force_variant = v;
            const batch::Plan pv = batch::make_plan(offsets_h, S, d, k, R, prec, rerank);
            batch::enqueue(pv, X, dtype, d, ld, metric, k, R, prec, graphs, knn, ws, s, false);
            SG_HIP(hipEventRecord(e0, s));
            batch::enqueue(pv, X, dtype, d, ld, metric, k, R, prec, graphs, knn, ws, s, false);
            SG_HIP(hipEventRecord(e1, s));
            SG_HIP(hipEventSynchronize(e1));
            SG_HIP(hipEventElapsedTime(&ms[v], e0, e1));
        }
        int best = 0;
        for (int v = 1; v < nv; ++v)
            if (ms[v] < ms[best]) best = v;
        {
            std::lock_guard<std::mutex> g(knn::g_tune_mu);
            knn::g_tune[knn::batched_tune_key(prec, d, p0.ksel, p0.n_max)] = best;
        }
        if (chosen) *chosen = best;
        for (int v = 0; v < nv && v < max_times; ++v) times_ms[v] = ms[v];
    });
}

extern "C" void sg_batch_plan_destroy(sg_batch_plan* plan) {
    if (!plan) return;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    delete plan;
}

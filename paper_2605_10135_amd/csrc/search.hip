// search.hip -- greedy best-first beam search on the merged graph (the
// DiskANN-style query of the merged index, Sec. VI).
//
// One wave per query.  The beam (capacity L <= 512) lives in LDS as sorted
// (distance, id) keys plus an expanded flag per entry; the visited set is a
// bitmap per query slot in the workspace.  Each round expands the first
// unexpanded entry.  Its neighbours are taken 64 at a time: each lane claims
// one neighbour in the bitmap (atomicOr, so an id is evaluated once per
// query), computes its FP32 distance, keeps it if it beats the current L-th
// entry; the wave sorts the survivors and merges them into the beam by rank.
// Inserting a sorted chunk and keeping the best L yields the same beam as
// inserting the neighbours one at a time in list order, since the admission
// bound only tightens and keys are unique.
//
// The medoid entry (entry < 0) is the row nearest (FP32) to the FP64 mean of
// the rows; the mean is a fixed-order two-level sum, the argmin an atomicMin
// on (distance, id) keys, so it is deterministic.
#include "common.hpp"

namespace sg {
namespace search {

constexpr int WAVES = 4;
constexpr int MAX_L = 512;
constexpr int MAX_DEG = 256;
constexpr int MAX_D = 1024;
constexpr int BATCH = 8192;    // queries per launch (bounds the bitmap workspace)
constexpr int MEAN_ROWS = 4096;

__device__ inline float load_elem(const void* X, int dtype, int64_t idx) {
    switch (dtype) {
        case SG_F32: return static_cast<const float*>(X)[idx];
        case SG_F16: return (float)static_cast<const _Float16*>(X)[idx];
        case SG_BF16: return __builtin_bit_cast(float, (uint32_t) static_cast<const uint16_t*>(X)[idx] << 16);
        default: return (float)static_cast<const uint8_t*>(X)[idx];
    }
}

__device__ inline float delta(const float* q, const void* X, int dtype, int64_t rowbase, int d,
                              int metric) {
    float s = 0.f;
    if (metric == SG_L2) {
        for (int t = 0; t < d; ++t) {
            float u = q[t] - load_elem(X, dtype, rowbase + t);
            s = fmaf(u, u, s);
        }
        return s;
    }
    for (int t = 0; t < d; ++t) s = fmaf(q[t], load_elem(X, dtype, rowbase + t), s);
    return -s;
}

struct WaveSmem {
    uint64_t beam[MAX_L];
    uint64_t tmpk[MAX_L];
    uint64_t nbuf[64];
    uint8_t expd[MAX_L];
    uint8_t tmpf[MAX_L];
    float q[MAX_D];
};

__global__ __launch_bounds__(256) void search_kernel(const void* __restrict__ X, int dtype, int64_t n,
                                                     int d, int64_t ld, int metric,
                                                     const int32_t* __restrict__ graph, int max_degree,
                                                     const void* __restrict__ Q, int64_t q0, int64_t q1,
                                                     int64_t ldq, int topk, int L,
                                                     const int64_t* __restrict__ entry_p,
                                                     uint32_t* __restrict__ bitmap, int64_t words,
                                                     int32_t* __restrict__ out_ids,
                                                     float* __restrict__ out_dist) {
    extern __shared__ __align__(16) char smem[];
    const int l = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    WaveSmem& S = reinterpret_cast<WaveSmem*>(smem)[w];
    const int64_t slot = (int64_t)blockIdx.x * WAVES + w;
    const int64_t qi = q0 + slot;
    if (qi >= q1) return;
    const int64_t entry = *entry_p;
    for (int t = l; t < d; t += 64) S.q[t] = load_elem(Q, dtype, qi * ldq + t);
    uint32_t* vis = bitmap + slot * words;
    for (int64_t t = l; t < words; t += 64) vis[t] = 0u;
    asm volatile("s_waitcnt lgkmcnt(0)\n s_waitcnt vmcnt(0)" ::: "memory");
    if (l == 0) {
        atomicOr(&vis[entry >> 5], 1u << (entry & 31));
        S.beam[0] = make_key(delta(S.q, X, dtype, entry * ld, d, metric), (int32_t)entry);
        S.expd[0] = 0;
    }
    int size = 1;
    asm volatile("s_waitcnt lgkmcnt(0)\n s_waitcnt vmcnt(0)" ::: "memory");
    while (true) {
        int first = MAX_L;
        for (int t = l; t < size; t += 64)
            if (!S.expd[t]) {
                first = t;
                break;
            }
        for (int o = 32; o > 0; o >>= 1) first = min(first, __shfl_xor(first, o, 64));
        if (first >= size) break;
        const int32_t v = key_id(S.beam[first]);
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        if (l == 0) S.expd[first] = 1;
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        for (int c0 = 0; c0 < max_degree; c0 += 64) {
            const uint64_t bound = size == L ? S.beam[L - 1] : EMPTY_KEY;
            uint64_t key = EMPTY_KEY;
            const int e = c0 + l;
            if (e < max_degree) {
                const int32_t u = graph[(int64_t)v * max_degree + e];
                if (u >= 0 && u < n) {
                    const uint32_t bit = 1u << (u & 31);
                    const uint32_t old = atomicOr(&vis[u >> 5], bit);
                    if (!(old & bit)) {
                        const uint64_t k = make_key(delta(S.q, X, dtype, (int64_t)u * ld, d, metric), u);
                        if (k < bound) key = k;
                    }
                }
            }
            const int nnew = __builtin_popcountll(__builtin_amdgcn_ballot_w64(key != EMPTY_KEY));
            if (nnew == 0) continue;
            key = wave_sort_u64(key);
            S.nbuf[l] = key;
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            // merge by rank; positions past L fall off
            for (int t = l; t < size; t += 64) {
                const uint64_t k = S.beam[t];
                const int pos = t + lower_bound_u64(S.nbuf, nnew, k);
                if (pos < L) {
                    S.tmpk[pos] = k;
                    S.tmpf[pos] = S.expd[t];
                }
            }
            if (l < nnew) {
                const int pos = l + lower_bound_u64(S.beam, size, key);
                if (pos < L) {
                    S.tmpk[pos] = key;
                    S.tmpf[pos] = 0;
                }
            }
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            size = min(L, size + nnew);
            for (int t = l; t < size; t += 64) {
                S.beam[t] = S.tmpk[t];
                S.expd[t] = S.tmpf[t];
            }
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        }
    }
    for (int t = l; t < topk; t += 64) {
        const uint64_t k = t < size ? S.beam[t] : EMPTY_KEY;
        out_ids[qi * topk + t] = key_id(k);
        if (out_dist) out_dist[qi * topk + t] = key_dist(k);
    }
}

// ---------------------------------------------------------------------------
// medoid
// ---------------------------------------------------------------------------
__global__ void mean_partial_kernel(const void* __restrict__ X, int dtype, int64_t n, int d, int64_t ld,
                                    double* __restrict__ part) {
    for (int t = threadIdx.x; t < d; t += blockDim.x) {
        const int64_t r0 = (int64_t)blockIdx.x * MEAN_ROWS;
        const int64_t r1 = r0 + MEAN_ROWS < n ? r0 + MEAN_ROWS : n;
        double s = 0.0;
        for (int64_t r = r0; r < r1; ++r) s += (double)load_elem(X, dtype, r * ld + t);
        part[(int64_t)blockIdx.x * d + t] = s;
    }
}

__global__ void mean_final_kernel(const double* __restrict__ part, int nb, int d, int64_t n,
                                  float* __restrict__ meanf, unsigned long long* __restrict__ best) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < d; t += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[(int64_t)b * d + t];
        meanf[t] = (float)(s / (double)n);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *best = ~0ull;
}

__global__ void medoid_kernel(const void* __restrict__ X, int dtype, int64_t n, int d, int64_t ld,
                              const float* __restrict__ meanf, unsigned long long* __restrict__ best) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int t = 0; t < d; ++t) {
            float u = load_elem(X, dtype, i * ld + t) - meanf[t];
            s = fmaf(u, u, s);
        }
        atomicMin(best, (unsigned long long)make_key(s, (int32_t)i));
    }
}

__global__ void entry_from_key(const unsigned long long* __restrict__ best, int64_t* __restrict__ entry) {
    *entry = (int64_t)(uint32_t)(*best);
}

struct Layout {
    int64_t words;
    int nb_mean;
    size_t total;
};

inline Layout layout(int64_t n, int d, int64_t nq) {
    Layout L;
    L.words = (n + 31) / 32;
    L.nb_mean = cdiv(n, MEAN_ROWS);
    int64_t slots = std::min<int64_t>(std::max<int64_t>(nq, 1), BATCH);
    slots = (slots + WAVES - 1) / WAVES * WAVES;
    L.total = align_up((size_t)slots * L.words * 4, 256) + align_up((size_t)L.nb_mean * d * 8, 256) +
              align_up((size_t)d * 4, 256) + 256 + 256 + 1024;
    return L;
}

}  // namespace search
}  // namespace sg

using namespace sg;

extern "C" sg_status sg_search_workspace_size(int64_t n, int32_t d, int64_t nq, size_t* bytes) {
    return guarded([&] {
        SG_REQUIRE(bytes != nullptr, "bytes is NULL");
        SG_REQUIRE(n >= 1 && d >= 1 && nq >= 0, "bad sizes");
        *bytes = search::layout(n, d, nq).total;
    });
}

extern "C" sg_status sg_search(const void* X, sg_dtype dtype, int64_t n, int32_t d, int64_t ld,
                               sg_metric metric, const int32_t* graph, int32_t max_degree, const void* Q,
                               int64_t nq, int64_t ldq, int32_t topk, int32_t L, int64_t entry,
                               int32_t* out_ids, float* out_dist, void* ws, size_t ws_bytes,
                               void* stream) {
    return guarded([&] {
        SG_REQUIRE(n >= 1 && n <= MAX_ROWS, "n out of range (at most 2^26 - 1024 rows)");
        SG_REQUIRE(d >= 1 && d <= search::MAX_D, "d must be in 1..1024");
        SG_REQUIRE(ld >= d && ldq >= d, "ld and ldq must be >= d");
        SG_REQUIRE(metric == SG_L2 || metric == SG_IP, "unknown metric");
        SG_REQUIRE(dtype >= SG_F32 && dtype <= SG_U8, "unknown dtype");
        SG_REQUIRE(max_degree >= 1 && max_degree <= search::MAX_DEG, "max_degree must be in 1..256");
        SG_REQUIRE(topk >= 1 && topk <= L && L <= search::MAX_L, "need 1 <= topk <= L <= 512");
        SG_REQUIRE(entry < n, "entry out of range");
        SG_REQUIRE(nq >= 0 && nq <= MAX_ROWS, "nq out of range (at most 2^26 - 1024 queries)");
        if (nq == 0) return;
        SG_REQUIRE(X && graph && Q && out_ids, "NULL pointer");
        search::Layout Ly = search::layout(n, d, nq);
        if (ws == nullptr || ws_bytes < Ly.total) {
            set_error("sg_search: workspace too small (need " + std::to_string(Ly.total) + " bytes)");
            throw Fail{SG_ERR_WORKSPACE};
        }
        hipStream_t s = as_stream(stream);
        int64_t slots = std::min<int64_t>(nq, search::BATCH);
        slots = (slots + search::WAVES - 1) / search::WAVES * search::WAVES;
        Carver cv(ws);
        uint32_t* bitmap = cv.take<uint32_t>((size_t)slots * Ly.words);
        double* part = cv.take<double>((size_t)Ly.nb_mean * d);
        float* meanf = cv.take<float>(d);
        unsigned long long* best = cv.take<unsigned long long>(1);
        int64_t* entry_d = cv.take<int64_t>(1);
        if (entry < 0) {
            search::mean_partial_kernel<<<(unsigned)Ly.nb_mean, 256, 0, s>>>(X, dtype, n, d, ld, part);
            search::mean_final_kernel<<<cdiv(d, 256), 256, 0, s>>>(part, Ly.nb_mean, d, n, meanf, best);
            search::medoid_kernel<<<(unsigned)std::min<int64_t>(cdiv(n, 256), 8192), 256, 0, s>>>(
                X, dtype, n, d, ld, meanf, best);
            search::entry_from_key<<<1, 1, 0, s>>>(best, entry_d);
        } else {
            fill<int64_t>(entry_d, entry, 1, s);
        }
        SG_LAUNCH_CHECK();
        const size_t shm = sizeof(search::WaveSmem) * search::WAVES;
        SG_HIP(hipFuncSetAttribute((const void*)search::search_kernel,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
        for (int64_t q0 = 0; q0 < nq; q0 += search::BATCH) {
            const int64_t q1 = std::min<int64_t>(nq, q0 + search::BATCH);
            search::search_kernel<<<(unsigned)cdiv(q1 - q0, search::WAVES), 256, shm, s>>>(
                X, dtype, n, d, ld, metric, graph, max_degree, Q, q0, q1, ldq, topk, L, entry_d, bitmap,
                Ly.words, out_ids, out_dist);
            SG_LAUNCH_CHECK();
        }
    });
}

// prune.hip -- rank-based (detour-count) prune and reverse-edge pass.
//
// The graph-optimisation stage of the CAGRA-style shard build (Sec. II-A,
// Sec. IV step 2), as integer passes:
//  * Rows are visited in the caller's order (a permutation of the rows, e.g.
//    the locality order of the kNN build, so that concurrently processed rows
//    share neighbour lists in L2) or in row order; the results do not depend
//    on it.
//  * detour_kernel: one wave per row x.  N(x) goes into a per-wave LDS hash
//    (id -> position); the wave then streams the lists N(y_i) (one coalesced
//    row read per i, lists stay cache resident) and counts, for every
//    position j, the i < j whose list holds y_j before position j.  Positions
//    are ranked by (detour, j) and the first R written: P(x).
//  * count / scatter: in-degree histogram of P, exclusive scan, scatter of the
//    64-bit reverse keys (p << 32 | x) per target (slot order is arbitrary;
//    the next pass sorts, so the output does not depend on it).
//  * combine_kernel: one wave per row y: the R smallest reverse keys (wave
//    bitonic sort, chunked for high in-degree), then the list
//    P(y)[0:h] ++ Rev(y) ++ P(y)[h:R] is deduplicated in order and cut at R.
#include "common.hpp"

namespace sg {
namespace prune {

constexpr int WAVES = 4;

__device__ inline uint32_t hash_id(uint32_t v) { return v * 2654435761u; }

template <int HS>
__device__ inline int hash_find(const int32_t* hid, const int32_t* hpos, int32_t z) {
    uint32_t hsh = hash_id((uint32_t)z) >> (32 - __builtin_ctz(HS));
    while (true) {
        int32_t k = hid[hsh];
        if (k == z) return hpos[hsh];
        if (k == SG_NONE) return -1;
        hsh = (hsh + 1) & (HS - 1);
    }
}

// KP: list entries per lane (ceil(K/64)); HS: hash slots (power of two >= 2K)
template <int KP, int HS>
__global__ __launch_bounds__(256) void detour_kernel(const int32_t* __restrict__ knn, int64_t n,
                                                     int K, int R, const int32_t* __restrict__ order,
                                                     int32_t* __restrict__ P) {
    __shared__ int32_t s_hid[WAVES][HS];
    __shared__ int32_t s_hpos[WAVES][HS];
    __shared__ int32_t s_det[WAVES][64 * KP];
    __shared__ int32_t s_nx[WAVES][64 * KP];
    const int l = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t slot = (int64_t)blockIdx.x * WAVES + w;
    if (slot >= n) return;
    const int64_t x = order ? order[slot] : slot;
    if (x < 0 || x >= n) return;
    int32_t* hid = s_hid[w];
    int32_t* hpos = s_hpos[w];
    int32_t* det = s_det[w];
    int32_t* nx = s_nx[w];
    for (int t = l; t < HS; t += 64) hid[t] = SG_NONE;
    int32_t y[KP];
#pragma unroll
    for (int t = 0; t < KP; ++t) {
        int j = l + 64 * t;
        y[t] = j < K ? knn[x * K + j] : SG_NONE;
        if (y[t] < 0 || y[t] >= n) y[t] = SG_NONE;   // out-of-range ids count as absent
        nx[j] = y[t];
        det[j] = 0;
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    // insert id -> position (ids of a row are distinct)
#pragma unroll
    for (int t = 0; t < KP; ++t) {
        if (y[t] != SG_NONE) {
            uint32_t hsh = hash_id((uint32_t)y[t]) >> (32 - __builtin_ctz(HS));
            while (atomicCAS(&hid[hsh], SG_NONE, y[t]) != SG_NONE) hsh = (hsh + 1) & (HS - 1);
            hpos[hsh] = l + 64 * t;
        }
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    // detour counts: for each i, lane p reads z = N(y_i)[p]; 16 lists are
    // loaded per round so that their memory latencies overlap
    constexpr int UB = 16;
    for (int i0 = 0; i0 < K - 1; i0 += UB) {
        int32_t z[UB][KP];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const int i = i0 + u;
            const int32_t yi = i < K - 1 ? nx[i] : SG_NONE;
#pragma unroll
            for (int t = 0; t < KP; ++t) {
                const int p = l + 64 * t;
                z[u][t] = (yi != SG_NONE && p < K) ? knn[(int64_t)yi * K + p] : SG_NONE;
            }
        }
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const int i = i0 + u;
#pragma unroll
            for (int t = 0; t < KP; ++t) {
                const int p = l + 64 * t;
                if (z[u][t] != SG_NONE) {
                    int j = hash_find<HS>(hid, hpos, z[u][t]);
                    if (j > i && p < j) atomicAdd(&det[j], 1);
                }
            }
        }
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    // rank valid positions by (detour, j); keys are unique
    int nvalid = 0;
#pragma unroll
    for (int t = 0; t < KP; ++t) nvalid += __builtin_popcountll(__builtin_amdgcn_ballot_w64(y[t] != SG_NONE));
#pragma unroll
    for (int t = 0; t < KP; ++t) {
        int j = l + 64 * t;
        if (y[t] == SG_NONE) continue;
        int kj = det[j] * 1024 + j;
        int rank = 0;
        for (int u = 0; u < K; ++u) {
            if (nx[u] != SG_NONE && det[u] * 1024 + u < kj) ++rank;
        }
        if (rank < R) P[x * R + rank] = y[t];
    }
    for (int r = nvalid + l; r < R; r += 64) P[x * R + r] = SG_NONE;
}

__global__ void count_kernel(const int32_t* __restrict__ P, int64_t total, int64_t* __restrict__ cnt) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int32_t y = P[e];
        if (y != SG_NONE) atomicAdd(reinterpret_cast<unsigned long long*>(&cnt[y]), 1ull);   // P is ours: ids in range
    }
}

__global__ void scatter_kernel(const int32_t* __restrict__ P, int64_t total, int R,
                               const int64_t* __restrict__ off, int64_t* __restrict__ fillc,
                               uint64_t* __restrict__ rev) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int32_t y = P[e];
        if (y == SG_NONE) continue;
        int64_t x = e / R;
        int p = (int)(e - x * R);
        unsigned long long slot = atomicAdd(reinterpret_cast<unsigned long long*>(&fillc[y]), 1ull);
        rev[off[y] + (int64_t)slot] = ((uint64_t)p << 32) | (uint32_t)x;
    }
}

// Appends the chunk's values (one per lane, SG_NONE = absent) in lane order to
// the list kl[0..*kc), skipping values already present; stops at cap.
__device__ inline void append_unique(int32_t v, int32_t* kl, int* kc, int cap, int32_t* chunk) {
    const int l = lane_id();
    chunk[l] = v;
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    bool keep = v != SG_NONE;
    const int c0 = *kc;
    for (int t = 0; t < c0 && keep; ++t) keep = kl[t] != v;
    for (int t = 0; t < l && keep; ++t) keep = chunk[t] != v;
    uint64_t m = __builtin_amdgcn_ballot_w64(keep);
    int pos = c0 + __builtin_popcountll(m & ((1ull << l) - 1));
    if (keep && pos < cap) kl[pos] = v;
    int nc = c0 + __builtin_popcountll(m);
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    *kc = nc < cap ? nc : cap;
}

__global__ __launch_bounds__(256) void combine_kernel(const int32_t* __restrict__ P, int64_t n, int R,
                                                      const int64_t* __restrict__ off,
                                                      const uint64_t* __restrict__ rev,
                                                      const int32_t* __restrict__ order,
                                                      int32_t* __restrict__ F) {
    __shared__ int32_t s_kl[WAVES][64];
    __shared__ int32_t s_chunk[WAVES][64];
    const int l = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t slot = (int64_t)blockIdx.x * WAVES + w;
    if (slot >= n) return;
    const int64_t y = order ? order[slot] : slot;
    if (y < 0 || y >= n) return;
    const int h = (R + 1) / 2;
    const int64_t b = off[y], cnt = off[y + 1] - off[y];
    // the R smallest reverse keys, ascending, one per lane
    uint64_t best = l < cnt ? rev[b + l] : EMPTY_KEY;
    best = wave_sort_u64(best);
    for (int64_t c0 = 64; c0 < cnt; c0 += 64) {
        uint64_t v = c0 + l < cnt ? rev[b + c0 + l] : EMPTY_KEY;
        v = wave_sort_u64(v);
        // bitonic merge of two ascending runs: reverse one, take elementwise min, sort
        uint64_t vr = shfl_u64(v, 63 - l);
        best = wave_sort_u64(best < vr ? best : vr);
    }
    int32_t* kl = s_kl[w];
    int32_t* chunk = s_chunk[w];
    int kc = 0;
    // P(y)[0:h]
    append_unique(l < h ? P[y * R + l] : SG_NONE, kl, &kc, R, chunk);
    // reverse entries by (p, x)
    if (kc < R) append_unique(best == EMPTY_KEY ? SG_NONE : (int32_t)(uint32_t)best, kl, &kc, R, chunk);
    // P(y)[h:R]
    if (kc < R) append_unique(l < R - h ? P[y * R + h + l] : SG_NONE, kl, &kc, R, chunk);
    if (l < R) F[y * R + l] = l < kc ? kl[l] : SG_NONE;
}

struct Layout {
    size_t P, cnt, off, fillc, rev, scan, total;
};

inline Layout layout(int64_t n, int R) {
    Layout L;
    L.P = align_up((size_t)n * R * 4, 256);
    L.cnt = align_up((size_t)(n + 1) * 8, 256);
    L.off = align_up((size_t)(n + 1) * 8, 256);
    L.fillc = align_up((size_t)(n + 1) * 8, 256);
    L.rev = align_up((size_t)n * R * 8, 256);
    L.scan = align_up(exclusive_scan_tmp_bytes(n), 256);
    L.total = L.P + L.cnt + L.off + L.fillc + L.rev + L.scan + 1024;
    return L;
}

}  // namespace prune
}  // namespace sg

using namespace sg;

extern "C" sg_status sg_prune_workspace_size(int64_t n, int32_t K, int32_t R, size_t* bytes) {
    return guarded([&] {
        SG_REQUIRE(bytes != nullptr, "bytes is NULL");
        SG_REQUIRE(n >= 0 && K >= 1 && R >= 1, "bad sizes");
        *bytes = n == 0 ? 0 : prune::layout(n, R).total;
    });
}

extern "C" sg_status sg_prune(const int32_t* knn, int64_t n, int32_t K, int32_t R, const int32_t* order,
                              int32_t* out, void* ws, size_t ws_bytes, void* stream) {
    return guarded([&] {
        SG_REQUIRE(n >= 0 && n < (1ll << 31), "n out of range");
        SG_REQUIRE(K >= 1 && K <= 256, "K must be in 1..256");
        SG_REQUIRE(R >= 1 && R <= K && R <= 64, "R must be in 1..min(K, 64)");
        if (n == 0) return;
        SG_REQUIRE(knn != nullptr && out != nullptr, "NULL pointer");
        prune::Layout L = prune::layout(n, R);
        if (ws == nullptr || ws_bytes < L.total) {
            set_error("sg_prune: workspace too small (need " + std::to_string(L.total) + " bytes)");
            throw Fail{SG_ERR_WORKSPACE};
        }
        hipStream_t s = as_stream(stream);
        Carver cv(ws);
        int32_t* P = cv.take<int32_t>((size_t)n * R);
        int64_t* cnt = cv.take<int64_t>(n + 1);
        int64_t* off = cv.take<int64_t>(n + 1);
        int64_t* fillc = cv.take<int64_t>(n + 1);
        uint64_t* rev = cv.take<uint64_t>((size_t)n * R);
        void* scan_tmp = cv.take<char>(exclusive_scan_tmp_bytes(n));

        unsigned grid = (unsigned)cdiv(n, prune::WAVES);
        if (K <= 64)
            prune::detour_kernel<1, 256><<<grid, 256, 0, s>>>(knn, n, K, R, order, P);
        else if (K <= 128)
            prune::detour_kernel<2, 512><<<grid, 256, 0, s>>>(knn, n, K, R, order, P);
        else
            prune::detour_kernel<4, 1024><<<grid, 256, 0, s>>>(knn, n, K, R, order, P);
        SG_LAUNCH_CHECK();
        fill<int64_t>(cnt, 0, n + 1, s);
        fill<int64_t>(fillc, 0, n + 1, s);
        int64_t total = n * (int64_t)R;
        unsigned eg = (unsigned)std::min<int64_t>(cdiv(total, 256), 8192);
        prune::count_kernel<<<eg, 256, 0, s>>>(P, total, cnt);
        SG_LAUNCH_CHECK();
        exclusive_scan_i64(cnt, off, n, scan_tmp, s);
        prune::scatter_kernel<<<eg, 256, 0, s>>>(P, total, R, off, fillc, rev);
        SG_LAUNCH_CHECK();
        prune::combine_kernel<<<grid, 256, 0, s>>>(P, n, R, off, rev, order, out);
        SG_LAUNCH_CHECK();
    });
}

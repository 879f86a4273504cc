// prune.hip -- rank-based (detour-count) prune and reverse-edge pass.
//
// The graph-optimisation stage of the CAGRA-style shard build (Sec. II-A,
// Sec. IV step 2), as integer passes:
//  * Rows are visited in the caller's order (a permutation of the rows, e.g.
//    the locality order of the kNN build) or in row order, and each XCD takes
//    one contiguous range of that order, so that the rows one L2 serves at a
//    time are neighbours and share neighbour lists; the results do not depend
//    on the order.
//  * detour_kernel: one wave per row x.  N(x) goes into a per-wave LDS hash
//    (id -> position, one 64-bit slot per entry, at most 1/8 full for
//    K <= 64); the wave then streams the lists N(y_i) (one coalesced row read
//    per i, the next 16/KP lists in flight while the current ones are probed)
//    and counts, for every position j, the i < j whose list holds y_j before
//    position j.  Positions are ranked by (detour, j) (a wave sort of the
//    keys) and the first R written: P(x); the in-degree histogram of P is
//    counted as they are written.
//  * exclusive scan of the in-degrees, scatter of the 64-bit reverse keys
//    (p << 32 | x) per target (slot order is arbitrary; the next pass sorts,
//    so the output does not depend on it).
//  * combine_kernel: one wave per row y: the R smallest reverse keys (wave
//    bitonic sort, chunked for high in-degree), then the list
//    P(y)[0:h] ++ Rev(y) ++ P(y)[h:R] is deduplicated in order (values
//    compared by lane broadcasts) and cut at R.
#include "common.hpp"

namespace sg {
namespace prune {

constexpr int WAVES = 4;

__device__ inline uint32_t hash_id(uint32_t v) { return v * 2654435761u; }

// A row's hash table (open addressing, linear probing) maps a neighbour id to
// its list position; each slot holds (position << 32) | id, so one 64-bit LDS
// read answers a probe.  All ones marks an empty slot.
constexpr uint64_t EMPTY_SLOT = ~0ull;

template <int HS>
__device__ inline uint32_t slot_of(int32_t z) {
    return hash_id((uint32_t)z) >> (32 - __builtin_ctz(HS));
}

// Position of id z (not SG_NONE) in the row's list, -1 if absent; v is the
// value already read from z's first slot.
template <int HS>
__device__ inline int resolve(const uint64_t* h, int32_t z, uint64_t v) {
    uint32_t s = slot_of<HS>(z);
    while ((int32_t)(uint32_t)v != z) {
        if (v == EMPTY_SLOT) return -1;
        s = (s + 1) & (HS - 1);
        v = h[s];
    }
    return (int)(v >> 32);
}

// KP: list entries per lane (ceil(K/64)); HS: hash slots (power of two, at
// least 4K so that most probes end at the first slot)
// Also counts the in-degree of every row in P (cnt, zeroed by the caller).
template <int KP, int HS>
__global__ __launch_bounds__(256) void detour_kernel(const int32_t* __restrict__ knn, int64_t n,
                                                     int K, int R, const int32_t* __restrict__ order,
                                                     int32_t* __restrict__ P, int64_t* __restrict__ cnt) {
    __shared__ uint64_t s_h[WAVES][HS];
    __shared__ int32_t s_det[WAVES][64 * KP];
    __shared__ int32_t s_nx[WAVES][64 * KP];
    const int l = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t slot = xcd_contiguous(blockIdx.x, gridDim.x) * WAVES + w;
    if (slot >= n) return;
    const int64_t x = order ? order[slot] : slot;
    if (x < 0 || x >= n) return;
    uint64_t* h = s_h[w];
    int32_t* det = s_det[w];
    int32_t* nx = s_nx[w];
    for (int t = l; t < HS; t += 64) h[t] = EMPTY_SLOT;
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
            const uint64_t e = ((uint64_t)(uint32_t)(l + 64 * t) << 32) | (uint32_t)y[t];
            uint32_t s2 = slot_of<HS>(y[t]);
            while (atomicCAS(reinterpret_cast<unsigned long long*>(&h[s2]), (unsigned long long)EMPTY_SLOT,
                             (unsigned long long)e) != EMPTY_SLOT)
                s2 = (s2 + 1) & (HS - 1);
        }
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    // detour counts: for each i, lane p reads z = N(y_i)[p] and looks it up;
    // UB lists per round, the next round's lists loading while this round's
    // first probes (all issued together) are resolved
    constexpr int UB = 16 / KP;
    int32_t z[UB][KP], zn[UB][KP];
    auto load = [&](int32_t (&dst)[UB][KP], int i0) {
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const int i = i0 + u;
            const int32_t yi = i < K - 1 ? nx[i] : SG_NONE;
#pragma unroll
            for (int t = 0; t < KP; ++t) {
                const int p = l + 64 * t;
                dst[u][t] = (yi != SG_NONE && p < K) ? knn[(int64_t)yi * K + p] : SG_NONE;
            }
        }
    };
    load(z, 0);
    for (int i0 = 0; i0 < K - 1; i0 += UB) {
        if (i0 + UB < K - 1) load(zn, i0 + UB);
        uint64_t hv[UB][KP];
#pragma unroll
        for (int u = 0; u < UB; ++u)
#pragma unroll
            for (int t = 0; t < KP; ++t) hv[u][t] = z[u][t] != SG_NONE ? h[slot_of<HS>(z[u][t])] : EMPTY_SLOT;
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const int i = i0 + u;
#pragma unroll
            for (int t = 0; t < KP; ++t) {
                const int p = l + 64 * t;
                if (z[u][t] != SG_NONE) {
                    const int j = resolve<HS>(h, z[u][t], hv[u][t]);
                    if (j > i && p < j) atomicAdd(&det[j], 1);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < UB; ++u)
#pragma unroll
            for (int t = 0; t < KP; ++t) z[u][t] = zn[u][t];
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    // rank valid positions by (detour, j); keys are unique
    if constexpr (KP == 1) {
        uint64_t key = y[0] != SG_NONE ? ((uint64_t)(uint32_t)det[l] << 10) | (uint32_t)l : EMPTY_KEY;
        key = wave_sort_u64(key);
        if (l < R) {
            const int32_t v = key == EMPTY_KEY ? SG_NONE : nx[key & 1023];
            P[x * R + l] = v;
            if (v != SG_NONE) atomicAdd(reinterpret_cast<unsigned long long*>(&cnt[v]), 1ull);
        }
    } else {
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
            if (rank < R) {
                P[x * R + rank] = y[t];
                atomicAdd(reinterpret_cast<unsigned long long*>(&cnt[y[t]]), 1ull);
            }
        }
        for (int r = nvalid + l; r < R; r += 64) P[x * R + r] = SG_NONE;
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

// Keeps, of one value per lane (SG_NONE = absent), those that neither an
// earlier lane of the same segment nor any lane of the earlier segments
// e0[0..n0) / e1[0..n1) holds: the in-order deduplication of a segment, by
// broadcasting each compared value from its lane (no LDS round trips).
__device__ inline bool first_occurrence(int32_t v, int nv, int32_t e0, int n0, int32_t e1, int n1) {
    const int l = lane_id();
    bool keep = v != SG_NONE;
    for (int t = 0; t < n0; ++t) keep &= v != __builtin_amdgcn_readlane(e0, t);
    for (int t = 0; t < n1; ++t) keep &= v != __builtin_amdgcn_readlane(e1, t);
    for (int t = 0; t < nv; ++t) keep &= !(t < l && v == __builtin_amdgcn_readlane(v, t));
    return keep;
}

// Lanes below the highest lane holding a value (0 when none).
__device__ inline int span_of(int32_t v) {
    const uint64_t m = __builtin_amdgcn_ballot_w64(v != SG_NONE);
    return m ? 64 - __builtin_clzll(m) : 0;
}

__global__ __launch_bounds__(256) void combine_kernel(const int32_t* __restrict__ P, int64_t n, int R,
                                                      const int64_t* __restrict__ off,
                                                      const uint64_t* __restrict__ rev,
                                                      const int32_t* __restrict__ order,
                                                      int32_t* __restrict__ F) {
    const int l = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t slot = xcd_contiguous(blockIdx.x, gridDim.x) * WAVES + w;
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
    // the sequence P(y)[0:h] ++ Rev(y) ++ P(y)[h:R], deduplicated in order
    // and cut at R: segment A in lanes 0..h-1, B (the 64 smallest reverse
    // keys' sources, by (p, x)) in lanes 0..63, C in lanes 0..R-h-1
    const int32_t va = l < h ? P[y * R + l] : SG_NONE;
    const int32_t vb = best != EMPTY_KEY ? (int32_t)(uint32_t)best : SG_NONE;
    const int32_t vc = l < R - h ? P[y * R + h + l] : SG_NONE;
    const int na = span_of(va), nb = span_of(vb), nc = span_of(vc);
    const bool ka = first_occurrence(va, na, SG_NONE, 0, SG_NONE, 0);
    const bool kb = first_occurrence(vb, nb, va, na, SG_NONE, 0);
    const bool kc = first_occurrence(vc, nc, va, na, vb, nb);
    const uint64_t below = (1ull << l) - 1;
    const uint64_t ma = __builtin_amdgcn_ballot_w64(ka), mb = __builtin_amdgcn_ballot_w64(kb),
                   mc = __builtin_amdgcn_ballot_w64(kc);
    const int ca = __builtin_popcountll(ma), cb = __builtin_popcountll(mb), cc = __builtin_popcountll(mc);
    int32_t* row = F + y * R;
    if (ka) row[__builtin_popcountll(ma & below)] = va;              // ca <= h <= R
    if (kb) {
        const int pos = ca + __builtin_popcountll(mb & below);
        if (pos < R) row[pos] = vb;
    }
    if (kc) {
        const int pos = ca + cb + __builtin_popcountll(mc & below);
        if (pos < R) row[pos] = vc;
    }
    const int total = ca + cb + cc;
    if (l >= total && l < R) row[l] = SG_NONE;
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
        fill<int64_t>(cnt, 0, n + 1, s);
        fill<int64_t>(fillc, 0, n + 1, s);
        if (K <= 64)
            prune::detour_kernel<1, 512><<<grid, 256, 0, s>>>(knn, n, K, R, order, P, cnt);
        else if (K <= 128)
            prune::detour_kernel<2, 1024><<<grid, 256, 0, s>>>(knn, n, K, R, order, P, cnt);
        else
            prune::detour_kernel<4, 1024><<<grid, 256, 0, s>>>(knn, n, K, R, order, P, cnt);
        SG_LAUNCH_CHECK();
        int64_t total = n * (int64_t)R;
        unsigned eg = (unsigned)std::min<int64_t>(cdiv(total, 256), 8192);
        exclusive_scan_i64(cnt, off, n, scan_tmp, s);
        prune::scatter_kernel<<<eg, 256, 0, s>>>(P, total, R, off, fillc, rev);
        SG_LAUNCH_CHECK();
        prune::combine_kernel<<<grid, 256, 0, s>>>(P, n, R, off, rev, order, out);
        SG_LAUNCH_CHECK();
    });
}

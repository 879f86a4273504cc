// prune.hip -- rank-based (detour-count) prune and reverse-edge pass.
//
// The graph-optimisation stage of the CAGRA-style shard build (Sec. II-A,
// Sec. IV step 2), as integer passes:
//  * Rows are visited in the caller's order (a permutation of the rows, e.g.
//    the locality order of the kNN build; anything else is detected on the
//    device and replaced by row order) or in row order, and each XCD takes
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
//    counted as they are written, and the count an edge x -> y reads is its
//    slot in y's reverse list: the edge's reverse key (p << 26 | x, 32 bits)
//    goes straight to y's fixed bucket of 2R slots when the slot is below 2R
//    (the slot order depends on timing, but the combine sorts, so the output
//    does not).
//  * exclusive scan of the in-degrees' excess over the bucket, and placement
//    of the few overflowing keys (rows of in-degree above 2R) by their slots
//    (no atomics).
//  * combine_kernel: one wave per row y: the R smallest reverse keys (wave
//    bitonic sort, chunked for high in-degree), then the list
//    P(y)[0:h] ++ Rev(y) ++ P(y)[h:R] is deduplicated in order (values
//    compared by lane broadcasts) and cut at R.
#include <mutex>

#include "common.hpp"

namespace sg {
namespace prune {

constexpr int WAVES = 4;

// A row's neighbour table, id -> list position, by cuckoo hashing over two
// tables of CT slots (together at most a quarter full): every id sits in T0[h0(id)]
// or in T1[h1(id)], so a lookup is two independent 64-bit LDS reads with no
// probe loop.  A slot holds (position << 32) | id; all ones marks an empty
// slot (its id field is SG_NONE, whose position field, -1, never counts).
constexpr uint64_t EMPTY_SLOT = ~0ull;

// Both slots come from one 24-bit product of the id (v_mul_u32_u24, full
// rate; it reads the low 24 bits of the id, so ids that differ only above bit
// 23 share both slots, which only rows of shards over 2^24 rows can meet and
// which the compare-with-every-entry path then handles): T0 takes bits 8.. of
// the product, T1 bits 20.. (bits 8-15 depend on the low 16 bits of the id
// only, bits 20-29 on all 24).
__device__ inline uint32_t mul_u24(uint32_t c, uint32_t m) {
    uint32_t r;
    asm("v_mul_u32_u24 %0, %1, %2" : "=v"(r) : "s"(c), "v"(m));
    return r;
}
// The hash constants: K <= 128 uses the first; rows of K > 128 whose insertion
// does not settle insert again with the next one before falling back.
constexpr uint32_t CUCKOO_C0 = 0x9E3779u, CUCKOO_C1 = 0x85EBCBu, CUCKOO_C2 = 0xC2B2AFu;
__device__ inline uint32_t cuckoo_product(uint32_t c, int32_t z) { return mul_u24(c, (uint32_t)z); }
template <int CT>
__device__ inline uint32_t cuckoo_h0(uint32_t p) { return (p >> 8) & (CT - 1); }
template <int CT>
__device__ inline uint32_t cuckoo_h1(uint32_t p) { return (p >> 20) & (CT - 1); }

// Flags *bad unless order[0..n) is a permutation of 0..n-1: every entry in
// range and no row seen twice (n entries, so none is then missing).  seen
// (n counters) and *bad start at zero.
__global__ void order_check_kernel(const int32_t* __restrict__ order, int64_t n, int32_t* __restrict__ seen,
                                   int32_t* __restrict__ bad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = order[i];
        if (x < 0 || x >= n || atomicAdd(&seen[x], 1) != 0) *bad = 1;
    }
}

// The row a wave at position `slot` of the visiting order handles: order[slot]
// when the caller's order passed the check, else the row at that position.
__device__ inline int64_t visit_row(const int32_t* order, const int32_t* order_bad, int64_t slot) {
    return (order && *order_bad == 0) ? (int64_t)order[slot] : slot;
}

// Ascending bitonic sort of 64 KP 32-bit keys, element p * 64 + l in v[p]:
// exchanges at distances of 64 and more compare registers of one lane, shorter
// ones compare lanes (lane_xor).
template <int KP>
__device__ inline void sort_multi_u32(uint32_t (&v)[KP]) {
    const int l = lane_id();
#pragma unroll
    for (int k = 2; k <= 64 * KP; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 64) {
                const int jp = j >> 6;
#pragma unroll
                for (int p = 0; p < KP; ++p) {
                    const int q = p ^ jp;
                    if (q > p) {
                        const bool up = ((p * 64) & k) == 0;   // element p*64+l; bit k of it
                        const uint32_t a = v[p], b = v[q];
                        const bool sw = up ? a > b : a < b;
                        v[p] = sw ? b : a;
                        v[q] = sw ? a : b;
                    }
                }
            } else {
#pragma unroll
                for (int p = 0; p < KP; ++p) {
                    const int e = p * 64 + l;
                    const uint32_t o = lane_xor(v[p], j);
                    const bool low = (e & j) == 0, up = (e & k) == 0;
                    // the lower element of a pair keeps the smaller key in an ascending block
                    v[p] = (o < v[p]) == (low == up) ? o : v[p];
                }
            }
        }
    }
}

// Reverse-edge keys (p, x) ordered by p, then x.  For R <= 64 they are
// 32-bit (p << 26 | x): p < 64 and x < MAX_ROWS < 2^26 - 1, so no key equals
// the all-ones empty marker, and the reverse lists hold and the combine sorts
// half the bytes of a 64-bit key.  Wider rows (R <= 128) use (p << 32 | x).
constexpr int REV_XBITS = 26;
static_assert(MAX_ROWS < (int64_t(1) << REV_XBITS) - 1, "row ids must fit the reverse key");
template <typename KT>
struct RevKey;
template <>
struct RevKey<uint32_t> {
    static constexpr uint32_t EMPTY = ~0u;
    __device__ static uint32_t make(int p, int64_t x) { return ((uint32_t)p << REV_XBITS) | (uint32_t)x; }
    __device__ static int32_t source(uint32_t k) { return (int32_t)(k & ((1u << REV_XBITS) - 1)); }
    __device__ static uint32_t sort(uint32_t k) { return wave_sort_u32(k); }
    __device__ static uint32_t xor_lane(uint32_t k, int j) { return lane_xor(k, j); }
    __device__ static uint32_t from_lane(uint32_t k, int src) { return (uint32_t)__shfl((int)k, src, 64); }
};
template <>
struct RevKey<uint64_t> {
    static constexpr uint64_t EMPTY = ~0ull;
    __device__ static uint64_t make(int p, int64_t x) { return ((uint64_t)(uint32_t)p << 32) | (uint64_t)x; }
    __device__ static int32_t source(uint64_t k) { return (int32_t)(uint32_t)k; }
    __device__ static uint64_t sort(uint64_t k) { return wave_sort_u64(k); }
    __device__ static uint64_t xor_lane(uint64_t k, int j) { return lane_xor_u64(k, j); }
    __device__ static uint64_t from_lane(uint64_t k, int src) { return shfl_u64(k, src); }
};

// Row y's reverse keys: the first CAP (in the order the detour pass counts
// them) in y's bucket rev[y * CAP ..], written by the detour pass as it
// counts the edge, the rest (rows of in-degree above CAP) in the overflow
// area at oof[y] .. (exclusive scan of the excess), placed by overflow_kernel.
// CAP = 2R rounded up to 16 entries: the mean in-degree is at most R, so few
// edges overflow.
inline int bucket_cap(int R) { return (2 * R + 15) / 16 * 16; }

// KP: list entries per lane (ceil(K/64)); CT: slots per cuckoo table (power of
// two: 256 for K <= 64 (one eighth full), 256 and 512 for K = 128 and 256 (a
// quarter full, so that six and three waves per SIMD fit; rows of K = 256 that
// do not settle rehash before comparing every entry)).  Also counts the
// in-degree of every row in P (cnt, zeroed by the caller): the count edge
// x -> y reads is its slot in y's reverse list, kept in rslot (-1 for absent
// positions), and the edge's key goes to y's bucket when the slot is below
// cap (rev: 32-bit keys for R <= 64, else 64-bit).
template <int KP, int CT>
__global__ __launch_bounds__(256) void detour_kernel(const int32_t* __restrict__ knn, int64_t n,
                                                     int K, int R, const int32_t* __restrict__ order,
                                                     const int32_t* __restrict__ order_bad,
                                                     int32_t* __restrict__ P, int32_t* __restrict__ rslot,
                                                     int64_t* __restrict__ cnt, int cap, void* __restrict__ rev) {
    __shared__ uint64_t s_t[WAVES][2 * CT];
    __shared__ int32_t s_det[WAVES][64 * KP + 64];   // + one discard slot per lane
    __shared__ int32_t s_nx[WAVES][64 * KP];
    const int l = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t slot = xcd_contiguous(blockIdx.x, gridDim.x) * WAVES + w;
    if (slot >= n) return;
    const int64_t x = visit_row(order, order_bad, slot);
    uint64_t* T0 = s_t[w];
    uint64_t* T1 = s_t[w] + CT;
    int32_t* det = s_det[w];
    int32_t* nx = s_nx[w];
    for (int t = l; t < 2 * CT; t += 64) T0[t] = EMPTY_SLOT;
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
    // insert (ids of a row are distinct): every lane carries an entry until it
    // lands in an empty slot, evicting the occupant to its other table; for
    // K > 128 a row that does not settle starts again with the next constant
    constexpr int ATTEMPTS = KP >= 4 ? 3 : 1;   // (more attempts cost K = 128 registers)
    uint32_t hc = CUCKOO_C0;
    bool failed = true;
    for (int attempt = 0; attempt < ATTEMPTS && failed; ++attempt) {
        if (attempt > 0) {
            hc = attempt == 1 ? CUCKOO_C1 : CUCKOO_C2;
            for (int t = l; t < 2 * CT; t += 64) T0[t] = EMPTY_SLOT;
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        }
        failed = false;
#pragma unroll
        for (int t = 0; t < KP; ++t) {
            bool active = y[t] != SG_NONE;
            uint64_t e = ((uint64_t)(uint32_t)(l + 64 * t) << 32) | (uint32_t)y[t];
            int tb = 0;
            for (int it = 0; it < 128 && __builtin_amdgcn_ballot_w64(active); ++it) {
                if (active) {
                    const uint32_t m = cuckoo_product(hc, (int32_t)(uint32_t)e);
                    unsigned long long* a = reinterpret_cast<unsigned long long*>(
                        tb ? &T1[cuckoo_h1<CT>(m)] : &T0[cuckoo_h0<CT>(m)]);
                    const uint64_t old = atomicExch(a, (unsigned long long)e);
                    if (old == EMPTY_SLOT) {
                        active = false;
                    } else {
                        e = old;        // the evicted entry moves to its slot in the other table
                        tb ^= 1;
                    }
                }
            }
            failed |= __builtin_amdgcn_ballot_w64(active) != 0;
        }
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    }
    // detour counts: for each i, lane p reads z = N(y_i)[p] and looks it up;
    // UB lists per round, the next round's lists loading while this round's
    // are probed
    constexpr int UB = 16 / KP;
    int32_t zA[UB][KP], zB[UB][KP];
    // Raw list entries: every lane loads an index inside a valid row (no
    // branch, so the loads of a round stay in flight together); the returned
    // bit u says whether list u exists (y_i != SG_NONE), and the probes mask
    // lanes past K and absent lists when they consume the values.
    auto load = [&](int32_t (&dst)[UB][KP], int i0) -> uint32_t {
        uint32_t okm = 0;
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const int i = i0 + u;
            // y_i = N(x)[i], wave-uniform: read from the lane holding it (K <= 64)
            // or from LDS
            int32_t yi;
            if constexpr (KP == 1)
                yi = i < K - 1 ? __builtin_amdgcn_readlane(y[0], i) : SG_NONE;
            else
                yi = __builtin_amdgcn_readfirstlane(i < K - 1 ? nx[i] : SG_NONE);
            const bool ok = yi != SG_NONE;
            okm |= ok ? 1u << u : 0u;
            const int32_t* row = knn + (int64_t)(ok ? yi : 0) * K;
#pragma unroll
            for (int t = 0; t < KP; ++t) {
                const int p = l + 64 * t;
                dst[u][t] = row[p < K ? p : 0];
            }
        }
        return okm;
    };
    // count the detour of position j via i: i < j and y_j before position j
    // in N(y_i) (other lanes add to their discard slot)
    auto count = [&](int j, int i, int p) { atomicAdd(&det[(j > i && p < j) ? j : 64 * KP + l], 1); };
    auto entry = [&](const int32_t (&z)[UB][KP], uint32_t okm, int u, int t) -> int32_t {
        return ((okm >> u) & 1u) && l + 64 * t < K ? z[u][t] : SG_NONE;
    };
    auto probe = [&](const int32_t (&z)[UB][KP], uint32_t okm, int i0) {
        uint64_t v0[UB][KP], v1[UB][KP];
#pragma unroll
        for (int u = 0; u < UB; ++u)
#pragma unroll
            for (int t = 0; t < KP; ++t) {
                const uint32_t m = cuckoo_product(hc, entry(z, okm, u, t));
                v0[u][t] = T0[cuckoo_h0<CT>(m)];
                v1[u][t] = T1[cuckoo_h1<CT>(m)];
            }
#pragma unroll
        for (int u = 0; u < UB; ++u)
#pragma unroll
            for (int t = 0; t < KP; ++t) {
                const int32_t zz = entry(z, okm, u, t);
                const uint64_t a = v0[u][t], b = v1[u][t];
                const int j = (int32_t)(uint32_t)a == zz ? (int)(a >> 32) : (int32_t)(uint32_t)b == zz ? (int)(b >> 32) : -1;
                count(j, i0 + u, l + 64 * t);
            }
    };
    // a row whose insertion did not settle (never for distinct ids in
    // practice) finds positions by comparing with every entry
    auto probe_scan = [&](const int32_t (&z)[UB][KP], uint32_t okm, int i0) {
        for (int u = 0; u < UB; ++u)
#pragma unroll
            for (int t = 0; t < KP; ++t) {
                const int32_t zz = entry(z, okm, u, t);
                int j = -1;
                for (int v = K - 1; v >= 0; --v)
                    if (zz != SG_NONE && nx[v] == zz) j = v;
                count(j, i0 + u, l + 64 * t);
            }
    };
    uint32_t okA = load(zA, 0), okB = 0;
    for (int i0 = 0; i0 < K - 1; i0 += 2 * UB) {
        if (i0 + UB < K - 1) okB = load(zB, i0 + UB);
        if (!failed) probe(zA, okA, i0); else probe_scan(zA, okA, i0);
        if (i0 + UB >= K - 1) break;
        if (i0 + 2 * UB < K - 1) okA = load(zA, i0 + 2 * UB);
        if (!failed) probe(zB, okB, i0 + UB); else probe_scan(zB, okB, i0 + UB);
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    // rank valid positions by (detour, j); keys are unique
    {
        // 32-bit keys (detour << 10 | j): detour <= K - 1 < 2^10 and j < 2^10;
        // absent positions all ones, after every valid key.  A bitonic sort of
        // the 64 KP keys (element p * 64 + l in key[p]) puts the rank-r key
        // in element r.
        uint32_t key[KP];
#pragma unroll
        for (int t = 0; t < KP; ++t) {
            const int j = l + 64 * t;
            key[t] = y[t] != SG_NONE ? ((uint32_t)det[j] << 10) | (uint32_t)j : ~0u;
        }
        sort_multi_u32<KP>(key);
#pragma unroll
        for (int p = 0; p < KP; ++p) {
            const int r = p * 64 + l;
            if (r < R) {
                const int32_t v = key[p] == ~0u ? SG_NONE : nx[key[p] & 1023u];
                // (streaming stores: this pass never reads these lines back)
                __builtin_nontemporal_store(v, &P[x * R + r]);
                int32_t sl = -1;
                if (v != SG_NONE) {
                    sl = (int32_t)atomicAdd(reinterpret_cast<unsigned long long*>(&cnt[v]), 1ull);
                    if (sl < cap) {
                        const int64_t at = (int64_t)v * cap + sl;
                        if (R <= 64)
                            __builtin_nontemporal_store(RevKey<uint32_t>::make(r, x), &static_cast<uint32_t*>(rev)[at]);
                        else
                            __builtin_nontemporal_store(RevKey<uint64_t>::make(r, x), &static_cast<uint64_t*>(rev)[at]);
                    }
                }
                __builtin_nontemporal_store(sl, &rslot[x * R + r]);
            }
        }
    }
}

// Ascending order of a bitonic sequence of one key per lane (the merge
// stages of a bitonic sort).
template <typename KT>
__device__ inline KT bitonic_finish(KT x) {
    const int l = lane_id();
#pragma unroll
    for (int j = 32; j > 0; j >>= 1) {
        const KT o = RevKey<KT>::xor_lane(x, j);
        x = (o < x) == ((l & j) == 0) ? o : x;
    }
    return x;
}

// The excess of each row's in-degree over the bucket: ovn[y] = max(cnt[y] - cap, 0).
__global__ void excess_kernel(const int64_t* __restrict__ cnt, int64_t n, int cap, int64_t* __restrict__ ovn) {
    for (int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; y < n; y += (int64_t)gridDim.x * blockDim.x)
        ovn[y] = cnt[y] > cap ? cnt[y] - cap : 0;
}

// Edge e = x * R + p whose slot rslot[e] (its in-degree count of y = P[e]) is
// cap or more goes to over[oof[y] + rslot[e] - cap]: the slots of y's
// overflowing edges are cap .. in-degree(y) - 1, each taken once.  Only those
// edges read P and oof; the rest of the pass is one read of rslot, four slots
// per 16-byte load when rslot is 16-byte aligned.
template <typename KT>
__global__ void overflow_kernel(const int32_t* __restrict__ P, const int32_t* __restrict__ rslot,
                                int64_t total, int R, int cap, const int64_t* __restrict__ oof,
                                KT* __restrict__ over) {
    auto place = [&](int64_t e, int32_t sl) {
        if (sl < cap) return;   // in the bucket, or no edge (-1)
        const int32_t y = P[e];
        const int64_t x = e / R;
        const int p = (int)(e - x * R);
        over[oof[y] + (sl - cap)] = RevKey<KT>::make(p, x);
    };
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t e0 = 0;
    if ((reinterpret_cast<uintptr_t>(rslot) & 15) == 0) {
        const int64_t quads = total / 4;
        const int4* r4 = reinterpret_cast<const int4*>(rslot);
        for (int64_t q = t0; q < quads; q += stride) {
            const int4 v = r4[q];
            place(4 * q, v.x);
            place(4 * q + 1, v.y);
            place(4 * q + 2, v.z);
            place(4 * q + 3, v.w);
        }
        e0 = quads * 4;
    }
    for (int64_t e = e0 + t0; e < total; e += stride) place(e, rslot[e]);
}

// Keeps, of one value per lane (SG_NONE = absent), those that no lane of the
// earlier segment e[0..ne) holds, by broadcasting each compared value from its
// lane (no LDS round trips).  This is all the in-order deduplication needs:
// P(y) lists distinct ids (its kNN row does), so its head and tail share no
// id and neither repeats one, and each row x adds y to its own list at most
// once, so Rev(y) repeats no source either.
__device__ inline bool first_occurrence(int32_t v, int32_t e, int ne) {
    bool keep = v != SG_NONE;
    for (int t = 0; t < ne; ++t) keep &= v != __builtin_amdgcn_readlane(e, t);
    return keep;
}

// The same test from the other side, for a short v and a long e: lane l keeps
// v unless some lane of e holds it, found by one ballot per lane of v below nv
// (the lanes holding v values) instead of one comparison per lane of e.
__device__ inline bool absent_from(int32_t v, int32_t e, int nv) {
    bool keep = v != SG_NONE;
    const int l = lane_id();
    for (int t = 0; t < nv; ++t) {
        const int32_t x = __builtin_amdgcn_readlane(v, t);
        const bool found = __builtin_amdgcn_ballot_w64(e == x) != 0;
        keep &= !(found && l == t);
    }
    return keep;
}

// Lanes below the highest lane holding a value (0 when none).
__device__ inline int span_of(int32_t v) {
    const uint64_t m = __builtin_amdgcn_ballot_w64(v != SG_NONE);
    return m ? 64 - __builtin_clzll(m) : 0;
}

// Ascending sort of one 32-bit key per lane when only the lanes below m (a
// wave-uniform count) hold keys and the rest hold the all-ones key: after the
// bitonic stage of block size k, lanes 0..k-1 are ascending, so the stages
// stop once m <= k (10 compare-exchange steps for m <= 16, 15 for m <= 32,
// all 21 beyond).
__device__ inline uint32_t wave_sort_u32_first(uint32_t x, int m) {
    const int l = lane_id();
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
        if (m <= (k >> 1)) break;
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint32_t o = lane_xor(x, j);
            x = (o < x) == (((l & k) == 0) == ((l & j) == 0)) ? o : x;
        }
    }
    return x;
}

// NB: the reverse list is cut to its 64 * NB smallest keys (NB = 1 for
// R <= 64, 2 for R <= 128), which always suffices: h = ceil(R/2) <= 32 * NB
// entries of P(y) come first, so at most that many of the smallest keys are
// repeats, and the rest fill the R - h places left before P(y)[h:R] is reached.
template <typename KT, int NB>
__global__ __launch_bounds__(256) void combine_kernel(const int32_t* __restrict__ P, int64_t n, int R,
                                                      const int64_t* __restrict__ cnts, int cap,
                                                      const KT* __restrict__ rev,
                                                      const int64_t* __restrict__ oof,
                                                      const KT* __restrict__ over,
                                                      const int32_t* __restrict__ order,
                                                      const int32_t* __restrict__ order_bad,
                                                      int32_t* __restrict__ F) {
    using RK = RevKey<KT>;
    const int l = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t slot = xcd_contiguous(blockIdx.x, gridDim.x) * WAVES + w;
    if (slot >= n) return;
    const int64_t y = visit_row(order, order_bad, slot);
    const int h = (R + 1) / 2;
    const int64_t cnt = cnts[y];
    const KT* bk = rev + y * cap;
    const int64_t ob = cnt > cap ? oof[y] : 0;
    // reverse key i of y (EMPTY past the in-degree): bucket, then overflow area
    auto key_at = [&](int64_t i) -> KT { return i < cnt ? (i < cap ? bk[i] : over[ob + (i - cap)]) : RK::EMPTY; };
    // the 64 * NB smallest reverse keys, ascending: element p * 64 + l in best[p]
    KT best[NB];
    if constexpr (NB == 1)   // a low in-degree sorts only the lanes it fills
        best[0] = wave_sort_u32_first(key_at(l), __builtin_amdgcn_readfirstlane((int)(cnt < 64 ? cnt : 64)));
    else
        best[0] = RK::sort(key_at(l));
    if constexpr (NB == 2) {
        // two sorted runs; the second reversed makes the pair one bitonic sequence
        const KT v = RK::sort(key_at(64 + l));
        best[1] = RK::from_lane(v, 63 - l);
        const KT lo = best[0] < best[1] ? best[0] : best[1], hi = best[0] < best[1] ? best[1] : best[0];
        best[0] = bitonic_finish(lo);
        best[1] = bitonic_finish(hi);
    }
    for (int64_t c0 = 64 * NB; c0 < cnt; c0 += 64) {
        const KT v = RK::sort(key_at(c0 + l));
        // the element-wise minimum of the list's last run and the reversed new
        // run leaves the 64 * NB smallest of both as a bitonic sequence
        const KT vr = RK::from_lane(v, 63 - l);
        best[NB - 1] = best[NB - 1] < vr ? best[NB - 1] : vr;
        if constexpr (NB == 2) {
            const KT lo = best[0] < best[1] ? best[0] : best[1], hi = best[0] < best[1] ? best[1] : best[0];
            best[0] = bitonic_finish(lo);
            best[1] = bitonic_finish(hi);
        } else {
            best[0] = bitonic_finish(best[0]);
        }
    }
    // the sequence P(y)[0:h] ++ Rev(y) ++ P(y)[h:R], deduplicated in order
    // and cut at R: segment A in lanes 0..h-1, B (the smallest reverse keys'
    // sources, by (p, x)) in lanes 0..63 of each best[], C in lanes 0..R-h-1
    const int32_t va = l < h ? P[y * R + l] : SG_NONE;
    const int32_t vc = l < R - h ? P[y * R + h + l] : SG_NONE;
    // (every ballot and lane read below runs with all lanes active: a span
    // taken under a lane condition would miss the other lanes' values)
    const int spa = span_of(va), spc = span_of(vc);
    int32_t vb[NB];
    bool kb[NB];
    bool kc = vc != SG_NONE;
#pragma unroll
    for (int p = 0; p < NB; ++p) {
        vb[p] = best[p] != RK::EMPTY ? RK::source(best[p]) : SG_NONE;
        kb[p] = first_occurrence(vb[p], va, spa);
        const bool c_new = absent_from(vc, vb[p], spc);
        kc = kc & c_new;
    }
    const uint64_t below = (1ull << l) - 1;
    const bool ka = va != SG_NONE;
    const uint64_t ma = __builtin_amdgcn_ballot_w64(ka), mc = __builtin_amdgcn_ballot_w64(kc);
    int32_t* row = F + y * R;
    int pos0 = __builtin_popcountll(ma);
    if (ka) row[__builtin_popcountll(ma & below)] = va;              // ca <= h <= R
#pragma unroll
    for (int p = 0; p < NB; ++p) {
        const uint64_t mb = __builtin_amdgcn_ballot_w64(kb[p]);
        if (kb[p]) {
            const int pos = pos0 + __builtin_popcountll(mb & below);
            if (pos < R) row[pos] = vb[p];
        }
        pos0 += __builtin_popcountll(mb);
    }
    if (kc) {
        const int pos = pos0 + __builtin_popcountll(mc & below);
        if (pos < R) row[pos] = vc;
    }
    const int total = pos0 + __builtin_popcountll(mc);
    for (int r = l; r < R; r += 64)
        if (r >= total) row[r] = SG_NONE;
}

struct Layout {
    size_t P, rslot, cnt, ovn, oof, rev, over, scan, seen, total;
};

// Reverse keys are 4 bytes for R <= 64, 8 beyond.
inline size_t rev_bytes(int R) { return R <= 64 ? 4 : 8; }

inline Layout layout(int64_t n, int R) {
    Layout L;
    L.P = align_up((size_t)n * R * 4, 256);
    L.rslot = align_up((size_t)n * R * 4, 256);
    L.cnt = align_up((size_t)(n + 1) * 8, 256);
    L.ovn = align_up((size_t)(n + 1) * 8, 256);
    L.oof = align_up((size_t)(n + 1) * 8, 256);
    L.rev = align_up((size_t)n * bucket_cap(R) * rev_bytes(R), 256);
    L.over = align_up((size_t)n * R * rev_bytes(R), 256);   // at most every edge overflows
    L.scan = align_up(exclusive_scan_tmp_bytes(n), 256);
    L.seen = align_up((size_t)(n + 64) * 4, 256);   // order check: per-row counters + flag
    L.total = L.P + L.rslot + L.cnt + L.ovn + L.oof + L.rev + L.over + L.scan + L.seen + 1024;
    return L;
}

inline void check_args(const int32_t* knn, int64_t n, int K, int R, int32_t* out) {
    SG_REQUIRE(n >= 0 && n <= MAX_ROWS, "n out of range (at most 2^26 - 1024 rows)");
    SG_REQUIRE(K >= 1 && K <= 256, "K must be in 1..256");
    SG_REQUIRE(R >= 1 && R <= K && R <= 128, "R must be in 1..min(K, 128)");
    SG_REQUIRE(n == 0 || (knn != nullptr && out != nullptr), "NULL pointer");
}

// The prune's launches on a workspace of layout(n, R).total bytes at ws
// (arguments already checked, n > 0).  Every buffer the kernels read is
// written or cleared here first, so the workspace may hold anything.
inline void enqueue(const int32_t* knn, int64_t n, int K, int R, const int32_t* order, int32_t* out, void* ws,
                    hipStream_t s) {
    Carver cv(ws);
    int32_t* P = cv.take<int32_t>((size_t)n * R);
    int32_t* rslot = cv.take<int32_t>((size_t)n * R);
    int64_t* cnt = cv.take<int64_t>(n + 1);
    int64_t* ovn = cv.take<int64_t>(n + 1);
    int64_t* oof = cv.take<int64_t>(n + 1);
    const int cap = bucket_cap(R);
    void* rev = cv.take<char>((size_t)n * cap * rev_bytes(R));
    void* over = cv.take<char>((size_t)n * R * rev_bytes(R));
    void* scan_tmp = cv.take<char>(exclusive_scan_tmp_bytes(n));
    int32_t* seen = cv.take<int32_t>(n + 64);
    int32_t* order_bad = seen + n;

    unsigned grid = (unsigned)cdiv(n, WAVES);
    fill<int64_t>(cnt, 0, n + 1, s);
    if (order) {   // a non-permutation falls back to row order (same result)
        fill<int32_t>(seen, 0, n + 1, s);
        order_check_kernel<<<(unsigned)std::min<int64_t>(cdiv(n, 256), 4096), 256, 0, s>>>(order, n, seen,
                                                                                          order_bad);
        SG_LAUNCH_CHECK();
    }
    if (K <= 64)
        detour_kernel<1, 256><<<grid, 256, 0, s>>>(knn, n, K, R, order, order_bad, P, rslot, cnt, cap,
                                                     rev);
    else if (K <= 128)
        detour_kernel<2, 256><<<grid, 256, 0, s>>>(knn, n, K, R, order, order_bad, P, rslot, cnt, cap,
                                                     rev);
    else
        detour_kernel<4, 512><<<grid, 256, 0, s>>>(knn, n, K, R, order, order_bad, P, rslot, cnt, cap,
                                                     rev);
    SG_LAUNCH_CHECK();
    int64_t total = n * (int64_t)R;
    const unsigned og = (unsigned)std::min<int64_t>(cdiv(total, 1024), 8192);   // four slots per thread
    excess_kernel<<<(unsigned)std::min<int64_t>(cdiv(n, 256), 4096), 256, 0, s>>>(cnt, n, cap, ovn);
    SG_LAUNCH_CHECK();
    exclusive_scan_i64(ovn, oof, n, scan_tmp, s);
    if (R <= 64) {
        overflow_kernel<uint32_t><<<og, 256, 0, s>>>(P, rslot, total, R, cap, oof, static_cast<uint32_t*>(over));
        SG_LAUNCH_CHECK();
        combine_kernel<uint32_t, 1><<<grid, 256, 0, s>>>(P, n, R, cnt, cap, static_cast<const uint32_t*>(rev), oof,
                                                         static_cast<const uint32_t*>(over), order, order_bad, out);
    } else {
        overflow_kernel<uint64_t><<<og, 256, 0, s>>>(P, rslot, total, R, cap, oof, static_cast<uint64_t*>(over));
        SG_LAUNCH_CHECK();
        combine_kernel<uint64_t, 2><<<grid, 256, 0, s>>>(P, n, R, cnt, cap, static_cast<const uint64_t*>(rev), oof,
                                                         static_cast<const uint64_t*>(over), order, order_bad, out);
    }
    SG_LAUNCH_CHECK();
}

// Scratch of sg_prune_noalloc: a file-scope device array (each GPU the
// library runs on holds its own copy until the process ends).  Host code
// never passes its name to a kernel: the device address of each GPU's copy
// is looked up once, with that GPU current, and kept per device.
constexpr size_t NOALLOC_BYTES = SG_PRUNE_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];
constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[MAX_DEVICES] = {};

inline void* scratch_of_current_device() {
    int dev = 0;
    SG_HIP(hipGetDevice(&dev));
    SG_REQUIRE(dev >= 0 && dev < MAX_DEVICES, "device index out of range for the static scratch");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        SG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        SG_REQUIRE(p != nullptr, "no device address for the static scratch");
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
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
        prune::check_args(knn, n, K, R, out);
        if (n == 0) return;
        const prune::Layout L = prune::layout(n, R);
        if (ws == nullptr || ws_bytes < L.total) {
            set_error("sg_prune: workspace too small (need " + std::to_string(L.total) + " bytes)");
            throw Fail{SG_ERR_WORKSPACE};
        }
        prune::enqueue(knn, n, K, R, order, out, ws, as_stream(stream));
    });
}

extern "C" sg_status sg_prune_noalloc(const int32_t* knn, int64_t n, int32_t K, int32_t R, const int32_t* order,
                                      int32_t* out, void* stream) {
    return guarded([&] {
        prune::check_args(knn, n, K, R, out);
        if (n == 0) return;
        const prune::Layout L = prune::layout(n, R);
        if (L.total > prune::NOALLOC_BYTES) {
            set_error("sg_prune_noalloc: n = " + std::to_string(n) + ", R = " + std::to_string(R) + " needs " +
                      std::to_string(L.total) + " bytes of scratch; the static scratch holds " +
                      std::to_string(prune::NOALLOC_BYTES) + " (use sg_prune with a workspace)");
            throw Fail{SG_ERR_ARG};
        }
        prune::enqueue(knn, n, K, R, order, out, prune::scratch_of_current_device(), as_stream(stream));
    });
}

// merge.hip -- edge-union merge of shard graphs over replicated vectors
// (Sec. II-A, Sec. IV step 3).
//
//  * count_kernel: occurrences of every global id over all shard rows.
//  * exclusive scan -> per-id offsets; scatter_kernel is launched once per
//    shard, in ascending shard order.  A global id occurs at most once per
//    shard (member lists are sets), so its slots fill in ascending shard
//    order whatever the thread timing: the layout is deterministic.  Each slot
//    records the row of the occurrence and its shard's first row.
//  * merge_kernel: one wave per global id.  The lists of its m occurrences are
//    read position-major (pos 0 of every occurrence, then pos 1, ...),
//    translated to global ids and appended in that order without repeats or
//    self, up to max_degree.  Within a chunk of 64 entries the first
//    occurrence of each id is found by a wave sort of (id, lane) keys; against
//    the ids kept from earlier chunks by comparison.
#include "common.hpp"

namespace sg {
namespace merge {

constexpr int WAVES = 4;
constexpr int MAX_DEG = 1024;

// member ids outside [0, n_global) are ignored (never dereferenced)
__global__ void count_kernel(const int32_t* __restrict__ member_ids, int64_t total, int64_t n_global,
                             int64_t* __restrict__ cnt) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < total;
         r += (int64_t)gridDim.x * blockDim.x) {
        int32_t g = member_ids[r];
        if (g >= 0 && g < n_global) atomicAdd(reinterpret_cast<unsigned long long*>(&cnt[g]), 1ull);
    }
}

// rows [r0, r1) of one shard whose first row is r0
__global__ void scatter_kernel(const int32_t* __restrict__ member_ids, int64_t r0, int64_t r1,
                               int64_t n_global, const int64_t* __restrict__ off, int64_t* __restrict__ fillc,
                               int32_t* __restrict__ occ_row, int32_t* __restrict__ occ_base) {
    for (int64_t r = r0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < r1;
         r += (int64_t)gridDim.x * blockDim.x) {
        int32_t g = member_ids[r];
        if (g < 0 || g >= n_global) continue;
        int64_t slot = off[g] + fillc[g];
        fillc[g] += 1;                       // unique g within a shard: no race
        occ_row[slot] = (int32_t)r;      // rows < MAX_ROWS < 2^26
        occ_base[slot] = (int32_t)r0;
    }
}

// Global ids per wave: the gathers of their first chunks are issued together,
// so that one id's dependent loads wait while the other's are in flight.
constexpr int IDS = 2;

__global__ __launch_bounds__(256) void merge_kernel(
    const int32_t* __restrict__ member_ids, const int32_t* __restrict__ graphs, int R,
    int64_t total_rows, int64_t n_global, int max_degree, const int64_t* __restrict__ off,
    const int32_t* __restrict__ occ_row, const int32_t* __restrict__ occ_base,
    int32_t* __restrict__ out, int32_t* __restrict__ degree) {
    __shared__ int32_t s_kl[WAVES][MAX_DEG];
    __shared__ int32_t s_chunk[WAVES][64];
    const int l = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t g0 = ((int64_t)blockIdx.x * WAVES + w) * IDS;
    if (g0 >= n_global) return;
    int32_t* kl = s_kl[w];
    int32_t* chunk = s_chunk[w];
    int64_t gi[IDS], bi[IDS];
    uint32_t mi[IDS];   // occurrences: <= S when member lists are sets
    uint64_t Li[IDS];
#pragma unroll
    for (int i = 0; i < IDS; ++i) {
        gi[i] = g0 + i;
        const bool ok = gi[i] < n_global;
        bi[i] = ok ? off[gi[i]] : 0;
        mi[i] = ok ? (uint32_t)(off[gi[i] + 1] - bi[i]) : 0u;
        Li[i] = (uint64_t)mi[i] * (uint64_t)R;
    }
    // Global id of list entry e of id i (position-major: position e / m of
    // occurrence e % m), or SG_NONE: absent, self, or out of range.
    auto finish = [&](int i, bool live, int32_t lv, int64_t base, int32_t gv) -> int32_t {
        // ids outside [0, n_global) are skipped (so every kept id is < 2^26)
        return live && lv >= 0 && base + lv < total_rows && gv != (int32_t)gi[i] && gv >= 0 && gv < n_global
                   ? gv : SG_NONE;
    };
    // the first chunk of every id, stage by stage over the ids, without
    // branches: lanes past an id's list read index 0 (in bounds, as
    // total_rows > 0 here) and are masked afterwards
    int32_t v0[IDS];
    if (total_rows > 0) {
        bool live[IDS];
        uint32_t pos[IDS];
        int64_t orow[IDS], obase[IDS];
#pragma unroll
        for (int i = 0; i < IDS; ++i) {
            live[i] = (uint64_t)l < Li[i];
            const uint32_t m1 = mi[i] > 0 ? mi[i] : 1u;
            const uint32_t p_ = (uint32_t)l / m1;
            const int64_t oi = live[i] ? bi[i] + ((uint32_t)l - p_ * m1) : 0;
            const int32_t r_ = occ_row[oi], b_ = occ_base[oi];
            orow[i] = live[i] ? r_ : 0;
            obase[i] = live[i] ? b_ : 0;
            pos[i] = live[i] ? p_ : 0u;
        }
        int32_t lv[IDS];
#pragma unroll
        for (int i = 0; i < IDS; ++i) lv[i] = graphs[orow[i] * R + pos[i]];
#pragma unroll
        for (int i = 0; i < IDS; ++i) {
            const int64_t mr = obase[i] + lv[i];
            const bool ok = live[i] && lv[i] >= 0 && mr < total_rows;
            v0[i] = finish(i, live[i], lv[i], obase[i], member_ids[ok ? mr : 0]);
        }
    } else {
#pragma unroll
        for (int i = 0; i < IDS; ++i) v0[i] = SG_NONE;
    }
    // Appends the chunk's first occurrences (in lane order) not yet kept:
    // sort (id, lane) and flag the first lane of each run of equal ids at the
    // lane it came from; then compare with the ids kept from earlier chunks.
    auto append = [&](int32_t v, int kc) -> int {
        const uint32_t sk = v != SG_NONE ? ((uint32_t)v << 6) | (uint32_t)l : 0xFFFFFFFFu;
        const uint32_t srt = wave_sort_u32(sk);
        const uint32_t prev = (uint32_t)__shfl((int)srt, l > 0 ? l - 1 : 0, 64);
        if (srt != 0xFFFFFFFFu) chunk[srt & 63u] = (l == 0 || (prev >> 6) != (srt >> 6)) ? 1 : 0;
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        bool keep = v != SG_NONE && chunk[l] != 0;
        for (int t = 0; t < kc && keep; ++t) keep = kl[t] != v;
        const uint64_t mk = __builtin_amdgcn_ballot_w64(keep);
        const int p = kc + __builtin_popcountll(mk & ((1ull << l) - 1));
        if (keep && p < max_degree) kl[p] = v;
        kc += __builtin_popcountll(mk);
        if (kc > max_degree) kc = max_degree;
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        return kc;
    };
#pragma unroll
    for (int i = 0; i < IDS; ++i) {
        if (gi[i] >= n_global) break;
        const int64_t b = bi[i];
        const uint32_t m = mi[i];
        const uint64_t L = Li[i];
        int kc = append(v0[i], 0);
        // further chunks (an id in more than 64 / R shards)
        for (uint64_t e0 = 64; e0 < L && kc < max_degree; e0 += 64) {
            const uint64_t e = e0 + l;
            int32_t v = SG_NONE;
            if (e < L) {
                // 32-bit division while e fits, the usual case
                uint32_t pos, t;
                if (e0 < 0xFFFFFF00ull) {
                    pos = (uint32_t)e / m;
                    t = (uint32_t)e - pos * m;
                } else {
                    pos = (uint32_t)(e / m);
                    t = (uint32_t)(e - (uint64_t)pos * m);
                }
                const int64_t r = occ_row[b + t];
                const int32_t lv = graphs[r * R + pos];
                const int64_t base = occ_base[b + t];
                const bool ok = lv >= 0 && base + lv < total_rows;   // out-of-range local ids count as absent
                v = finish(i, true, lv, base, ok ? member_ids[base + lv] : SG_NONE);
            }
            kc = append(v, kc);
        }
        int32_t* o = out + gi[i] * max_degree;
        for (int q = l; q < max_degree; q += 64) o[q] = q < kc ? kl[q] : SG_NONE;
        if (l == 0) degree[gi[i]] = kc;
        // kl is rewritten by the next id: every lane has read its entries
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    }
}

struct Layout {
    size_t cnt, off, fillc, occ_row, occ_base, scan, total;
};

inline Layout layout(int64_t total_rows, int64_t n_global) {
    Layout L;
    L.cnt = align_up((size_t)(n_global + 1) * 8, 256);
    L.off = L.cnt;
    L.fillc = L.cnt;
    L.occ_row = align_up((size_t)std::max<int64_t>(total_rows, 1) * 4, 256);
    L.occ_base = L.occ_row;
    L.scan = align_up(exclusive_scan_tmp_bytes(n_global), 256);
    L.total = L.cnt + L.off + L.fillc + L.occ_row + L.occ_base + L.scan + 1024;
    return L;
}

}  // namespace merge
}  // namespace sg

using namespace sg;

extern "C" sg_status sg_merge_workspace_size(int32_t S, const int64_t* shard_offsets_h,
                                             int64_t n_global, size_t* bytes) {
    return guarded([&] {
        SG_REQUIRE(bytes != nullptr && shard_offsets_h != nullptr, "NULL pointer");
        SG_REQUIRE(S >= 1 && n_global >= 0, "bad sizes");
        *bytes = merge::layout(shard_offsets_h[S], n_global).total;
    });
}

extern "C" sg_status sg_merge(int32_t S, const int64_t* shard_offsets_h, const int32_t* member_ids,
                              const int32_t* graphs, int32_t R, int64_t n_global, int32_t max_degree,
                              int32_t* out, int32_t* degree, void* ws, size_t ws_bytes, void* stream) {
    return guarded([&] {
        SG_REQUIRE(S >= 1 && S <= 65536, "S must be in 1..65536");
        SG_REQUIRE(shard_offsets_h != nullptr, "shard_offsets_h is NULL");
        SG_REQUIRE(shard_offsets_h[0] == 0, "shard_offsets_h[0] must be 0");
        for (int s = 0; s < S; ++s)
            SG_REQUIRE(shard_offsets_h[s + 1] >= shard_offsets_h[s],
                       "shard offsets must be non-decreasing");
        SG_REQUIRE(R >= 1 && R <= 256, "R must be in 1..256");
        SG_REQUIRE(max_degree >= 1 && max_degree <= merge::MAX_DEG, "max_degree must be in 1..1024");
        SG_REQUIRE(n_global >= 0 && n_global <= MAX_ROWS, "n_global out of range (at most 2^26 - 1024)");
        if (n_global == 0) return;
        SG_REQUIRE(out != nullptr && degree != nullptr, "NULL output");
        const int64_t total = shard_offsets_h[S];
        SG_REQUIRE(total <= MAX_ROWS, "too many shard rows (at most 2^26 - 1024)");
        SG_REQUIRE(total == 0 || (member_ids != nullptr && graphs != nullptr), "NULL input");
        merge::Layout L = merge::layout(total, n_global);
        if (ws == nullptr || ws_bytes < L.total) {
            set_error("sg_merge: workspace too small (need " + std::to_string(L.total) + " bytes)");
            throw Fail{SG_ERR_WORKSPACE};
        }
        hipStream_t s = as_stream(stream);
        Carver cv(ws);
        int64_t* cnt = cv.take<int64_t>(n_global + 1);
        int64_t* off = cv.take<int64_t>(n_global + 1);
        int64_t* fillc = cv.take<int64_t>(n_global + 1);
        int32_t* occ_row = cv.take<int32_t>(std::max<int64_t>(total, 1));
        int32_t* occ_base = cv.take<int32_t>(std::max<int64_t>(total, 1));
        void* scan_tmp = cv.take<char>(exclusive_scan_tmp_bytes(n_global));
        fill<int64_t>(cnt, 0, n_global + 1, s);
        fill<int64_t>(fillc, 0, n_global + 1, s);
        if (total > 0) {
            unsigned eg = (unsigned)std::min<int64_t>(cdiv(total, 256), 8192);
            merge::count_kernel<<<eg, 256, 0, s>>>(member_ids, total, n_global, cnt);
            SG_LAUNCH_CHECK();
        }
        exclusive_scan_i64(cnt, off, n_global, scan_tmp, s);
        for (int sh = 0; sh < S; ++sh) {
            const int64_t r0 = shard_offsets_h[sh], r1 = shard_offsets_h[sh + 1];
            if (r1 == r0) continue;
            unsigned sg_ = (unsigned)std::min<int64_t>(cdiv(r1 - r0, 256), 4096);
            merge::scatter_kernel<<<sg_, 256, 0, s>>>(member_ids, r0, r1, n_global, off, fillc, occ_row,
                                                      occ_base);
            SG_LAUNCH_CHECK();
        }
        merge::merge_kernel<<<(unsigned)cdiv(n_global, merge::WAVES * merge::IDS), 256, 0, s>>>(
            member_ids, graphs, R, total, n_global, max_degree, off, occ_row, occ_base, out, degree);
        SG_LAUNCH_CHECK();
    });
}

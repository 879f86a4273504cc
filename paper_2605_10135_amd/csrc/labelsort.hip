// labelsort.hip -- stable sort of rows by a small integer label.
//
// The locality order of the shard build groups rows by their nearest pivot;
// within a label rows keep ascending row order, so the order (which sg_knn_graph
// returns and sg_prune takes) is the same on every run.  LSD radix sort with
// 8-bit digits, one pass per digit:
//  * count: per block of 4096 keys, a 256-bucket histogram in LDS, written
//    digit-major (cnt[digit * nb + block]), so that one exclusive scan of the
//    whole matrix gives every (digit, block) its first output position;
//  * place: each block walks its keys in 16 rounds of 256 in index order; a
//    wave finds the lanes sharing its digit with eight ballots (no atomics),
//    ranks itself among them, and adds the counts of the block's earlier waves
//    and rounds -- a stable placement, identical on every run.
#include <algorithm>

#include "common.hpp"

namespace sg {
namespace lsort {

constexpr int THREADS = 256;
constexpr int ROUNDS = 16;
constexpr int BLOCK_KEYS = THREADS * ROUNDS;
constexpr int RADIX = 256;

__global__ __launch_bounds__(THREADS) void digit_count_kernel(const int32_t* __restrict__ key, int64_t n, int shift,
                                                              int64_t nb, int64_t* __restrict__ cnt) {
    __shared__ int h[RADIX];
    const int t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * BLOCK_KEYS;
    for (int r = 0; r < ROUNDS; ++r) {
        const int64_t i = b0 + r * THREADS + t;
        if (i < n) atomicAdd(&h[((uint32_t)key[i] >> shift) & (RADIX - 1)], 1);
    }
    __syncthreads();
    cnt[(int64_t)t * nb + blockIdx.x] = h[t];
}

// kin/rin: keys and their rows (rin NULL: the rows are the indices); off: the
// scanned count matrix.
__global__ __launch_bounds__(THREADS) void digit_place_kernel(const int32_t* __restrict__ kin,
                                                              const int32_t* __restrict__ rin, int64_t n, int shift,
                                                              int64_t nb, const int64_t* __restrict__ off,
                                                              int32_t* __restrict__ kout, int32_t* __restrict__ rout) {
    __shared__ int64_t base[RADIX];
    __shared__ int wc[THREADS / 64][RADIX];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const uint64_t below = (1ull << l) - 1;
    base[t] = off[(int64_t)t * nb + blockIdx.x];
    const int64_t b0 = (int64_t)blockIdx.x * BLOCK_KEYS;
    for (int r = 0; r < ROUNDS; ++r) {
        const int64_t i = b0 + r * THREADS + t;
        const bool valid = i < n;
        const int32_t k = valid ? kin[i] : 0;
        const int dig = (int)(((uint32_t)k >> shift) & (RADIX - 1));
        // lanes of this wave with the same digit
        uint64_t same = __builtin_amdgcn_ballot_w64(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (dig >> bit) & 1;
            const uint64_t m = __builtin_amdgcn_ballot_w64(on);
            same &= on ? m : ~m;
        }
        const int rank = __builtin_popcountll(same & below);
#pragma unroll
        for (int u = 0; u < THREADS / 64; ++u) wc[u][t] = 0;
        __syncthreads();
        if (valid && rank == 0) wc[w][dig] = __builtin_popcountll(same);
        __syncthreads();
        if (valid) {
            int before = 0;
            for (int u = 0; u < w; ++u) before += wc[u][dig];
            const int64_t pos = base[dig] + before + rank;
            kout[pos] = k;
            rout[pos] = rin ? rin[i] : (int32_t)i;
        }
        __syncthreads();
        int tot = 0;
#pragma unroll
        for (int u = 0; u < THREADS / 64; ++u) tot += wc[u][t];
        base[t] += tot;
        __syncthreads();
    }
}

inline int passes_for(int bits) { return bits <= 8 ? 1 : (bits + 7) / 8; }

}  // namespace lsort

size_t label_sort_tmp_bytes(int64_t n, int bits) {
    const int64_t nb = (n + lsort::BLOCK_KEYS - 1) / lsort::BLOCK_KEYS;
    const int64_t m = (int64_t)lsort::RADIX * std::max<int64_t>(nb, 1);
    (void)bits;
    return 3 * align_up((size_t)std::max<int64_t>(n, 1) * 4, 256) + 2 * align_up((size_t)(m + 1) * 8, 256) +
           align_up(exclusive_scan_tmp_bytes(m), 256);
}

void label_sort(const int32_t* lab, int64_t n, int bits, int32_t* rows_out, void* tmp, hipStream_t s) {
    if (n <= 0) return;
    const int64_t nb = (n + lsort::BLOCK_KEYS - 1) / lsort::BLOCK_KEYS;
    const int64_t m = (int64_t)lsort::RADIX * nb;
    Carver cv(tmp);
    int32_t* kA = cv.take<int32_t>(n);
    int32_t* kB = cv.take<int32_t>(n);
    int32_t* rA = cv.take<int32_t>(n);
    int64_t* cnt = cv.take<int64_t>(m + 1);
    int64_t* off = cv.take<int64_t>(m + 1);
    void* scan_tmp = cv.take<char>(exclusive_scan_tmp_bytes(m));
    int32_t* rB = rows_out;   // the last pass always writes rows_out (see below)
    const int P = lsort::passes_for(bits);
    for (int p = 0; p < P; ++p) {
        const int32_t* kin = p == 0 ? lab : ((p - 1) % 2 == 0 ? kA : kB);
        int32_t* kout = p % 2 == 0 ? kA : kB;
        // rows ping-pong between rA and rows_out so that pass P-1 lands in rows_out
        const bool to_out = ((P - 1 - p) % 2) == 0;
        const int32_t* rin = p == 0 ? nullptr : (to_out ? rA : rB);
        int32_t* rout = to_out ? rB : rA;
        lsort::digit_count_kernel<<<(unsigned)nb, lsort::THREADS, 0, s>>>(kin, n, 8 * p, nb, cnt);
        SG_LAUNCH_CHECK();
        exclusive_scan_i64(cnt, off, m, scan_tmp, s);
        lsort::digit_place_kernel<<<(unsigned)nb, lsort::THREADS, 0, s>>>(kin, rin, n, 8 * p, nb, off, kout, rout);
        SG_LAUNCH_CHECK();
    }
}

}  // namespace sg

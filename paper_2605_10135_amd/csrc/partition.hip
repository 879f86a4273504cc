// partition.hip -- k-means partition with selective replication
// (Sec. IV step 1; Sec. V-B and Algorithm 1 for one in-memory block).
//
//  * assign_kernel: nearest centroid per row (FP32 squared L2 against FP32
//    copies of the FP64 centroids, summed per centroid in ascending dimension
//    order, ties to the lower index); rows are staged through LDS, one thread
//    per row, every centroid's sum in a register.
//  * sum_kernel / finalize_kernel: FP64 centroid sums in a fixed-order
//    two-level reduction.  A block owns a contiguous row range and a 128-wide
//    slice of dimensions; thread t alone accumulates dimension t of every
//    cluster in LDS, walking its rows in ascending order, so each partial sum
//    has one fixed order.  The finalize pass adds the partials in block order.
//    No floating-point atomics are involved: results are bit-reproducible.
//  * radius_kernel, replica_kernel: the radius of each cluster (largest
//    Euclidean distance of a primary member; a max, so order-free) and the
//    Algorithm 1 rule: visit centroids by ascending distance, join c' when
//    d' < eps*d and d' < eps*tau*r[c'], until omega shards.
//  * membership: per (shard, block) counts, one exclusive scan over the
//    shard-major count matrix, then each block writes its members of every
//    shard at the scanned offset in row order (a block scan per shard), so
//    each shard's list is ascending.
#include <cmath>
#include <vector>

#include "common.hpp"

namespace sg {
namespace part {

constexpr int SUM_ROWS = 2048;    // rows per partial-sum block
constexpr int DSLICE = 128;       // dimensions per partial-sum block
constexpr int MAX_S = 64;
constexpr int MAX_OMEGA = 8;
constexpr int MEM_BLOCK = 256;    // rows per membership block

__device__ inline float load_elem(const void* X, int dtype, int64_t idx) {
    switch (dtype) {
        case SG_F32: return static_cast<const float*>(X)[idx];
        case SG_F16: return (float)static_cast<const _Float16*>(X)[idx];
        case SG_BF16: return __builtin_bit_cast(float, (uint32_t) static_cast<const uint16_t*>(X)[idx] << 16);
        default: return (float)static_cast<const uint8_t*>(X)[idx];
    }
}

__device__ inline double load_elem_d(const void* X, int dtype, int64_t idx) {
    return (double)load_elem(X, dtype, idx);   // every stored type widens exactly
}

__global__ void init_centroids(const void* X, int dtype, int64_t ld, int d, int S,
                               const int64_t* __restrict__ init_idx, double* __restrict__ C) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < S * d; e += gridDim.x * blockDim.x) {
        int c = e / d, t = e % d;
        C[e] = load_elem_d(X, dtype, init_idx[c] * ld + t);
    }
}

__global__ void to_f32(const double* __restrict__ C, float* __restrict__ Cf, int m) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gridDim.x * blockDim.x) Cf[e] = (float)C[e];
}

// grid: (row blocks, dimension slices); block: DSLICE threads
__global__ __launch_bounds__(DSLICE) void sum_kernel(const void* __restrict__ X, int dtype, int64_t n,
                                                     int d, int64_t ld, const int32_t* __restrict__ label,
                                                     int S, double* __restrict__ part,
                                                     int64_t* __restrict__ pcount) {
    __shared__ double acc[MAX_S][DSLICE];
    __shared__ int64_t cnt[MAX_S];
    const int t = threadIdx.x;
    const int dim = blockIdx.y * DSLICE + t;
    for (int c = 0; c < S; ++c) acc[c][t] = 0.0;
    if (t < S) cnt[t] = 0;
    __syncthreads();
    const int64_t r0 = (int64_t)blockIdx.x * SUM_ROWS;
    const int64_t r1 = r0 + SUM_ROWS < n ? r0 + SUM_ROWS : n;
    for (int64_t r = r0; r < r1; ++r) {
        const int c = label[r];
        if (dim < d) acc[c][t] += load_elem_d(X, dtype, r * ld + dim);
        if (t == 0 && blockIdx.y == 0) cnt[c] += 1;
    }
    __syncthreads();
    const int64_t pb = (int64_t)blockIdx.x;
    for (int c = 0; c < S; ++c)
        if (dim < d) part[(pb * S + c) * d + dim] = acc[c][t];
    if (blockIdx.y == 0 && t < S) pcount[pb * S + t] = cnt[t];
}

__global__ void finalize_kernel(const double* __restrict__ part, const int64_t* __restrict__ pcount,
                                int nb, int S, int d, double* __restrict__ C) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < S * d; e += gridDim.x * blockDim.x) {
        const int c = e / d, t = e % d;
        double s = 0.0;
        int64_t k = 0;
        for (int b = 0; b < nb; ++b) {
            s += part[((int64_t)b * S + c) * d + t];
            k += pcount[(int64_t)b * S + c];
        }
        if (k > 0) C[e] = s / (double)k;
    }
}

// Squared FP32 distances of each thread's row (row0 + threadIdx.x) to every
// centroid, in the order of the plain per-row loop: for each centroid,
// s = fmaf(x_t - c_t, x_t - c_t, s) for t ascending from s = 0.  Rows are
// staged through LDS in chunks of ADC dimensions, transposed (xs[t][row]) so
// that the global loads are coalesced along rows and the LDS reads are
// conflict-free; the centroids' chunk is staged beside them.
constexpr int AR = 256;    // rows per block, one per thread
constexpr int ADC = 32;    // dimensions per staged chunk

template <int SMAX>
struct DistSmem {
    float xs[ADC][AR + 1];
    float cs[SMAX][ADC];
};

template <int SMAX>
__device__ void row_dists(DistSmem<SMAX>& sm, const void* __restrict__ X, int dtype, int64_t n, int d, int64_t ld,
                          const float* __restrict__ Cf, int S, int64_t row0, float (&acc)[SMAX]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int c = 0; c < SMAX; ++c) acc[c] = 0.f;
    for (int t0 = 0; t0 < d; t0 += ADC) {
        const int dc = d - t0 < ADC ? d - t0 : ADC;
        __syncthreads();
        for (int e = tid; e < AR * ADC; e += AR) {
            const int r = e / ADC, col = e % ADC;
            const int64_t row = row0 + r;
            sm.xs[col][r] = (row < n && col < dc) ? load_elem(X, dtype, row * ld + t0 + col) : 0.f;
        }
        for (int e = tid; e < S * ADC; e += AR) {
            const int c = e / ADC, col = e % ADC;
            sm.cs[c][col] = col < dc ? Cf[(int64_t)c * d + t0 + col] : 0.f;
        }
        __syncthreads();
        for (int col = 0; col < dc; ++col) {
            const float x = sm.xs[col][tid];
#pragma unroll
            for (int c = 0; c < SMAX; ++c) {
                if (c < S) {
                    const float u = x - sm.cs[c][col];
                    acc[c] = fmaf(u, u, acc[c]);
                }
            }
        }
    }
}

// nearest centroid (ties to the lower index) -> label
template <int SMAX>
__global__ __launch_bounds__(AR) void assign_kernel(const void* __restrict__ X, int dtype, int64_t n, int d,
                                                    int64_t ld, const float* __restrict__ Cf, int S,
                                                    int32_t* __restrict__ label) {
    __shared__ DistSmem<SMAX> sm;
    const int64_t row0 = (int64_t)blockIdx.x * AR;
    float acc[SMAX];
    row_dists<SMAX>(sm, X, dtype, n, d, ld, Cf, S, row0, acc);
    const int64_t i = row0 + threadIdx.x;
    if (i >= n) return;
    float best = __builtin_inff();
    int bi = 0;
#pragma unroll
    for (int c = 0; c < SMAX; ++c) {
        if (c < S && acc[c] < best) {
            best = acc[c];
            bi = c;
        }
    }
    label[i] = bi;
}

// radius of each cluster: largest Euclidean distance of a primary member
// (a max of non-negative floats, ordered like their bit patterns: order-free)
template <int SMAX>
__global__ __launch_bounds__(AR) void radius_kernel(const void* __restrict__ X, int dtype, int64_t n, int d,
                                                    int64_t ld, const float* __restrict__ Cf, int S,
                                                    const int32_t* __restrict__ label,
                                                    unsigned int* __restrict__ radius_bits) {
    __shared__ DistSmem<SMAX> sm;
    const int64_t row0 = (int64_t)blockIdx.x * AR;
    float acc[SMAX];
    row_dists<SMAX>(sm, X, dtype, n, d, ld, Cf, S, row0, acc);
    const int64_t i = row0 + threadIdx.x;
    if (i >= n) return;
    const int c0 = label[i];
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < SMAX; ++c)
        if (c == c0) s = acc[c];
    atomicMax(&radius_bits[c0], __builtin_bit_cast(unsigned int, sqrtf(s)));
}

// assign: n x omega shard ids (primary first, -1 padded).  Algorithm 1 for
// one block: visit centroids by ascending (distance, index); join c' when
// d' < eps * d and d' < eps * tau * r[c'] (or always when eps = inf), until
// omega shards.
template <int SMAX>
__global__ __launch_bounds__(AR) void replica_kernel(const void* __restrict__ X, int dtype, int64_t n, int d,
                                                     int64_t ld, const float* __restrict__ Cf, int S,
                                                     const int32_t* __restrict__ label,
                                                     const unsigned int* __restrict__ radius_bits, int omega,
                                                     float eps, float tau, int accept_all,
                                                     int32_t* __restrict__ assign) {
    __shared__ DistSmem<SMAX> sm;
    const int64_t row0 = (int64_t)blockIdx.x * AR;
    float dist[SMAX];
    row_dists<SMAX>(sm, X, dtype, n, d, ld, Cf, S, row0, dist);
    const int64_t i = row0 + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int c = 0; c < SMAX; ++c) dist[c] = sqrtf(dist[c]);
    const int prim = label[i];
    float dc = 0.f;
#pragma unroll
    for (int c = 0; c < SMAX; ++c)
        if (c == prim) dc = dist[c];
    int32_t* a = assign + i * omega;
    a[0] = prim;
    int assigned = 1;
    uint64_t visited = 0;
    for (int step = 0; step < S && assigned < omega; ++step) {
        int bi = -1;
        float bd = 0.f;
#pragma unroll
        for (int c = 0; c < SMAX; ++c) {
            if (c >= S || (visited >> c & 1ull)) continue;
            if (bi < 0 || dist[c] < bd) {
                bi = c;
                bd = dist[c];
            }
        }
        visited |= 1ull << bi;
        if (bi == prim) continue;
        const float r = __builtin_bit_cast(float, radius_bits[bi]);
        if (accept_all || (bd < eps * dc && bd < eps * tau * r)) a[assigned++] = bi;
    }
    for (int k = assigned; k < omega; ++k) a[k] = SG_NONE;
}

// ---------------------------------------------------------------------------
// blockwise-adaptive assignment (Sec. V-A, Sec. V-B, Algorithm 1)
// ---------------------------------------------------------------------------

// Squared FP32 distances of every row to every centroid (the sums of
// row_dists), D2[i * S + c].
template <int SMAX>
__global__ __launch_bounds__(AR) void sqdist_kernel(const void* __restrict__ X, int dtype, int64_t n, int d,
                                                    int64_t ld, const float* __restrict__ Cf, int S,
                                                    float* __restrict__ D2) {
    __shared__ DistSmem<SMAX> sm;
    const int64_t row0 = (int64_t)blockIdx.x * AR;
    float acc[SMAX];
    row_dists<SMAX>(sm, X, dtype, n, d, ld, Cf, S, row0, acc);
    const int64_t i = row0 + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int c = 0; c < SMAX; ++c)
        if (c < S) D2[i * S + c] = acc[c];
}

// d[c] for a run-time c without indexing the register array
template <int SMAX>
__device__ inline float pick(const float (&d)[SMAX], int c) {
    float r = 0.f;
#pragma unroll
    for (int u = 0; u < SMAX; ++u)
        if (u == c) r = d[u];
    return r;
}

// The clusters of one row in visiting order (ascending squared distance,
// ties to the lower index), one at a time: next() returns the next cluster
// or -1 once all S are visited.
template <int SMAX>
struct Visit {
    const float (&d)[SMAX];
    int S;
    uint64_t seen = 0;
    __device__ Visit(const float (&dd)[SMAX], int s) : d(dd), S(s) {}
    __device__ int next() {
        int bi = -1;
        float bd = 0.f;
#pragma unroll
        for (int c = 0; c < SMAX; ++c) {
            if (c >= S || ((seen >> c) & 1ull)) continue;
            if (bi < 0 || d[c] < bd) {
                bi = c;
                bd = d[c];
            }
        }
        if (bi >= 0) seen |= 1ull << bi;
        return bi;
    }
};

// One wave walks the blocks of rows in order.  Cluster state lives in LDS:
// size (members), prim (primaries), rep (replicas), theta (replica
// threshold), R2 (largest squared primary distance, as float bits).  Each
// block: (1) primaries to the nearest available cluster, (2) thresholds,
// (3) replicas by Algorithm 1.  Rows go 64 at a time, one per lane; a chunk
// takes its decisions from the state at its start when no cluster it touches
// crosses a limit within the chunk -- then every lane decides exactly as it
// would row by row -- and otherwise replays the chunk row by row.
//   et2[t]: eps^2 * tau_t^2 of block t (FP32, from the host).
template <int SMAX>
__global__ __launch_bounds__(64) void blockwise_kernel(const float* __restrict__ D2, int64_t n, int S, int omega,
                                                       float eps2, const float* __restrict__ et2,
                                                       int64_t block_rows, int64_t cap, int adaptive,
                                                       int accept_all, int32_t* __restrict__ assign,
                                                       int32_t* __restrict__ primary) {
    __shared__ int64_t size[SMAX], prim[SMAX], rep[SMAX], theta[SMAX];
    __shared__ unsigned int R2[SMAX];
    __shared__ int cnt[SMAX];
    const int l = threadIdx.x;
    const int64_t UNLIMITED = INT64_MAX;
    if (l < SMAX) {
        size[l] = prim[l] = rep[l] = 0;
        theta[l] = UNLIMITED;
        R2[l] = 0u;
        cnt[l] = 0;
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    auto full = [&](int c) { return cap > 0 && size[c] >= cap; };
    auto load_row = [&](int64_t i, float (&d)[SMAX]) {
#pragma unroll
        for (int c = 0; c < SMAX; ++c) d[c] = (i < n && c < S) ? D2[i * S + c] : 0.f;
    };
    // primary of one row under the current sizes (nearest available, else nearest)
    auto choose_primary = [&](const float (&d)[SMAX]) {
        Visit<SMAX> v(d, S);
        int first = -1;
        for (int k = 0; k < S; ++k) {
            const int c = v.next();
            if (first < 0) first = c;
            if (!full(c)) return c;
        }
        return first;
    };
    // replicas of one row under the current state: up to omega - 1 proposals
    auto propose = [&](const float (&d)[SMAX], int c0, float et, int (&out)[8]) {
        const float dc2 = pick(d, c0);
        Visit<SMAX> v(d, S);
        int got = 1;
        for (int k = 0; k < S && got < omega; ++k) {
            const int c = v.next();
            if (c == c0 || full(c) || rep[c] >= theta[c]) continue;
            const float dp2 = pick(d, c);
            if (accept_all || (dp2 < eps2 * dc2 && dp2 < et * __builtin_bit_cast(float, R2[c]))) out[got++] = c;
        }
        return got;
    };

    int64_t t = 0;
    for (int64_t b0 = 0; b0 < n; b0 += block_rows, ++t) {
        const int64_t b1 = b0 + block_rows < n ? b0 + block_rows : n;
        // (1) primaries
        for (int64_t c0 = b0; c0 < b1; c0 += 64) {
            const int64_t i = c0 + l;
            const bool valid = i < b1;
            float d[SMAX];
            load_row(i, d);
            int ch = valid ? choose_primary(d) : 0;
            if (valid) atomicAdd(&cnt[ch], 1);
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            const bool over = valid && cap > 0 && size[ch] + cnt[ch] > cap;
            const bool serial = __builtin_amdgcn_ballot_w64(over) != 0;
            if (!serial) {
                if (l < S) {
                    size[l] += cnt[l];
                    prim[l] += cnt[l];
                }
            } else {
                for (int j = 0; j < 64; ++j) {
                    if (l == j && valid) {
                        ch = choose_primary(d);
                        size[ch] += 1;
                        prim[ch] += 1;
                    }
                    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
                }
            }
            if (valid) {
                atomicMax(&R2[ch], __builtin_bit_cast(unsigned int, pick(d, ch)));
                assign[i * omega] = ch;
                for (int k = 1; k < omega; ++k) assign[i * omega + k] = SG_NONE;
                primary[i] = ch;
            }
            if (l < SMAX) cnt[l] = 0;
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        }
        // (2) thresholds after the block's primaries
        if (l < S) {
            if (cap == 0 || !adaptive) {
                theta[l] = UNLIMITED;
            } else {
                const int64_t expect = (prim[l] * n + b1 - 1) / b1;   // ceil(prim * n / seen)
                theta[l] = cap - expect > 0 ? cap - expect : 0;
            }
        }
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        const float et = et2[t];
        // (3) replicas
        if (omega > 1) {
            for (int64_t c0 = b0; c0 < b1; c0 += 64) {
                const int64_t i = c0 + l;
                const bool valid = i < b1;
                float d[SMAX];
                load_row(i, d);
                const int pc = valid ? assign[i * omega] : 0;
                int out[8];
                int got = valid ? propose(d, pc, et, out) : 1;
                for (int k = 1; k < got; ++k) atomicAdd(&cnt[out[k]], 1);
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
                bool over = false;
                if (l < S && cnt[l] > 0)
                    over = (cap > 0 && size[l] + cnt[l] > cap) || rep[l] + cnt[l] > theta[l];
                const bool serial = __builtin_amdgcn_ballot_w64(over) != 0;
                if (!serial) {
                    if (l < S) {
                        size[l] += cnt[l];
                        rep[l] += cnt[l];
                    }
                } else {
                    for (int j = 0; j < 64; ++j) {
                        if (l == j && valid) {
                            got = propose(d, pc, et, out);
                            for (int k = 1; k < got; ++k) {
                                size[out[k]] += 1;
                                rep[out[k]] += 1;
                            }
                        }
                        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
                    }
                }
                if (valid)
                    for (int k = 1; k < got; ++k) assign[i * omega + k] = out[k];
                if (l < SMAX) cnt[l] = 0;
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            }
        }
    }
}

// per (shard, block) member counts, written shard-major: cm[s * nb + b]
__global__ __launch_bounds__(MEM_BLOCK) void member_count_kernel(const int32_t* __restrict__ assign,
                                                                 int64_t n, int omega, int S, int nb,
                                                                 int64_t* __restrict__ cm) {
    __shared__ int cnt[MAX_S];
    const int t = threadIdx.x;
    if (t < S) cnt[t] = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * MEM_BLOCK + t;
    if (i < n)
        for (int k = 0; k < omega; ++k) {
            int s = assign[i * omega + k];
            if (s >= 0) atomicAdd(&cnt[s], 1);
        }
    __syncthreads();
    if (t < S) cm[(int64_t)t * nb + blockIdx.x] = cnt[t];
}

__global__ __launch_bounds__(MEM_BLOCK) void member_write_kernel(const int32_t* __restrict__ assign,
                                                                 int64_t n, int omega, int S, int nb,
                                                                 const int64_t* __restrict__ cmoff,
                                                                 int64_t capacity,
                                                                 int32_t* __restrict__ member_ids) {
    __shared__ int wsum[MEM_BLOCK / 64];
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int64_t i = (int64_t)blockIdx.x * MEM_BLOCK + t;
    for (int s = 0; s < S; ++s) {
        bool in = false;
        if (i < n)
            for (int k = 0; k < omega; ++k) in |= assign[i * omega + k] == s;
        uint64_t m = __builtin_amdgcn_ballot_w64(in);
        if (lane == 0) wsum[w] = __builtin_popcountll(m);
        __syncthreads();
        int before = 0;
        for (int u = 0; u < w; ++u) before += wsum[u];
        int64_t pos = cmoff[(int64_t)s * nb + blockIdx.x] + before +
                      __builtin_popcountll(m & ((1ull << lane) - 1));
        if (in && pos < capacity) member_ids[pos] = (int32_t)i;
        __syncthreads();
    }
}

struct Layout {
    int nb_sum, nb_mem;
    size_t total;
};

inline Layout layout(int64_t n, int d, int S, int omega) {
    Layout L;
    L.nb_sum = cdiv(n, SUM_ROWS);
    L.nb_mem = cdiv(n, MEM_BLOCK);
    size_t b = 0;
    b += align_up((size_t)S * d * 4, 256);                              // FP32 centroids
    b += align_up((size_t)n * 4, 256);                                  // labels
    b += align_up((size_t)L.nb_sum * S * d * 8, 256);                   // FP64 partials
    b += align_up((size_t)L.nb_sum * S * 8, 256);                       // partial counts
    b += align_up((size_t)S * 4, 256);                                  // radius bits
    b += align_up((size_t)n * omega * 4, 256);                          // assignment
    b += align_up((size_t)((int64_t)S * L.nb_mem + 1) * 8, 256) * 2;    // counts + offsets
    b += align_up(exclusive_scan_tmp_bytes((int64_t)S * L.nb_mem), 256);
    b += align_up((size_t)S * 8, 256);                                  // init rows
    L.total = b + 2048;
    return L;
}

// Blockwise extra: squared distances of every row (n x S FP32) and the
// per-block eps^2 tau_t^2 table.
inline size_t blockwise_extra(int64_t n, int S, int64_t block_rows) {
    const int64_t nblocks = (n + block_rows - 1) / block_rows;
    return align_up((size_t)n * S * 4, 256) + align_up((size_t)nblocks * 4, 256) + 512;
}

// The workspace pieces both entry points share.
struct Bufs {
    float* Cf;
    int32_t* label;
    double* partial;
    int64_t* pcount;
    unsigned int* rbits;
    int32_t* assign;
    int64_t* cm;
    int64_t* cmoff;
    void* scan_tmp;
    int64_t* init_d;
    int64_t ncm;
};

inline Bufs carve(Carver& cv, const Layout& L, int64_t n, int d, int S, int omega) {
    Bufs B;
    B.Cf = cv.take<float>((size_t)S * d);
    B.label = cv.take<int32_t>(n);
    B.partial = cv.take<double>((size_t)L.nb_sum * S * d);
    B.pcount = cv.take<int64_t>((size_t)L.nb_sum * S);
    B.rbits = cv.take<unsigned int>(S);
    B.assign = cv.take<int32_t>((size_t)n * omega);
    B.ncm = (int64_t)S * L.nb_mem;
    B.cm = cv.take<int64_t>(B.ncm + 1);
    B.cmoff = cv.take<int64_t>(B.ncm + 1);
    B.scan_tmp = cv.take<char>(exclusive_scan_tmp_bytes(B.ncm));
    B.init_d = cv.take<int64_t>(S);
    return B;
}

inline int smax_of(int S) { return S <= 8 ? 8 : S <= 16 ? 16 : S <= 32 ? 32 : 64; }

#define SG_BY_SMAX(KERNEL, ...)                                                        \
    do {                                                                               \
        switch (::sg::part::smax_of(S)) {                                              \
            case 8: part::KERNEL<8><<<rg, part::AR, 0, s>>>(__VA_ARGS__); break;       \
            case 16: part::KERNEL<16><<<rg, part::AR, 0, s>>>(__VA_ARGS__); break;     \
            case 32: part::KERNEL<32><<<rg, part::AR, 0, s>>>(__VA_ARGS__); break;     \
            default: part::KERNEL<64><<<rg, part::AR, 0, s>>>(__VA_ARGS__); break;     \
        }                                                                              \
        SG_LAUNCH_CHECK();                                                             \
    } while (0)

// Lloyd k-means (FP64 centroids, fixed-order sums), leaving the FP32 copy of
// the final centroids in B.Cf.
inline void run_kmeans(const void* X, int dtype, int64_t n, int d, int64_t ld, int S, int iters,
                       const int64_t* init_idx_h, double* centroids, const Layout& L, const Bufs& B,
                       hipStream_t s) {
    SG_HIP(hipMemcpyAsync(B.init_d, init_idx_h, S * sizeof(int64_t), hipMemcpyHostToDevice, s));
    init_centroids<<<cdiv((int64_t)S * d, 256), 256, 0, s>>>(X, dtype, ld, d, S, B.init_d, centroids);
    SG_LAUNCH_CHECK();
    const unsigned rg = (unsigned)cdiv(n, AR);
    const unsigned cg = (unsigned)cdiv((int64_t)S * d, 256);
    for (int it = 0; it < iters; ++it) {
        to_f32<<<cg, 256, 0, s>>>(centroids, B.Cf, S * d);
        SG_BY_SMAX(assign_kernel, X, dtype, n, d, ld, B.Cf, S, B.label);
        dim3 sgrid((unsigned)L.nb_sum, (unsigned)cdiv(d, DSLICE));
        sum_kernel<<<sgrid, DSLICE, 0, s>>>(X, dtype, n, d, ld, B.label, S, B.partial, B.pcount);
        finalize_kernel<<<cg, 256, 0, s>>>(B.partial, B.pcount, L.nb_sum, S, d, centroids);
        SG_LAUNCH_CHECK();
    }
    to_f32<<<cg, 256, 0, s>>>(centroids, B.Cf, S * d);
    SG_LAUNCH_CHECK();
}

// CSR membership from the n x omega assignment, then the shard offsets on
// the host (synchronises s).
inline void run_membership(int64_t n, int S, int omega, int64_t capacity, int32_t* member_ids,
                           int64_t* shard_offsets_h, const Layout& L, const Bufs& B, hipStream_t s) {
    member_count_kernel<<<(unsigned)L.nb_mem, MEM_BLOCK, 0, s>>>(B.assign, n, omega, S, L.nb_mem, B.cm);
    SG_LAUNCH_CHECK();
    exclusive_scan_i64(B.cm, B.cmoff, B.ncm, B.scan_tmp, s);
    member_write_kernel<<<(unsigned)L.nb_mem, MEM_BLOCK, 0, s>>>(B.assign, n, omega, S, L.nb_mem, B.cmoff,
                                                                  capacity, member_ids);
    SG_LAUNCH_CHECK();
    std::vector<int64_t> all((size_t)B.ncm + 1);
    SG_HIP(hipMemcpyAsync(all.data(), B.cmoff, (B.ncm + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SG_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < S; ++c) shard_offsets_h[c] = all[(size_t)c * L.nb_mem];
    shard_offsets_h[S] = all[(size_t)B.ncm];
    if (shard_offsets_h[S] > capacity) {
        set_error("sg_partition: membership (" + std::to_string(shard_offsets_h[S]) + ") exceeds capacity");
        throw Fail{SG_ERR_ARG};
    }
}

inline void check_common(const void* X, int dtype, int64_t n, int d, int64_t ld, int S, int omega, int iters,
                         float epsilon, const int64_t* init_idx_h, const double* centroids, const int32_t* primary,
                         const int64_t* shard_offsets_h, const int32_t* member_ids) {
    SG_REQUIRE(n >= 1 && n < (1ll << 31), "n out of range");
    SG_REQUIRE(d >= 1 && d <= 4096, "d must be in 1..4096");
    SG_REQUIRE(ld >= d, "ld must be >= d");
    SG_REQUIRE(S >= 1 && S <= MAX_S, "S must be in 1..64");
    SG_REQUIRE(omega >= 1 && omega <= S && omega <= MAX_OMEGA, "omega must be in 1..min(S, 8)");
    SG_REQUIRE(iters >= 0, "iters must be >= 0");
    SG_REQUIRE(dtype >= SG_F32 && dtype <= SG_U8, "unknown dtype");
    SG_REQUIRE(!(epsilon != epsilon), "epsilon must not be NaN");
    SG_REQUIRE(X && init_idx_h && centroids && primary && shard_offsets_h && member_ids, "NULL pointer");
    for (int c = 0; c < S; ++c) SG_REQUIRE(init_idx_h[c] >= 0 && init_idx_h[c] < n, "init_idx out of range");
}

}  // namespace part
}  // namespace sg

using namespace sg;

extern "C" sg_status sg_partition_workspace_size(int64_t n, int32_t d, int32_t S, int32_t omega,
                                                 size_t* bytes) {
    return guarded([&] {
        SG_REQUIRE(bytes != nullptr, "bytes is NULL");
        SG_REQUIRE(n >= 1 && d >= 1 && S >= 1 && omega >= 1, "bad sizes");
        *bytes = part::layout(n, d, S, omega).total;
    });
}

extern "C" sg_status sg_partition(const void* X, sg_dtype dtype, int64_t n, int32_t d, int64_t ld,
                                  int32_t S, int32_t omega, int32_t iters, float epsilon, float tau,
                                  const int64_t* init_idx_h, double* centroids, int32_t* primary,
                                  int64_t* shard_offsets_h, int32_t* member_ids, int64_t capacity,
                                  void* ws, size_t ws_bytes, void* stream) {
    return guarded([&] {
        part::check_common(X, dtype, n, d, ld, S, omega, iters, epsilon, init_idx_h, centroids, primary,
                           shard_offsets_h, member_ids);
        SG_REQUIRE(!(tau != tau), "tau must not be NaN");
        part::Layout L = part::layout(n, d, S, omega);
        if (ws == nullptr || ws_bytes < L.total) {
            set_error("sg_partition: workspace too small (need " + std::to_string(L.total) + " bytes)");
            throw Fail{SG_ERR_WORKSPACE};
        }
        hipStream_t s = as_stream(stream);
        Carver cv(ws);
        const part::Bufs B = part::carve(cv, L, n, d, S, omega);
        part::run_kmeans(X, dtype, n, d, ld, S, iters, init_idx_h, centroids, L, B, s);
        const unsigned rg = (unsigned)cdiv(n, part::AR);
        SG_BY_SMAX(assign_kernel, X, dtype, n, d, ld, B.Cf, S, B.label);
        fill<unsigned int>(B.rbits, 0u, S, s);
        SG_BY_SMAX(radius_kernel, X, dtype, n, d, ld, B.Cf, S, B.label, B.rbits);
        const int accept_all = std::isinf(epsilon) && epsilon > 0;
        SG_BY_SMAX(replica_kernel, X, dtype, n, d, ld, B.Cf, S, B.label, B.rbits, omega, epsilon, tau, accept_all,
                   B.assign);
        SG_HIP(hipMemcpyAsync(primary, B.label, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        part::run_membership(n, S, omega, capacity, member_ids, shard_offsets_h, L, B, s);
    });
}

extern "C" sg_status sg_partition_blockwise_workspace_size(int64_t n, int32_t d, int32_t S, int32_t omega,
                                                           int64_t block_rows, size_t* bytes) {
    return guarded([&] {
        SG_REQUIRE(bytes != nullptr, "bytes is NULL");
        SG_REQUIRE(n >= 1 && d >= 1 && S >= 1 && omega >= 1 && block_rows >= 1, "bad sizes");
        *bytes = part::layout(n, d, S, omega).total + part::blockwise_extra(n, S, block_rows);
    });
}

extern "C" sg_status sg_partition_blockwise(const void* X, sg_dtype dtype, int64_t n, int32_t d, int64_t ld,
                                            int32_t S, int32_t omega, int32_t iters, float epsilon, float tau0,
                                            int64_t block_rows, int64_t shard_cap, int32_t adaptive,
                                            const int64_t* init_idx_h, double* centroids, int32_t* primary,
                                            int64_t* shard_offsets_h, int32_t* member_ids, int64_t capacity,
                                            void* ws, size_t ws_bytes, void* stream) {
    return guarded([&] {
        part::check_common(X, dtype, n, d, ld, S, omega, iters, epsilon, init_idx_h, centroids, primary,
                           shard_offsets_h, member_ids);
        SG_REQUIRE(tau0 >= 1.0f, "tau0 must be >= 1 (and not NaN)");
        SG_REQUIRE(block_rows >= 1, "block_rows must be >= 1");
        SG_REQUIRE(shard_cap >= 0, "shard_cap must be >= 0 (0: no limit)");
        SG_REQUIRE(adaptive == 0 || adaptive == 1, "adaptive must be 0 or 1");
        part::Layout L = part::layout(n, d, S, omega);
        const size_t need = L.total + part::blockwise_extra(n, S, block_rows);
        if (ws == nullptr || ws_bytes < need) {
            set_error("sg_partition_blockwise: workspace too small (need " + std::to_string(need) + " bytes)");
            throw Fail{SG_ERR_WORKSPACE};
        }
        hipStream_t s = as_stream(stream);
        Carver cv(ws);
        const part::Bufs B = part::carve(cv, L, n, d, S, omega);
        const int64_t nblocks = (n + block_rows - 1) / block_rows;
        float* D2 = cv.take<float>((size_t)n * S);
        float* et2_d = cv.take<float>((size_t)nblocks);
        part::run_kmeans(X, dtype, n, d, ld, S, iters, init_idx_h, centroids, L, B, s);
        const unsigned rg = (unsigned)cdiv(n, part::AR);
        SG_BY_SMAX(sqdist_kernel, X, dtype, n, d, ld, B.Cf, S, D2);
        // eps^2 and eps^2 tau_t^2 per block, in FP32 on the host:
        // tau_t = 1 + (tau0 - 1) / t for block t = 1, 2, ...
        const int accept_all = std::isinf(epsilon) && epsilon > 0;
        const float eps2 = accept_all ? 0.f : epsilon * epsilon;
        std::vector<float> et2((size_t)nblocks);
        for (int64_t t = 1; t <= nblocks; ++t) {
            const float tau_t = 1.0f + (tau0 - 1.0f) / (float)t;
            et2[(size_t)t - 1] = eps2 * (tau_t * tau_t);
        }
        SG_HIP(hipMemcpyAsync(et2_d, et2.data(), (size_t)nblocks * sizeof(float), hipMemcpyHostToDevice, s));
        switch (part::smax_of(S)) {
#define SG_BW(SM)                                                                                              \
            case SM:                                                                                           \
                part::blockwise_kernel<SM><<<1, 64, 0, s>>>(D2, n, S, omega, eps2, et2_d, block_rows, shard_cap, \
                                                            adaptive, accept_all, B.assign, primary);          \
                break;
            SG_BW(8) SG_BW(16) SG_BW(32) SG_BW(64)
#undef SG_BW
        }
        SG_LAUNCH_CHECK();
        part::run_membership(n, S, omega, capacity, member_ids, shard_offsets_h, L, B, s);
    });
}

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
        SG_REQUIRE(n >= 1 && n < (1ll << 31), "n out of range");
        SG_REQUIRE(d >= 1 && d <= 4096, "d must be in 1..4096");
        SG_REQUIRE(ld >= d, "ld must be >= d");
        SG_REQUIRE(S >= 1 && S <= part::MAX_S, "S must be in 1..64");
        SG_REQUIRE(omega >= 1 && omega <= S && omega <= part::MAX_OMEGA, "omega must be in 1..min(S, 8)");
        SG_REQUIRE(iters >= 0, "iters must be >= 0");
        SG_REQUIRE(dtype >= SG_F32 && dtype <= SG_U8, "unknown dtype");
        SG_REQUIRE(!(epsilon != epsilon) && !(tau != tau), "epsilon and tau must not be NaN");
        SG_REQUIRE(X && init_idx_h && centroids && primary && shard_offsets_h && member_ids,
                   "NULL pointer");
        for (int c = 0; c < S; ++c)
            SG_REQUIRE(init_idx_h[c] >= 0 && init_idx_h[c] < n, "init_idx out of range");
        part::Layout L = part::layout(n, d, S, omega);
        if (ws == nullptr || ws_bytes < L.total) {
            set_error("sg_partition: workspace too small (need " + std::to_string(L.total) + " bytes)");
            throw Fail{SG_ERR_WORKSPACE};
        }
        hipStream_t s = as_stream(stream);
        Carver cv(ws);
        float* Cf = cv.take<float>((size_t)S * d);
        int32_t* label = cv.take<int32_t>(n);
        double* partial = cv.take<double>((size_t)L.nb_sum * S * d);
        int64_t* pcount = cv.take<int64_t>((size_t)L.nb_sum * S);
        unsigned int* rbits = cv.take<unsigned int>(S);
        int32_t* assign = cv.take<int32_t>((size_t)n * omega);
        const int64_t ncm = (int64_t)S * L.nb_mem;
        int64_t* cm = cv.take<int64_t>(ncm + 1);
        int64_t* cmoff = cv.take<int64_t>(ncm + 1);
        void* scan_tmp = cv.take<char>(exclusive_scan_tmp_bytes(ncm));
        int64_t* init_d = cv.take<int64_t>(S);

        SG_HIP(hipMemcpyAsync(init_d, init_idx_h, S * sizeof(int64_t), hipMemcpyHostToDevice, s));
        part::init_centroids<<<cdiv((int64_t)S * d, 256), 256, 0, s>>>(X, dtype, ld, d, S, init_d, centroids);
        SG_LAUNCH_CHECK();
        const unsigned rg = (unsigned)cdiv(n, part::AR);
        const unsigned cg = (unsigned)cdiv((int64_t)S * d, 256);
        const int smax = S <= 8 ? 8 : S <= 16 ? 16 : S <= 32 ? 32 : 64;
#define SG_BY_SMAX(KERNEL, ...)                                                        \
        do {                                                                           \
            switch (smax) {                                                            \
                case 8: part::KERNEL<8><<<rg, part::AR, 0, s>>>(__VA_ARGS__); break;   \
                case 16: part::KERNEL<16><<<rg, part::AR, 0, s>>>(__VA_ARGS__); break; \
                case 32: part::KERNEL<32><<<rg, part::AR, 0, s>>>(__VA_ARGS__); break; \
                default: part::KERNEL<64><<<rg, part::AR, 0, s>>>(__VA_ARGS__); break; \
            }                                                                          \
            SG_LAUNCH_CHECK();                                                         \
        } while (0)
        for (int it = 0; it < iters; ++it) {
            part::to_f32<<<cg, 256, 0, s>>>(centroids, Cf, S * d);
            SG_BY_SMAX(assign_kernel, X, dtype, n, d, ld, Cf, S, label);
            dim3 sgrid((unsigned)L.nb_sum, (unsigned)cdiv(d, part::DSLICE));
            part::sum_kernel<<<sgrid, part::DSLICE, 0, s>>>(X, dtype, n, d, ld, label, S, partial, pcount);
            part::finalize_kernel<<<cg, 256, 0, s>>>(partial, pcount, L.nb_sum, S, d, centroids);
            SG_LAUNCH_CHECK();
        }
        part::to_f32<<<cg, 256, 0, s>>>(centroids, Cf, S * d);
        SG_BY_SMAX(assign_kernel, X, dtype, n, d, ld, Cf, S, label);
        fill<unsigned int>(rbits, 0u, S, s);
        SG_BY_SMAX(radius_kernel, X, dtype, n, d, ld, Cf, S, label, rbits);
        const int accept_all = std::isinf(epsilon) && epsilon > 0;
        SG_BY_SMAX(replica_kernel, X, dtype, n, d, ld, Cf, S, label, rbits, omega, epsilon, tau, accept_all,
                   assign);
#undef SG_BY_SMAX
        part::member_count_kernel<<<(unsigned)L.nb_mem, part::MEM_BLOCK, 0, s>>>(assign, n, omega, S,
                                                                                 L.nb_mem, cm);
        SG_LAUNCH_CHECK();
        exclusive_scan_i64(cm, cmoff, ncm, scan_tmp, s);
        part::member_write_kernel<<<(unsigned)L.nb_mem, part::MEM_BLOCK, 0, s>>>(
            assign, n, omega, S, L.nb_mem, cmoff, capacity, member_ids);
        SG_LAUNCH_CHECK();
        SG_HIP(hipMemcpyAsync(primary, label, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        // shard offsets: the scanned count matrix at each shard's first block
        std::vector<int64_t> all((size_t)ncm + 1);
        SG_HIP(hipMemcpyAsync(all.data(), cmoff, (ncm + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        SG_HIP(hipStreamSynchronize(s));
        for (int c = 0; c < S; ++c) shard_offsets_h[c] = all[(size_t)c * L.nb_mem];
        shard_offsets_h[S] = all[(size_t)ncm];
        if (shard_offsets_h[S] > capacity) {
            set_error("sg_partition: membership (" + std::to_string(shard_offsets_h[S]) +
                      ") exceeds capacity");
            throw Fail{SG_ERR_ARG};
        }
    });
}

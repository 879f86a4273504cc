// common.hpp -- internal helpers of the shard-graph library (gfx950 only).
//
// Error reporting for the C ABI, argument-check macros, the (distance, id)
// 64-bit ordering key, and wave64 primitives shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/sg.h"

namespace sg {

// ---------------------------------------------------------------------------
// error state (one text per calling thread)
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
const char* get_error();

struct Fail {
    sg_status code;
};

#define SG_REQUIRE(cond, msg)                                                    \
    do {                                                                         \
        if (!(cond)) {                                                           \
            ::sg::set_error(std::string(__func__) + ": " + (msg));              \
            throw ::sg::Fail{SG_ERR_ARG};                                        \
        }                                                                        \
    } while (0)

#define SG_HIP(call)                                                             \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess) {                                                  \
            ::sg::set_error(std::string(__func__) + ": " #call " -> " +        \
                            hipGetErrorString(e_));                              \
            throw ::sg::Fail{SG_ERR_HIP};                                        \
        }                                                                        \
    } while (0)

#define SG_LAUNCH_CHECK() SG_HIP(hipGetLastError())

// Runs `body` and maps exceptions to a status (no exception crosses the ABI).
template <class F>
sg_status guarded(F&& body) {
    try {
        body();
        return SG_OK;
    } catch (const Fail& f) {
        return f.code;
    } catch (const std::exception& e) {
        set_error(std::string("internal: ") + e.what());
        return SG_ERR_INTERNAL;
    } catch (...) {
        set_error("internal: unknown exception");
        return SG_ERR_INTERNAL;
    }
}

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Carves aligned sub-buffers out of a caller workspace.
struct Carver {
    char* base;
    size_t used = 0;
    explicit Carver(void* b) : base(static_cast<char*>(b)) {}
    template <class T>
    T* take(size_t count) {
        used = align_up(used, 256);
        T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
        used += count * sizeof(T);
        return p;
    }
};

// ---------------------------------------------------------------------------
// (distance, id) ordering key: the float is mapped to an unsigned integer
// with the same order, placed above the id, so that comparing keys compares
// (distance, id) lexicographically.  ~0 marks an empty slot.
// ---------------------------------------------------------------------------
constexpr uint64_t EMPTY_KEY = ~0ull;

__host__ __device__ inline uint32_t f2ord(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    uint32_t mask = (uint32_t)((int32_t)u >> 31) | 0x80000000u;
    return u ^ mask;
}

__host__ __device__ inline float ord2f(uint32_t o) {
    uint32_t u = (o & 0x80000000u) ? (o ^ 0x80000000u) : ~o;
    return __builtin_bit_cast(float, u);
}

__host__ __device__ inline uint64_t make_key(float dist, int32_t id) {
    return ((uint64_t)f2ord(dist) << 32) | (uint32_t)id;
}

__host__ __device__ inline int32_t key_id(uint64_t k) {
    return k == EMPTY_KEY ? SG_NONE : (int32_t)(uint32_t)k;
}

__host__ __device__ inline float key_dist(uint64_t k) {
    return k == EMPTY_KEY ? __builtin_inff() : ord2f((uint32_t)(k >> 32));
}

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------
__device__ inline int lane_id() { return __lane_id(); }

__device__ inline uint64_t shfl_u64(uint64_t v, int src) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    lo = __shfl((int)lo, src, 64);
    hi = __shfl((int)hi, src, 64);
    return ((uint64_t)hi << 32) | lo;
}

// The value that lane (l ^ j) holds, j in {1, 2, 4, 8, 16, 32}, without LDS
// traffic: DPP quad/row permutes inside 16-lane rows (row_shl:4 / row_shr:4 on
// alternate groups of four lanes for j = 4, a rotate by 8 for j = 8) and the
// permlane swaps across rows (j = 16) and wave halves (j = 32).  Each swap
// returns the even-row (even-half) values in element 0 and the odd ones in
// element 1 in every lane.  j must be a compile-time constant after unrolling.
__device__ inline uint32_t lane_xor(uint32_t v, int j) {
    const int x = (int)v;
    switch (j) {
    case 1: return (uint32_t)__builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false);
    case 2: return (uint32_t)__builtin_amdgcn_update_dpp(x, x, 0x4E, 0xF, 0xF, false);
    case 4: {
        const int t = __builtin_amdgcn_update_dpp(x, x, 0x104, 0xF, 0x5, false);
        return (uint32_t)__builtin_amdgcn_update_dpp(t, x, 0x114, 0xF, 0xA, false);
    }
    case 8: return (uint32_t)__builtin_amdgcn_update_dpp(x, x, 0x128, 0xF, 0xF, false);
    case 16: {
        const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (__lane_id() & 16) ? p[0] : p[1];
    }
    default: {
        const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (__lane_id() & 32) ? p[0] : p[1];
    }
    }
}

__device__ inline uint64_t lane_xor_u64(uint64_t v, int j) {
    const uint32_t lo = lane_xor((uint32_t)v, j), hi = lane_xor((uint32_t)(v >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}

// Lanes 32..63 receive the value of lane l - 32 (lanes 0..31 keep theirs).
__device__ inline uint64_t low_half_to_high(uint64_t v) {
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)v, (uint32_t)v, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(v >> 32), (uint32_t)(v >> 32), false, false);
    return ((uint64_t)hi[0] << 32) | lo[0];
}

// Compare-exchange with lane l ^ j: the smaller key where take_min, else the larger.
__device__ inline uint64_t cmpx(uint64_t x, int j, bool take_min) {
    const uint64_t o = lane_xor_u64(x, j);
    return (o < x) == take_min ? o : x;
}

__device__ inline uint64_t readlane_u64(uint64_t v, int lane) {
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// Ascending bitonic sort of one 64-bit key per lane across the wave.
__device__ inline uint64_t wave_sort_u64(uint64_t x) {
    const int l = lane_id();
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) x = cmpx(x, j, ((l & k) == 0) == ((l & j) == 0));
    }
    return x;
}

// Ascending bitonic sort of one 32-bit key per lane across the wave.
__device__ inline uint32_t wave_sort_u32(uint32_t x) {
    const int l = lane_id();
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint32_t o = lane_xor(x, j);
            x = (o < x) == (((l & k) == 0) == ((l & j) == 0)) ? o : x;
        }
    }
    return x;
}

// Each 32-lane half sorted on its own: lanes 0..31 descending, 32..63 ascending.
__device__ inline uint64_t half_sort_desc_u64(uint64_t x) {
    const int l = lane_id();
#pragma unroll
    for (int k = 2; k <= 32; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) x = cmpx(x, j, ((l & k) != 0) == ((l & j) == 0));
    }
    return x;
}

// Number of elements of the ascending array a[0..len) that are < v.
__device__ inline int lower_bound_u64(const uint64_t* a, int len, uint64_t v) {
    int lo = 0, hi = len;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Largest row count one call takes: kernels that give every row a wavefront
// launch 64 work-items per row, and a dispatch holds fewer than 2^32
// work-items per dimension.
constexpr int64_t MAX_ROWS = (int64_t(1) << 26) - 1024;

// Workgroups are dispatched to the 8 XCDs of the chip round robin (block b
// on XCD b % 8), each XCD with its own L2.  This bijection of [0, G) hands
// each XCD one contiguous range of block indices, so that blocks working on
// neighbouring data share an L2 (any bijection gives the same results).
constexpr int NUM_XCD = 8;
__device__ inline int64_t xcd_contiguous(int64_t b, int64_t G) {
    const int64_t q = G / NUM_XCD, r = G % NUM_XCD;
    const int64_t x = b % NUM_XCD, i = b / NUM_XCD;
    return x * q + (x < r ? x : r) + i;
}

// Grid-stride fill (used instead of hipMemsetAsync so that every clear is a
// kernel and stays valid inside captured graphs).
template <class T>
__global__ void fill_kernel(T* __restrict__ p, T v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <class T>
void fill(T* p, T v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    fill_kernel<T><<<blocks, 256, 0, s>>>(p, v, n);
    SG_LAUNCH_CHECK();
}

// Event pair around a distance-kernel launch while sg_profile_begin is active.
void profile_record(hipStream_t s, bool before);

__global__ inline void iota_kernel(int64_t* __restrict__ p, int64_t start, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = start + i;
}

inline void fill_iota(int64_t* p, int64_t start, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    iota_kernel<<<(unsigned)std::min<int64_t>((n + 255) / 256, 4096), 256, 0, s>>>(p, start, n);
    SG_LAUNCH_CHECK();
}

// Exclusive scan of int64 counts (n entries) into out (n+1 entries).
void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, void* tmp, hipStream_t s);
size_t exclusive_scan_tmp_bytes(int64_t n);

// Stable sort of rows 0..n-1 by label (labels in [0, 2^bits)): rows_out[p] is
// the row at position p of the (label, row) order.  Deterministic, no atomics
// in the placement, no memset (valid inside a captured graph).
void label_sort(const int32_t* lab, int64_t n, int bits, int32_t* rows_out, void* tmp, hipStream_t s);
size_t label_sort_tmp_bytes(int64_t n, int bits);
inline int bits_for(int64_t count) {
    int b = 0;
    while ((int64_t(1) << b) < count) ++b;
    return b;
}

}  // namespace sg

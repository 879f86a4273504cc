// knn.hip -- exact (and reduced-precision) kNN graph of one shard.
//
// The shard build of Sec. IV step 2 as a tiled all-pairs distance contraction
// (the dense-product formulation named in Sec. II-A) fused with a per-row
// top-k selection, for gfx950:
//
//  * prep: rows -> MFMA operand rows (FP32 / FP16 / BF16 / FP8 with a
//    power-of-two per-row scale), zero-padded to the k granule, plus the
//    squared norms of the operand rows (+inf for padding rows).
//  * dist_topk: a 512-thread workgroup (8 waves, two per SIMD so that one
//    wave's selection overlaps the other's MFMAs) owns 256 query rows, 32
//    per wave, and streams every candidate row of the shard through LDS in
//    double-buffered tiles (the next tile is already loading into registers
//    while the current one is computed).  Each 32x32 MFMA output tile holds
//    candidates on its rows and queries on its columns, so every lane sees
//    16 candidates of ONE query and keeps that query's admission threshold in
//    a register.  The accumulator starts at ||c||^2 and the query operand is
//    pre-scaled by -2 (exact), so the MFMA result is already the ranking key
//    ||c||^2 - 2 q.c (L2) or -q.c (IP).  Keys below the threshold go to a
//    32-entry LDS buffer per query; a buffer that overflows is merged in
//    registers (wave bitonic sort + bitonic merge) into the query's sorted
//    top-K list kept in the workspace, which lowers the threshold, and the
//    overflowing keys are re-admitted against it.  Candidates are visited in
//    ascending id order, so a key equal to the threshold can never enter the
//    list and the strict comparison is exact.
//  * rerank: the top-c candidates of a reduced-precision key re-scored with
//    the exact FP32 difference-form distance, best k kept.
#include <algorithm>

#include "common.hpp"

namespace sg {
namespace knn {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int intx8 __attribute__((ext_vector_type(8)));
typedef int intx4 __attribute__((ext_vector_type(4)));

constexpr int TWAVES = 8;        // waves per workgroup of the distance kernel
constexpr int TQB = 1;           // 32-query blocks per wave
constexpr int BQ = 32 * TQB * TWAVES;   // query rows per workgroup
constexpr int CB = 32;           // per-query candidate buffer
constexpr int PAD_ROWS = BQ;     // operand rows are padded to a multiple of this (>= any tile)

// ---------------------------------------------------------------------------
// operand traits: element bytes, elements per lane per MFMA step
// ---------------------------------------------------------------------------
template <int P> struct Tr;
template <> struct Tr<SG_PREC_FP32> { static constexpr int EB = 4, VEC = 1; };
template <> struct Tr<SG_PREC_F16> { static constexpr int EB = 2, VEC = 8; };
template <> struct Tr<SG_PREC_BF16> { static constexpr int EB = 2, VEC = 8; };
template <> struct Tr<SG_PREC_FP8> { static constexpr int EB = 1, VEC = 32; };

// padded row length (elements) for a given d: two lane-halves, each a whole
// number of MFMA steps
__host__ __device__ inline int padded_d(int prec, int d) {
    int g = 2 * (prec == SG_PREC_FP32 ? 2 : prec == SG_PREC_FP8 ? 32 : 8);
    return (d + g - 1) / g * g;
}
__host__ __device__ inline int elem_bytes(int prec) {
    return prec == SG_PREC_FP32 ? 4 : prec == SG_PREC_FP8 ? 1 : 2;
}

// ---------------------------------------------------------------------------
// prep: conversion, norms, FP8 scales
// ---------------------------------------------------------------------------
__device__ inline float load_elem(const void* X, int dtype, int64_t idx) {
    switch (dtype) {
        case SG_F32: return static_cast<const float*>(X)[idx];
        case SG_F16: return (float)static_cast<const _Float16*>(X)[idx];
        case SG_BF16: {
            uint32_t b = (uint32_t) static_cast<const uint16_t*>(X)[idx] << 16;
            return __builtin_bit_cast(float, b);
        }
        default: return (float)static_cast<const uint8_t*>(X)[idx];
    }
}

// FP32 -> BF16 bits, round to nearest even (NaN kept quiet)
__device__ inline uint16_t to_bf16_bits(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// FP32 -> OCP E4M3 code, round to nearest even, saturating at 448.  Works on
// the bit pattern: normal codes carry 3 mantissa bits, subnormals are
// multiples of 2^-9.
__device__ inline uint8_t to_fp8_bits(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    uint8_t sign = (uint8_t)((u >> 24) & 0x80);
    uint32_t a = u & 0x7fffffffu;
    if (a > 0x7f800000u) return 0x7f;                       // NaN
    if (a >= 0x43e00000u) return sign | 0x7e;               // |f| >= 448
    int e = (int)(a >> 23) - 127;                           // unbiased exponent
    if (e < -6) {
        // subnormal range: value / 2^-9 rounded to an integer 0..8
        float v = __builtin_bit_cast(float, a) * 512.0f;    // exact (power of two)
        float r = __builtin_rintf(v);                       // ties to even
        return sign | (uint8_t)r;
    }
    uint32_t mant = a & 0x7fffffu;                          // 23 bits, keep 3
    uint32_t keep = mant >> 20;
    uint32_t rest = mant & 0xfffffu;
    if (rest > 0x80000u || (rest == 0x80000u && (keep & 1u))) keep += 1;
    int ex = e + 7;
    if (keep == 8) {
        keep = 0;
        ex += 1;
    }
    uint32_t code = ((uint32_t)ex << 3) | keep;
    if (code > 0x7e) code = 0x7e;
    return sign | (uint8_t)code;
}

__device__ inline float fp8_value(uint8_t c) {
    int e = (c >> 3) & 15, m = c & 7;
    float v = e == 0 ? (float)m * (1.0f / 512.0f)
                     : __builtin_ldexpf(1.0f + (float)m * 0.125f, e - 7);
    return (c & 0x80) ? -v : v;
}

// Ranking-key form per (metric, precision):
//   L2             key = ||c~||^2 - 2 q~.c~            dist = key + ||q~||^2
//   IP, FP32/F16   key = -q.c                           dist = key
//   IP, BF16/FP8   key = ||c~||^2 - ||c||^2 - 2 q~.c~   dist = (key + ||q~||^2 - ||q||^2) / 2
// (x~ = the rounded operand row).  The reduced-precision IP key is the L2 key
// of the rounded rows with the exact norm put back: its rounding error scales
// with ||q - c|| instead of ||q|| ||c||, which keeps near neighbours apart.
__host__ __device__ inline bool norm_corrected_ip(int metric, int prec) {
    return metric == SG_IP && (prec == SG_PREC_BF16 || prec == SG_PREC_FP8);
}

// One wave per operand row (source row rowmap[row], or row itself when
// rowmap is NULL).  Writes the converted row (zero padded to DP),
// the accumulator start of the row as a candidate (ninit, +inf for padding
// rows), its output offset as a query (nout) and, for FP8, the row's scale
// exponent.
__global__ void prep_kernel(const void* __restrict__ X, int dtype, int64_t n, int d, int64_t ld,
                            const int64_t* __restrict__ rowmap, int64_t n_src, int64_t n_pad, int DP,
                            int prec, int metric, uint8_t* __restrict__ ops, float* __restrict__ ninit,
                            float* __restrict__ nout, int32_t* __restrict__ sexp) {
    const int l = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= n_pad) return;
    const int eb = elem_bytes(prec);
    uint8_t* out = ops + row * (int64_t)DP * eb;
    const int64_t src_row = row < n ? (rowmap ? rowmap[row] : row) : -1;
    if (src_row < 0 || src_row >= n_src) {      // padding (or an out-of-range listed row)
        for (int t = l; t < DP; t += 64) {
            if (eb == 4) reinterpret_cast<float*>(out)[t] = 0.f;
            else if (eb == 2) reinterpret_cast<uint16_t*>(out)[t] = 0;
            else out[t] = 0;
        }
        if (l == 0) {
            ninit[row] = __builtin_inff();
            nout[row] = 0.f;
            if (sexp) sexp[row] = 0;
        }
        return;
    }
    const int64_t base = src_row * ld;
    int sx = 0;
    float inv = 1.0f;
    if (prec == SG_PREC_FP8) {
        float amax = 0.f;
        for (int t = l; t < d; t += 64) amax = fmaxf(amax, fabsf(load_elem(X, dtype, base + t)));
        for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
        // smallest power of two s with amax / s <= 448
        if (amax > 0.f) {
            sx = (int)ceilf(log2f(amax / 448.0f));
            while (__builtin_ldexpf(amax, -sx) > 448.0f) ++sx;
            while (sx > -126 && __builtin_ldexpf(amax, -(sx - 1)) <= 448.0f) --sx;
        }
        inv = __builtin_ldexpf(1.0f, -sx);
    }
    float ssq = 0.f, ssx = 0.f;
    for (int t = l; t < DP; t += 64) {
        float v = t < d ? load_elem(X, dtype, base + t) : 0.f;
        float q;
        switch (prec) {
            case SG_PREC_FP32:
                reinterpret_cast<float*>(out)[t] = v;
                q = v;
                break;
            case SG_PREC_F16: {
                _Float16 h = (_Float16)v;
                reinterpret_cast<_Float16*>(out)[t] = h;
                q = (float)h;
                break;
            }
            case SG_PREC_BF16: {
                uint16_t b = to_bf16_bits(v);
                reinterpret_cast<uint16_t*>(out)[t] = b;
                q = __builtin_bit_cast(float, (uint32_t)b << 16);
                break;
            }
            default: {
                uint8_t c = to_fp8_bits(v * inv);
                out[t] = c;
                q = __builtin_ldexpf(fp8_value(c), sx);
                break;
            }
        }
        ssq += q * q;
        ssx += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) {
        ssq += __shfl_xor(ssq, o, 64);
        ssx += __shfl_xor(ssx, o, 64);
    }
    if (l == 0) {
        if (metric == SG_L2) {
            ninit[row] = ssq;
            nout[row] = ssq;
        } else if (norm_corrected_ip(metric, prec)) {
            ninit[row] = ssq - ssx;
            nout[row] = ssq - ssx;
        } else {
            ninit[row] = 0.f;
            nout[row] = 0.f;
        }
        if (sexp) sexp[row] = sx;
    }
}

// ---------------------------------------------------------------------------
// fused distance tile + top-k
// ---------------------------------------------------------------------------

// row of the 32x32 MFMA output held by accumulator register i of lane l
__device__ inline int out_row(int i, int l) { return ((i >> 2) << 3) + ((l >> 5) << 2) + (i & 3); }

template <int P, int NSTEP>
struct Frag;

template <int NSTEP>
struct Frag<SG_PREC_FP32, NSTEP> {
    float v[NSTEP];
};
template <int NSTEP>
struct Frag<SG_PREC_F16, NSTEP> {
    half8 v[NSTEP];
};
template <int NSTEP>
struct Frag<SG_PREC_BF16, NSTEP> {
    bf16x8 v[NSTEP];
};
template <int NSTEP>
struct Frag<SG_PREC_FP8, NSTEP> {
    intx8 v[NSTEP];
};

// Load lane l's half-row (elements [h*DH, (h+1)*DH)) from a byte row.
template <int P, int NSTEP>
__device__ inline void load_frag(Frag<P, NSTEP>& f, const uint8_t* rowp) {
    if constexpr (P == SG_PREC_FP32) {
#pragma unroll
        for (int s = 0; s < NSTEP; s += 2) {
            float2 v = *reinterpret_cast<const float2*>(rowp + s * 4);
            f.v[s] = v.x;
            f.v[s + 1] = v.y;
        }
    } else if constexpr (P == SG_PREC_FP8) {
#pragma unroll
        for (int s = 0; s < NSTEP; ++s) {
            intx4 a = *reinterpret_cast<const intx4*>(rowp + s * 32);
            intx4 b = *reinterpret_cast<const intx4*>(rowp + s * 32 + 16);
            f.v[s] = intx8{a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
        }
    } else {
#pragma unroll
        for (int s = 0; s < NSTEP; ++s) {
            intx4 a = *reinterpret_cast<const intx4*>(rowp + s * 16);
            if constexpr (P == SG_PREC_F16)
                f.v[s] = __builtin_bit_cast(half8, a);
            else
                f.v[s] = __builtin_bit_cast(bf16x8, a);
        }
    }
}

// Scale the query fragment by qmul (-2 or -1, exact) so that the MFMA yields
// the ranking key.  FP8 (always the -2 form) flips the code signs and carries
// the x2 in the scale exponent.
template <int P, int NSTEP>
__device__ inline void scale_query(Frag<P, NSTEP>& f, float qmul) {
    if constexpr (P == SG_PREC_FP8) {
#pragma unroll
        for (int s = 0; s < NSTEP; ++s)
#pragma unroll
            for (int e = 0; e < 8; ++e) f.v[s][e] ^= (int)0x80808080u;
    } else {
        const float m = qmul;
#pragma unroll
        for (int s = 0; s < NSTEP; ++s) {
            if constexpr (P == SG_PREC_FP32) {
                f.v[s] *= m;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    if constexpr (P == SG_PREC_F16)
                        f.v[s][e] = (_Float16)((float)f.v[s][e] * m);
                    else
                        f.v[s][e] = (__bf16)((float)f.v[s][e] * m);
                }
            }
        }
    }
}

template <int P>
__device__ inline floatx16 mfma_step(const void* a, const void* b, floatx16 acc, int sa, int sb);

template <int P, int NSTEP>
__device__ inline floatx16 mfma_tile(const uint8_t* arow, const Frag<P, NSTEP>& q, floatx16 acc,
                                     int sa, int sb) {
    if constexpr (P == SG_PREC_FP32) {
#pragma unroll
        for (int s = 0; s < NSTEP; s += 4) {
            floatx4 a = *reinterpret_cast<const floatx4*>(arow + s * 4);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0], q.v[s], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1], q.v[s + 1], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[2], q.v[s + 2], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[3], q.v[s + 3], acc, 0, 0, 0);
        }
    } else if constexpr (P == SG_PREC_F16) {
#pragma unroll
        for (int s = 0; s < NSTEP; ++s) {
            half8 a = *reinterpret_cast<const half8*>(arow + s * 16);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, q.v[s], acc, 0, 0, 0);
        }
    } else if constexpr (P == SG_PREC_BF16) {
#pragma unroll
        for (int s = 0; s < NSTEP; ++s) {
            bf16x8 a = *reinterpret_cast<const bf16x8*>(arow + s * 16);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, q.v[s], acc, 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int s = 0; s < NSTEP; ++s) {
            intx4 lo = *reinterpret_cast<const intx4*>(arow + s * 32);
            intx4 hi = *reinterpret_cast<const intx4*>(arow + s * 32 + 16);
            intx8 a = intx8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
            acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, q.v[s], acc, 0, 0, 0, sa, 0,
                                                                   sb);
        }
    }
    return acc;
}

template <int P, int NSTEP>
struct Shape {
    static constexpr int DH = NSTEP * Tr<P>::VEC;             // elements per lane-half
    static constexpr int ROW_BYTES = 2 * DH * Tr<P>::EB;      // padded operand row
    static constexpr int RS = ROW_BYTES + 16;                 // LDS row stride (bank spread)
    // candidate rows per LDS tile: two tiles (double buffer) stay within ~70 KB
    static constexpr int BC = ROW_BYTES <= 256 ? 128 : ROW_BYTES <= 512 ? 64 : 32;
    static constexpr int NSUB = BC / 32;
};

// Bitonic merge (ascending) of 64*PER keys held as v[p] (element p*64 + lane)
// that already form a bitonic sequence.
template <int PER>
__device__ inline void bitonic_merge_multi(uint64_t (&v)[PER]) {
    const int l = lane_id();
#pragma unroll
    for (int j = 32 * PER; j > 0; j >>= 1) {
        if (j >= 64) {
            const int jp = j >> 6;
#pragma unroll
            for (int p = 0; p < PER; ++p) {
                const int q = p ^ jp;
                if (q > p) {
                    uint64_t a = v[p], b = v[q];
                    v[p] = a < b ? a : b;
                    v[q] = a < b ? b : a;
                }
            }
        } else {
#pragma unroll
            for (int p = 0; p < PER; ++p) {
                uint64_t o = shfl_xor_u64(v[p], j);
                bool lower = (l & j) == 0;
                uint64_t mn = v[p] < o ? v[p] : o, mx = v[p] < o ? o : v[p];
                v[p] = lower ? mn : mx;
            }
        }
    }
}

// Merge one query's candidate buffer (<= CB keys in LDS) into its sorted
// top-KSEL list in the workspace, all in registers: sort the buffer across the
// wave, take the element-wise minimum of the list and the reversed buffer
// (which holds the KSEL smallest of both as a bitonic sequence), bitonic-merge
// it.  Returns the new admission threshold: the KSEL-th distance (+inf while
// the list is not full).
template <int KSEL>
__device__ float merge_query(uint64_t* __restrict__ gstate, const uint64_t* buf, int c) {
    constexpr int PER = KSEL >= 64 ? KSEL / 64 : 1;
    const int l = lane_id();
    uint64_t b = l < c ? buf[l] : EMPTY_KEY;
    uint64_t v[PER];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int e = p * 64 + l;
        v[p] = e < KSEL ? gstate[e] : EMPTY_KEY;
    }
    b = wave_sort_u64(b);
    const uint64_t r = shfl_u64(b, 63 - l);
    v[PER - 1] = v[PER - 1] < r ? v[PER - 1] : r;
    bitonic_merge_multi<PER>(v);
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int e = p * 64 + l;
        if (e < KSEL) gstate[e] = v[p];
    }
    const uint64_t last = shfl_u64(v[(KSEL - 1) / 64], (KSEL - 1) & 63);
    return key_dist(last);
}

// Per-wave selection state: the admission threshold of each of the wave's
// 32*QB queries (lanes l and l+32 share query l%32 of each block), the id
// excluded as the query itself, and the LDS buffers / counters and workspace
// top-KSEL lists of those queries.
template <int KSEL, int QB>
struct Selector {
    float thr[QB];
    int64_t qself[QB];
    uint64_t* state;   // state row of the wave's first query
    uint64_t* buf;     // LDS buffers of the wave's queries (32*QB*CB keys)
    int* cnt;          // LDS counters of the wave's queries

    // Admit the candidates of one 32x32 subtile (rows cbase..cbase+31) that
    // beat the thresholds.  Each lane counts its hits, the two lanes of a
    // query exchange counts with one shuffle and read the buffer fill once;
    // a query whose new hits would not fit is merged first (which lowers its
    // threshold and empties its buffer) and its hits recounted; then every
    // lane writes its keys at slots known in advance -- no atomics.
    __device__ void admit(floatx16 (&acc)[QB], int64_t cbase) {
        const int l = lane_id();
        const int ql = l & 31;
        const int h = l >> 5;
#pragma unroll
        for (int b = 0; b < QB; ++b) {
            const bool mine = qself[b] >= cbase && qself[b] < cbase + 32;
            if (__builtin_amdgcn_ballot_w64(mine)) {
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    if (cbase + out_row(i, l) == qself[b]) acc[b][i] = __builtin_inff();
            }
        }
        bool any = false;
#pragma unroll
        for (int b = 0; b < QB; ++b)
#pragma unroll
            for (int i = 0; i < 16; ++i) any |= acc[b][i] < thr[b];
        if (!__builtin_amdgcn_ballot_w64(any)) return;
#pragma unroll
        for (int b = 0; b < QB; ++b) {
            const int qq = b * 32 + ql;
            int c = 0;
#pragma unroll
            for (int i = 0; i < 16; ++i) c += acc[b][i] < thr[b] ? 1 : 0;
            int cp = __shfl_xor(c, 32, 64);
            int base = cnt[qq];
            const uint64_t over = __builtin_amdgcn_ballot_w64(base + c + cp > CB);
            if (over) {
                uint32_t need = (uint32_t)over | (uint32_t)(over >> 32);
                while (need) {
                    const int qi = __builtin_ctz(need);
                    need &= need - 1;
                    const int q2 = b * 32 + qi;
                    const int fill = __builtin_amdgcn_readlane(base, qi);
                    const float t = merge_query<KSEL>(state + (int64_t)q2 * KSEL, buf + q2 * CB, fill);
                    if (ql == qi) {
                        thr[b] = t;
                        base = 0;
                    }
                }
                c = 0;
#pragma unroll
                for (int i = 0; i < 16; ++i) c += acc[b][i] < thr[b] ? 1 : 0;
                cp = __shfl_xor(c, 32, 64);
            }
            int slot = base + (h ? cp : 0);
            if (c) {
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    if (acc[b][i] < thr[b]) {
                        buf[qq * CB + slot] = make_key(acc[b][i], (int32_t)(cbase + out_row(i, l)));
                        ++slot;
                    }
                }
            }
            if (h == 0) cnt[qq] = base + c + cp;
        }
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    }

    // Merge every non-empty buffer (end of the candidate stream).
    __device__ void drain() {
        const int l = lane_id();
#pragma unroll
        for (int b = 0; b < QB; ++b) {
            const int qq = b * 32 + (l & 31);
            const uint64_t m = __builtin_amdgcn_ballot_w64(l < 32 && cnt[qq] > 0);
            uint32_t need = (uint32_t)m;
            while (need) {
                const int qi = __builtin_ctz(need);
                need &= need - 1;
                const int q2 = b * 32 + qi;
                merge_query<KSEL>(state + (int64_t)q2 * KSEL, buf + q2 * CB,
                                  __builtin_amdgcn_readfirstlane(cnt[q2]));
            }
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
};

// Final lists of the wave's queries: ids and output distances.
__device__ inline void write_lists(const uint64_t* __restrict__ state, int ksel, int64_t q0, int nqw,
                                   int64_t nq, const float* __restrict__ qnout, float osc,
                                   int32_t* __restrict__ nbr, float* __restrict__ dist, int k_out) {
    const int l = lane_id();
    for (int qi = 0; qi < nqw; ++qi) {
        const int64_t q = q0 + qi;
        if (q >= nq) break;
        const float qn = qnout[q];
        for (int t = l; t < k_out; t += 64) {
            const uint64_t key = state[q * ksel + t];
            nbr[q * k_out + t] = key_id(key);
            if (dist) dist[q * k_out + t] = key == EMPTY_KEY ? __builtin_inff() : (key_dist(key) + qn) * osc;
        }
    }
}

// LDS of the register-resident kernel.
template <int P, int NSTEP, int WAVES, int QB>
struct TopkSmem {
    using S = Shape<P, NSTEP>;
    static constexpr int NQ = 32 * QB * WAVES;
    __align__(16) uint8_t tile[2][S::BC * S::RS];
    __align__(16) float norm[2][S::BC];
    int32_t sexp[2][P == SG_PREC_FP8 ? S::BC : 1];
    uint64_t buf[NQ * CB];
    int cnt[NQ];
};

// One block of NQ = 32*QB*WAVES queries (query rows qb*NQ.. of qops) against
// all n candidate rows of ops: the fused distance tile + top-k with
// register-resident queries.  Candidate tiles (BC rows) are staged in LDS,
// double buffered, the next tile already in flight in registers while the
// current one is computed.  Within a tile the MFMAs of subtile s+1 are
// issued before the selection epilogue of subtile s so that both run at once.
template <int P, int NSTEP, int KSEL, int WAVES, int QB>
__device__ void topk_block(TopkSmem<P, NSTEP, WAVES, QB>& sm, int64_t qb, const uint8_t* __restrict__ ops,
                           const float* __restrict__ ninit, const int32_t* __restrict__ sexp, int n,
                           const uint8_t* __restrict__ qops, const int64_t* __restrict__ qid,
                           const float* __restrict__ qnout, const int32_t* __restrict__ qsexp, int nq,
                           float qmul, float osc, uint64_t* __restrict__ state, int32_t* __restrict__ nbr,
                           float* __restrict__ dist, int k_out) {
    using S = Shape<P, NSTEP>;
    constexpr int BC = S::BC, NSUB = S::NSUB, RB = S::ROW_BYTES, RS = S::RS;
    constexpr int NT = WAVES * 64;
    constexpr int NQ = 32 * QB * WAVES;
    constexpr int CHUNKS = BC * RB / 16;                        // 16-byte chunks per tile
    constexpr int CPT = (CHUNKS + NT - 1) / NT;                 // chunks per thread

    const int tid = threadIdx.x;
    const int l = tid & 63;
    const int w = tid >> 6;
    const int h = l >> 5;
    const int ql = l & 31;
    const int64_t qblk0 = qb * NQ + w * 32 * QB;   // first query of this wave

    for (int t = tid; t < NQ; t += NT) sm.cnt[t] = 0;

    Frag<P, NSTEP> qf[QB];
    int q_scale[QB];
    Selector<KSEL, QB> sel;
    sel.state = state + qblk0 * KSEL;
    sel.buf = sm.buf + w * 32 * QB * CB;
    sel.cnt = sm.cnt + w * 32 * QB;
#pragma unroll
    for (int b = 0; b < QB; ++b) {
        const int64_t qg = qblk0 + b * 32 + ql;
        load_frag<P, NSTEP>(qf[b], qops + qg * RB + h * (RB / 2));
        scale_query<P, NSTEP>(qf[b], qmul);
        q_scale[b] = 127;
        if constexpr (P == SG_PREC_FP8) q_scale[b] = 127 + qsexp[qg] + 1;
        sel.thr[b] = __builtin_inff();
        sel.qself[b] = qg < nq ? (qid ? qid[qg] : qg) : -1;
    }

    // tile staging: global -> registers (prefetch) -> LDS
    intx4 pre[CPT];
    float pre_norm = 0.f;
    int32_t pre_sexp = 0;
    auto prefetch = [&](int j0) {
        const uint8_t* src = ops + (int64_t)j0 * RB;
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int c = tid + u * NT;
            if (c < CHUNKS) pre[u] = *reinterpret_cast<const intx4*>(src + (int64_t)c * 16);
        }
        if (tid < BC) {
            pre_norm = ninit[j0 + tid];
            if constexpr (P == SG_PREC_FP8) pre_sexp = sexp[j0 + tid];
        }
    };
    auto commit = [&](int buf) {
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int c = tid + u * NT;
            if (c < CHUNKS) {
                const int r = c / (RB / 16), o = c % (RB / 16);
                *reinterpret_cast<intx4*>(&sm.tile[buf][r * RS + o * 16]) = pre[u];
            }
        }
        if (tid < BC) {
            sm.norm[buf][tid] = pre_norm;
            if constexpr (P == SG_PREC_FP8) sm.sexp[buf][tid] = pre_sexp;
        }
    };
    auto compute = [&](floatx16 (&acc)[QB], int buf, int sub) {
        floatx4 nv[4];
#pragma unroll
        for (int g = 0; g < 4; ++g)
            nv[g] = *reinterpret_cast<const floatx4*>(&sm.norm[buf][sub * 32 + g * 8 + h * 4]);
        int a_scale = 127;
        if constexpr (P == SG_PREC_FP8) a_scale = 127 + sm.sexp[buf][sub * 32 + ql];
        const uint8_t* arow = &sm.tile[buf][(sub * 32 + ql) * RS + h * (RB / 2)];
#pragma unroll
        for (int b = 0; b < QB; ++b) {
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[b][i] = nv[i >> 2][i & 3];
        }
#pragma unroll
        for (int b = 0; b < QB; ++b) acc[b] = mfma_tile<P, NSTEP>(arow, qf[b], acc[b], a_scale, q_scale[b]);
    };

    const int ntiles = (n + BC - 1) / BC;
    prefetch(0);
    commit(0);
    __syncthreads();
    if (ntiles > 1) prefetch(BC);
    for (int t = 0; t < ntiles; ++t) {
        const int buf = t & 1;
        const int j0 = t * BC;
        floatx16 accA[QB], accB[QB];
        compute(accA, buf, 0);
#pragma unroll
        for (int sub = 0; sub < NSUB; ++sub) {
            if (sub % 2 == 0) {
                if (sub + 1 < NSUB) compute(accB, buf, sub + 1);
                sel.admit(accA, j0 + sub * 32);
            } else {
                if (sub + 1 < NSUB) compute(accA, buf, sub + 1);
                sel.admit(accB, j0 + sub * 32);
            }
        }
        if (t + 1 < ntiles) {
            commit(buf ^ 1);
            if (t + 2 < ntiles) prefetch((t + 2) * BC);
        }
        __syncthreads();
    }
    sel.drain();
    if (nbr) write_lists(state, KSEL, qblk0, 32 * QB, nq, qnout, osc, nbr, dist, k_out);
    __syncthreads();   // LDS is reused by the next block of a persistent workgroup
}

// One query block per workgroup (blockIdx.x).
template <int P, int NSTEP, int KSEL, int WAVES, int QB>
__global__ __launch_bounds__(WAVES * 64, 1) void dist_topk_kernel(
    const uint8_t* __restrict__ ops, const float* __restrict__ ninit, const int32_t* __restrict__ sexp,
    int n, const uint8_t* __restrict__ qops, const int64_t* __restrict__ qid,
    const float* __restrict__ qnout, const int32_t* __restrict__ qsexp, int nq, float qmul, float osc,
    uint64_t* __restrict__ state, int32_t* __restrict__ nbr, float* __restrict__ dist, int k_out) {
    __shared__ TopkSmem<P, NSTEP, WAVES, QB> sm;
    topk_block<P, NSTEP, KSEL, WAVES, QB>(sm, blockIdx.x, ops, ninit, sexp, n, qops, qid, qnout, qsexp, nq, qmul,
                                          osc, state, nbr, dist, k_out);
}

// Many shards in one launch: a persistent grid pulls (shard, query block)
// items from a counter in the order of the work list (largest shards first)
// and runs each as above.  Shard s occupies operand / state rows
// [row0[s], row0[s] + ceil(n[s]/NQ)*NQ) and output rows [out0[s], out0[s] + n[s]);
// candidate ids are shard-local.  Every workgroup leaves once the counter
// passes the last item.
template <int P, int NSTEP, int KSEL, int WAVES, int QB>
__global__ __launch_bounds__(WAVES * 64, 1) void dist_topk_persistent_kernel(
    const uint8_t* __restrict__ ops, const float* __restrict__ ninit, const float* __restrict__ nout,
    const int32_t* __restrict__ sexp, const int64_t* __restrict__ row0, const int32_t* __restrict__ nrows,
    const int64_t* __restrict__ out0, const int32_t* __restrict__ items, int nitems,
    unsigned int* __restrict__ counter, float qmul, float osc, uint64_t* __restrict__ state,
    int32_t* __restrict__ nbr, float* __restrict__ dist, int k_out) {
    __shared__ TopkSmem<P, NSTEP, WAVES, QB> sm;
    __shared__ int s_item;
    using S = Shape<P, NSTEP>;
    constexpr int RB = S::ROW_BYTES;
    while (true) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= nitems) break;
        const int sh = items[2 * it], qb = items[2 * it + 1];
        const int64_t r0 = row0[sh];
        const int ns = nrows[sh];
        const uint8_t* o = ops + r0 * RB;
        topk_block<P, NSTEP, KSEL, WAVES, QB>(sm, qb, o, ninit + r0, sexp ? sexp + r0 : nullptr, ns, o, nullptr,
                                              nout + r0, sexp ? sexp + r0 : nullptr, ns, qmul, osc,
                                              state + r0 * KSEL, nbr + out0[sh] * k_out,
                                              dist ? dist + out0[sh] * k_out : nullptr, k_out);
    }
}

// Fused distance tile + top-k for FP32 rows too wide for register-resident
// queries: a 128 x 128 (queries x candidates) workgroup tile accumulated over
// k in chunks of 32, both operands staged through LDS (double buffered, the
// next chunk loading into registers during the current chunk's MFMAs); the
// selection runs on the four 32x32 subtiles of each wave once a candidate
// tile's k-loop is complete.
constexpr int KS_WAVES = 4;
constexpr int KS_NQ = 128;
constexpr int KS_BC = 128;
constexpr int KS_DC = 32;
constexpr int KS_RS = KS_DC + 4;    // LDS row stride (floats)

template <int KSEL>
__global__ __launch_bounds__(KS_WAVES * 64, 1) void dist_topk_kstream_kernel(
    const float* __restrict__ ops, int DP, const float* __restrict__ ninit, int n,
    const float* __restrict__ qops, const int64_t* __restrict__ qid, const float* __restrict__ qnout,
    int nq, float qmul, float osc, uint64_t* __restrict__ state, int32_t* __restrict__ nbr,
    float* __restrict__ dist, int k_out) {
    constexpr int NT = KS_WAVES * 64;
    constexpr int CPR = KS_DC / 4;                       // 16-byte chunks per row per k-chunk
    constexpr int CPT = (KS_NQ + KS_BC) * CPR / NT;      // per thread per k-chunk
    __shared__ __align__(16) float s_q[2][KS_NQ * KS_RS];
    __shared__ __align__(16) float s_c[2][KS_BC * KS_RS];
    __shared__ __align__(16) float s_norm[KS_BC];
    __shared__ uint64_t s_buf[KS_NQ * CB];
    __shared__ int s_cnt[KS_NQ];

    const int tid = threadIdx.x;
    const int l = tid & 63;
    const int w = tid >> 6;
    const int h = l >> 5;
    const int ql = l & 31;
    const int64_t qb0 = (int64_t)blockIdx.x * KS_NQ;
    const int64_t qblk0 = qb0 + w * 32;
    for (int t = tid; t < KS_NQ; t += NT) s_cnt[t] = 0;

    Selector<KSEL, 1> sel;
    sel.state = state + qblk0 * KSEL;
    sel.buf = s_buf + w * 32 * CB;
    sel.cnt = s_cnt + w * 32;
    {
        const int64_t qg = qblk0 + ql;
        sel.thr[0] = __builtin_inff();
        sel.qself[0] = qg < nq ? (qid ? qid[qg] : qg) : -1;
    }

    const int nch = DP / KS_DC;
    const int ntiles = (n + KS_BC - 1) / KS_BC;
    const int64_t total = (int64_t)ntiles * nch;
    intx4 pre[CPT];
    float pre_norm = 0.f;
    auto prefetch = [&](int64_t g) {
        const int t = (int)(g / nch), kc = (int)(g % nch);
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int c = tid + u * NT;
            const int r = c / CPR, o = c % CPR;
            const float* src = r < KS_NQ ? qops + (qb0 + r) * DP
                                         : ops + ((int64_t)t * KS_BC + (r - KS_NQ)) * DP;
            pre[u] = *reinterpret_cast<const intx4*>(src + kc * KS_DC + o * 4);
        }
        if (kc == 0 && tid < KS_BC) pre_norm = ninit[(int64_t)t * KS_BC + tid];
    };
    auto commit = [&](int64_t g, int buf) {
        const int kc = (int)(g % nch);
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int c = tid + u * NT;
            const int r = c / CPR, o = c % CPR;
            float* dst = r < KS_NQ ? &s_q[buf][r * KS_RS + o * 4] : &s_c[buf][(r - KS_NQ) * KS_RS + o * 4];
            *reinterpret_cast<intx4*>(dst) = pre[u];
        }
        if (kc == 0 && tid < KS_BC) s_norm[tid] = pre_norm;
    };

    prefetch(0);
    commit(0, 0);
    __syncthreads();
    if (total > 1) prefetch(1);
    floatx16 acc[4];
    for (int64_t g = 0; g < total; ++g) {
        const int buf = (int)(g & 1);
        const int t = (int)(g / nch), kc = (int)(g % nch);
        if (kc == 0) {
#pragma unroll
            for (int sub = 0; sub < 4; ++sub)
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[sub][i] = s_norm[sub * 32 + out_row(i, l)];
        }
        // B fragment: this lane's query, the lane half's 16 k values of the chunk
        float bq[KS_DC / 2];
#pragma unroll
        for (int v = 0; v < KS_DC / 8; ++v) {
            floatx4 x = *reinterpret_cast<const floatx4*>(&s_q[buf][(w * 32 + ql) * KS_RS + h * (KS_DC / 2) + v * 4]);
#pragma unroll
            for (int e = 0; e < 4; ++e) bq[v * 4 + e] = x[e] * qmul;
        }
#pragma unroll
        for (int sub = 0; sub < 4; ++sub) {
            const float* arow = &s_c[buf][(sub * 32 + ql) * KS_RS + h * (KS_DC / 2)];
#pragma unroll
            for (int v = 0; v < KS_DC / 8; ++v) {
                floatx4 a = *reinterpret_cast<const floatx4*>(arow + v * 4);
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    acc[sub] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[e], bq[v * 4 + e], acc[sub], 0, 0, 0);
            }
        }
        if (kc == nch - 1) {
#pragma unroll
            for (int sub = 0; sub < 4; ++sub) {
                floatx16 one[1] = {acc[sub]};
                sel.admit(one, (int64_t)t * KS_BC + sub * 32);
            }
        }
        if (g + 1 < total) {
            commit(g + 1, buf ^ 1);
            if (g + 2 < total) prefetch(g + 2);
        }
        __syncthreads();
    }
    sel.drain();
    if (nbr) write_lists(state, KSEL, qblk0, 32, nq, qnout, osc, nbr, dist, k_out);
}

// ---------------------------------------------------------------------------
// FP32 re-rank of the top-c candidates (difference form)
// ---------------------------------------------------------------------------

// Ascending bitonic sort of 64*PER keys held as v[p] in lane l (element p*64+l).
template <int PER>
__device__ inline void wave_sort_multi(uint64_t (&v)[PER]) {
    const int l = lane_id();
    constexpr int N = 64 * PER;
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 64) {
                const int jp = j >> 6;
#pragma unroll
                for (int p = 0; p < PER; ++p) {
                    int q = p ^ jp;
                    if (q > p) {
                        int e = p * 64 + l;
                        bool up = (e & k) == 0;
                        uint64_t a = v[p], b = v[q];
                        uint64_t mn = a < b ? a : b, mx = a < b ? b : a;
                        v[p] = up ? mn : mx;
                        v[q] = up ? mx : mn;
                    }
                }
            } else {
#pragma unroll
                for (int p = 0; p < PER; ++p) {
                    int e = p * 64 + l;
                    uint64_t o = shfl_xor_u64(v[p], j);
                    bool up = (e & k) == 0;
                    bool lower = (l & j) == 0;
                    uint64_t mn = v[p] < o ? v[p] : o, mx = v[p] < o ? o : v[p];
                    v[p] = (lower == up) ? mn : mx;
                }
            }
        }
    }
}

__device__ inline int32_t cand_id(uint64_t key) { return key_id(key); }
__device__ inline int32_t cand_id(int32_t id) { return id; }

template <int PER, typename CT = uint64_t>
__global__ __launch_bounds__(256) void rerank_kernel(const void* __restrict__ X, int dtype, int64_t n,
                                                     int d, int64_t ld, int metric,
                                                     const int64_t* __restrict__ rowmap,
                                                     int64_t n_src, const CT* __restrict__ cand,
                                                     int kstate,
                                                     int c, int k, int32_t* __restrict__ nbr,
                                                     float* __restrict__ dist) {
    extern __shared__ float s_q[];   // 4 waves x d
    const int l = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 4 + w;
    float* q = s_q + w * d;
    if (i < n) {
        int64_t src = rowmap ? rowmap[i] : i;
        if (src < 0 || src >= n_src) src = -1;
        for (int t = l; t < d; t += 64) q[t] = src >= 0 ? load_elem(X, dtype, src * ld + t) : 0.f;
    }
    __syncthreads();
    if (i >= n) return;
    uint64_t v[PER];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        int e = p * 64 + l;
        int32_t j = e < c ? cand_id(cand[i * kstate + e]) : SG_NONE;
        if (j < 0 || j >= n_src || j == (rowmap ? rowmap[i] : i)) {   // absent, out of range or self
            v[p] = EMPTY_KEY;
            continue;
        }
        const int64_t jb = (int64_t)j * ld;
        float s = 0.f;
        if (metric == SG_L2) {
            for (int t = 0; t < d; ++t) {
                float u = q[t] - load_elem(X, dtype, jb + t);
                s = fmaf(u, u, s);
            }
        } else {
            for (int t = 0; t < d; ++t) s = fmaf(q[t], load_elem(X, dtype, jb + t), s);
            s = -s;
        }
        v[p] = make_key(s, j);
    }
    wave_sort_multi<PER>(v);
    // a repeated candidate id gives equal adjacent keys: keep the first copy
    // (every lane runs every shuffle: element p*64+l-1 is lane l-1 of v[p],
    // or lane 63 of v[p-1] for l == 0)
    uint64_t prev[PER];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const uint64_t a = shfl_u64(v[p], (l + 63) & 63);
        const uint64_t b = shfl_u64(v[p > 0 ? p - 1 : 0], 63);
        prev[p] = l > 0 ? a : (p > 0 ? b : ~v[0]);
    }
    int kept = 0;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const bool keep = v[p] != EMPTY_KEY && v[p] != prev[p];
        const uint64_t m = __builtin_amdgcn_ballot_w64(keep);
        const int pos = kept + __builtin_popcountll(m & ((1ull << l) - 1));
        if (keep && pos < k) {
            nbr[i * k + pos] = key_id(v[p]);
            if (dist) dist[i * k + pos] = key_dist(v[p]);
        }
        kept += __builtin_popcountll(m);
    }
    for (int e = kept + l; e < k; e += 64) {
        nbr[i * k + e] = SG_NONE;
        if (dist) dist[i * k + e] = __builtin_inff();
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
inline int ksel_for(int k) { return k <= 32 ? 32 : k <= 64 ? 64 : k <= 128 ? 128 : 256; }

// Largest resident query half-row supported: the query fragment of 32 rows
// lives in 64 VGPRs per lane at most.
inline int nstep_for(int prec, int DP) {
    int vec = prec == SG_PREC_FP32 ? 1 : prec == SG_PREC_FP8 ? 32 : 8;
    return DP / 2 / vec;
}

struct Layout {
    int64_t n_pad;
    int DP;
    int ksel;
    size_t ops_bytes, norms_bytes, sexp_bytes, state_bytes, total;
};

inline Layout layout(int64_t n, int d, int k, int prec, int rerank) {
    Layout L;
    L.n_pad = (n + PAD_ROWS - 1) / PAD_ROWS * PAD_ROWS;
    L.DP = padded_d(prec, d);
    L.ksel = ksel_for(rerank > 0 ? rerank : k);
    L.ops_bytes = (size_t)L.n_pad * L.DP * elem_bytes(prec);
    L.norms_bytes = (size_t)L.n_pad * 4 * 2;
    L.sexp_bytes = prec == SG_PREC_FP8 ? (size_t)L.n_pad * 4 : 0;
    L.state_bytes = (size_t)L.n_pad * L.ksel * 8;
    L.total = align_up(L.ops_bytes, 256) + align_up(L.norms_bytes, 256) + align_up(L.sexp_bytes, 256) +
              align_up(L.state_bytes, 256) + 1024;
    return L;
}

typedef void (*topk_fn)(const uint8_t*, const float*, const int32_t*, int, const uint8_t*,
                        const int64_t*, const float*, const int32_t*, int, float, float, uint64_t*,
                        int32_t*, float*, int);
typedef void (*kstream_fn)(const float*, int, const float*, int, const float*, const int64_t*,
                           const float*, int, float, float, uint64_t*, int32_t*, float*, int);

// A distance kernel and its launch geometry.
struct Kern {
    topk_fn fn = nullptr;         // resident-query kernel, or
    kstream_fn ks = nullptr;      // k-streamed FP32 kernel
    int DP = 0;                   // padded operand row length it expects
    int nq_block = 0;             // queries per workgroup
    int threads = 0;
};

template <int P, int NSTEP, int W>
topk_fn pick_ksel(int ksel) {
    switch (ksel) {
        case 32: return dist_topk_kernel<P, NSTEP, 32, W, 1>;
        case 64: return dist_topk_kernel<P, NSTEP, 64, W, 1>;
        case 128: return dist_topk_kernel<P, NSTEP, 128, W, 1>;
        default: return dist_topk_kernel<P, NSTEP, 256, W, 1>;
    }
}

template <int P, int NSTEP, int W>
Kern resident(int ksel) {
    Kern k;
    k.fn = pick_ksel<P, NSTEP, W>(ksel);
    k.DP = 2 * NSTEP * Tr<P>::VEC;
    k.nq_block = 32 * W;
    k.threads = 64 * W;
    return k;
}

// Resident-query kernels are instantiated for the half-row lengths below
// (8 waves while the query fragment fits 2 waves per SIMD, 4 waves beyond);
// a smaller d pads up to the next one.  FP32 rows wider than 128 use the
// k-streamed kernel.
Kern pick_kernel(int prec, int d, int ksel) {
    const int need = nstep_for(prec, padded_d(prec, d));
    switch (prec) {
        case SG_PREC_FP32: {
            if (need <= 16) return resident<SG_PREC_FP32, 16, TWAVES>(ksel);
            if (need <= 32) return resident<SG_PREC_FP32, 32, TWAVES>(ksel);
            if (need <= 48) return resident<SG_PREC_FP32, 48, TWAVES>(ksel);
            if (need <= 64) return resident<SG_PREC_FP32, 64, TWAVES>(ksel);
            Kern k;
            switch (ksel) {
                case 32: k.ks = dist_topk_kstream_kernel<32>; break;
                case 64: k.ks = dist_topk_kstream_kernel<64>; break;
                case 128: k.ks = dist_topk_kstream_kernel<128>; break;
                default: k.ks = dist_topk_kstream_kernel<256>; break;
            }
            k.DP = (d + KS_DC - 1) / KS_DC * KS_DC;
            k.nq_block = KS_NQ;
            k.threads = KS_WAVES * 64;
            return k;
        }
        case SG_PREC_F16: {
            if (need <= 2) return resident<SG_PREC_F16, 2, TWAVES>(ksel);
            if (need <= 4) return resident<SG_PREC_F16, 4, TWAVES>(ksel);
            if (need <= 6) return resident<SG_PREC_F16, 6, TWAVES>(ksel);
            if (need <= 8) return resident<SG_PREC_F16, 8, TWAVES>(ksel);
            if (need <= 12) return resident<SG_PREC_F16, 12, TWAVES>(ksel);
            if (need <= 16) return resident<SG_PREC_F16, 16, TWAVES>(ksel);
            if (need <= 24) return resident<SG_PREC_F16, 24, 4>(ksel);
            if (need <= 32) return resident<SG_PREC_F16, 32, 4>(ksel);
            if (need <= 48) return resident<SG_PREC_F16, 48, 4>(ksel);
            return Kern();
        }
        case SG_PREC_BF16: {
            if (need <= 2) return resident<SG_PREC_BF16, 2, TWAVES>(ksel);
            if (need <= 4) return resident<SG_PREC_BF16, 4, TWAVES>(ksel);
            if (need <= 6) return resident<SG_PREC_BF16, 6, TWAVES>(ksel);
            if (need <= 8) return resident<SG_PREC_BF16, 8, TWAVES>(ksel);
            if (need <= 12) return resident<SG_PREC_BF16, 12, TWAVES>(ksel);
            if (need <= 16) return resident<SG_PREC_BF16, 16, TWAVES>(ksel);
            if (need <= 24) return resident<SG_PREC_BF16, 24, 4>(ksel);
            if (need <= 32) return resident<SG_PREC_BF16, 32, 4>(ksel);
            if (need <= 48) return resident<SG_PREC_BF16, 48, 4>(ksel);
            return Kern();
        }
        default: {
            if (need <= 1) return resident<SG_PREC_FP8, 1, TWAVES>(ksel);
            if (need <= 2) return resident<SG_PREC_FP8, 2, TWAVES>(ksel);
            if (need <= 4) return resident<SG_PREC_FP8, 4, TWAVES>(ksel);
            if (need <= 8) return resident<SG_PREC_FP8, 8, 4>(ksel);
            if (need <= 16) return resident<SG_PREC_FP8, 16, 4>(ksel);
            return Kern();
        }
    }
}

inline Layout layout_k(int64_t n, int d, int k, int prec, int rerank) {
    Layout L = layout(n, d, k, prec, rerank);
    Kern kk = pick_kernel(prec, d, L.ksel);
    if (kk.DP > 0) {
        L.DP = kk.DP;
        L.ops_bytes = (size_t)L.n_pad * L.DP * elem_bytes(prec);
        L.total = align_up(L.ops_bytes, 256) + align_up(L.norms_bytes, 256) +
                  align_up(L.sexp_bytes, 256) + align_up(L.state_bytes, 256) + 1024;
    }
    return L;
}

void check_args(const void* X, int dtype, int64_t n, int d, int64_t ld, int metric, int k, int prec,
                int rerank) {
    SG_REQUIRE(n >= 0 && n < (1ll << 31) - PAD_ROWS, "n out of range");
    SG_REQUIRE(d >= 1 && d <= 1024, "d must be in 1..1024");
    SG_REQUIRE(ld >= d, "ld must be >= d");
    SG_REQUIRE(k >= 1 && k <= 256, "k must be in 1..256");
    SG_REQUIRE(metric == SG_L2 || metric == SG_IP, "unknown metric");
    SG_REQUIRE(dtype >= SG_F32 && dtype <= SG_U8, "unknown dtype");
    SG_REQUIRE(prec >= SG_PREC_FP32 && prec <= SG_PREC_FP8, "unknown precision");
    SG_REQUIRE(rerank == 0 || (rerank >= k && rerank <= 256), "rerank must be 0 or in k..256");
    SG_REQUIRE(!(prec == SG_PREC_F16 && dtype != SG_F16 && dtype != SG_U8),
               "SG_PREC_F16 needs F16 or U8 input");
    SG_REQUIRE(!(prec == SG_PREC_F16 && dtype == SG_U8 && d > 128),
               "SG_PREC_F16 is exact on U8 input only for d <= 128");
    SG_REQUIRE(n == 0 || X != nullptr, "X is NULL");
}

}  // namespace knn
}  // namespace sg

using namespace sg;

extern "C" sg_status sg_knn_graph_workspace_size(int64_t n, int32_t d, int32_t k, sg_prec prec,
                                                 int32_t rerank, size_t* bytes) {
    return guarded([&] {
        SG_REQUIRE(bytes != nullptr, "bytes is NULL");
        SG_REQUIRE(n >= 0 && d >= 1 && d <= 1024 && k >= 1 && k <= 256, "bad sizes");
        knn::Layout L = knn::layout_k(n, d, k, prec, rerank);
        *bytes = n == 0 ? 0 : L.total;
    });
}

namespace sg {
namespace knn {

inline int64_t pad_rows(int64_t m) { return (m + PAD_ROWS - 1) / PAD_ROWS * PAD_ROWS; }

// Workspace of one call: candidate operands + side arrays for all n rows,
// and, for a row subset, the query operands + side arrays of its nq rows.
inline size_t total_bytes(const Layout& L, int64_t nq, int prec) {
    size_t t = L.total;
    if (nq >= 0) {
        const int64_t nqp = pad_rows(nq);
        t += align_up((size_t)nqp * L.DP * elem_bytes(prec), 256) + 2 * align_up((size_t)nqp * 4, 256) +
             align_up((size_t)nqp * 4, 256) + align_up((size_t)nqp * 8, 256);
        // the state then covers the query rows only
        t -= align_up(L.state_bytes, 256);
        t += align_up((size_t)nqp * L.ksel * 8, 256);
    }
    return t;
}

// kNN of rows (nq >= 0: the listed rows; nq < 0: every row) against all n rows.
void run(const void* X, int dtype, int64_t n, int d, int64_t ld, int metric, int k, int prec,
         int rerank, const int64_t* rows, int64_t nq, int32_t* nbr, float* dist, void* ws,
         size_t ws_bytes, hipStream_t s) {
    if (rerank == k) rerank = 0;
    Layout L = layout_k(n, d, k, prec, rerank);
    const Kern kern = pick_kernel(prec, d, L.ksel);
    if (!kern.fn && !kern.ks) {
        set_error("sg_knn: no distance kernel for this precision at d = " + std::to_string(d));
        throw Fail{SG_ERR_UNSUPPORTED};
    }
    const size_t need = total_bytes(L, rows ? nq : -1, prec);
    if (ws_bytes < need || ws == nullptr) {
        set_error("sg_knn: workspace too small (need " + std::to_string(need) + " bytes)");
        throw Fail{SG_ERR_WORKSPACE};
    }
    const bool subset = rows != nullptr;
    const int64_t nq_rows = subset ? nq : n;
    const int64_t nq_pad = subset ? pad_rows(nq) : L.n_pad;
    Carver cv(ws);
    uint8_t* ops = cv.take<uint8_t>(L.ops_bytes);
    float* ninit = cv.take<float>(L.n_pad);
    float* nout = cv.take<float>(L.n_pad);
    int32_t* sexp = prec == SG_PREC_FP8 ? cv.take<int32_t>(L.n_pad) : nullptr;
    uint8_t* qops = ops;
    float* qninit = ninit;
    float* qnout = nout;
    int32_t* qsexp = sexp;
    const int64_t* qid = nullptr;
    if (subset) {
        qops = cv.take<uint8_t>((size_t)nq_pad * L.DP * elem_bytes(prec));
        qninit = cv.take<float>(nq_pad);
        qnout = cv.take<float>(nq_pad);
        qsexp = cv.take<int32_t>(nq_pad);
        int64_t* qid_w = cv.take<int64_t>(nq_pad);
        fill<int64_t>(qid_w, -1, nq_pad, s);
        SG_HIP(hipMemcpyAsync(qid_w, rows, nq * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
        qid = qid_w;
    }
    uint64_t* state = cv.take<uint64_t>((size_t)nq_pad * L.ksel);

    prep_kernel<<<(unsigned)cdiv(L.n_pad, 4), 256, 0, s>>>(X, dtype, n, d, ld, nullptr, n, L.n_pad, L.DP,
                                                            prec, metric, ops, ninit, nout, sexp);
    SG_LAUNCH_CHECK();
    if (subset) {
        prep_kernel<<<(unsigned)cdiv(nq_pad, 4), 256, 0, s>>>(X, dtype, nq, d, ld, rows, n, nq_pad, L.DP,
                                                               prec, metric, qops, qninit, qnout, qsexp);
        SG_LAUNCH_CHECK();
    }
    fill<uint64_t>(state, EMPTY_KEY, nq_pad * L.ksel, s);
    const bool final_here = rerank == 0;
    const bool plain_ip = metric == SG_IP && !norm_corrected_ip(metric, prec);
    const float qmul = plain_ip ? -1.0f : -2.0f;
    const float osc = norm_corrected_ip(metric, prec) ? 0.5f : 1.0f;
    profile_record(s, true);
    const unsigned grid = (unsigned)(nq_pad / kern.nq_block);
    if (kern.fn)
        kern.fn<<<grid, kern.threads, 0, s>>>(ops, ninit, sexp, (int)n, qops, qid, qnout, qsexp,
                                              (int)nq_rows, qmul, osc, state, final_here ? nbr : nullptr,
                                              final_here ? dist : nullptr, k);
    else
        kern.ks<<<grid, kern.threads, 0, s>>>(reinterpret_cast<const float*>(ops), L.DP, ninit, (int)n,
                                              reinterpret_cast<const float*>(qops), qid, qnout,
                                              (int)nq_rows, qmul, osc, state, final_here ? nbr : nullptr,
                                              final_here ? dist : nullptr, k);
    SG_LAUNCH_CHECK();
    profile_record(s, false);
    if (!final_here) {
        const size_t shm = (size_t)4 * d * sizeof(float);
        const unsigned grid = (unsigned)cdiv(nq_rows, 4);
        if (rerank <= 64)
            rerank_kernel<1><<<grid, 256, shm, s>>>(X, dtype, nq_rows, d, ld, metric, rows, n, state, L.ksel,
                                                    rerank, k, nbr, dist);
        else if (rerank <= 128)
            rerank_kernel<2><<<grid, 256, shm, s>>>(X, dtype, nq_rows, d, ld, metric, rows, n, state, L.ksel,
                                                    rerank, k, nbr, dist);
        else
            rerank_kernel<4><<<grid, 256, shm, s>>>(X, dtype, nq_rows, d, ld, metric, rows, n, state, L.ksel,
                                                    rerank, k, nbr, dist);
        SG_LAUNCH_CHECK();
    }
}

}  // namespace knn
}  // namespace sg

extern "C" sg_status sg_knn_graph(const void* X, sg_dtype dtype, int64_t n, int32_t d, int64_t ld,
                                  sg_metric metric, int32_t k, sg_prec prec, int32_t rerank,
                                  int32_t* nbr, float* dist, void* ws, size_t ws_bytes, void* stream) {
    return guarded([&] {
        knn::check_args(X, dtype, n, d, ld, metric, k, prec, rerank);
        SG_REQUIRE(nbr != nullptr || n == 0, "nbr is NULL");
        if (n == 0) return;
        knn::run(X, dtype, n, d, ld, metric, k, prec, rerank, nullptr, -1, nbr, dist, ws, ws_bytes,
                 as_stream(stream));
    });
}

extern "C" sg_status sg_knn_rows_workspace_size(int64_t n, int32_t d, int64_t nq, int32_t k, sg_prec prec,
                                                int32_t rerank, size_t* bytes) {
    return guarded([&] {
        SG_REQUIRE(bytes != nullptr, "bytes is NULL");
        SG_REQUIRE(n >= 0 && nq >= 0 && d >= 1 && d <= 1024 && k >= 1 && k <= 256, "bad sizes");
        if (rerank == k) rerank = 0;
        knn::Layout L = knn::layout_k(n, d, k, prec, rerank);
        *bytes = (n == 0 || nq == 0) ? 0 : knn::total_bytes(L, nq, prec);
    });
}

extern "C" sg_status sg_knn_rows(const void* X, sg_dtype dtype, int64_t n, int32_t d, int64_t ld,
                                 sg_metric metric, const int64_t* rows, int64_t nq, int32_t k,
                                 sg_prec prec, int32_t rerank, int32_t* nbr, float* dist, void* ws,
                                 size_t ws_bytes, void* stream) {
    return guarded([&] {
        knn::check_args(X, dtype, n, d, ld, metric, k, prec, rerank);
        SG_REQUIRE(nq >= 0 && nq < (1ll << 31), "nq out of range");
        if (n == 0 || nq == 0) return;
        SG_REQUIRE(rows != nullptr && nbr != nullptr, "NULL pointer");
        knn::run(X, dtype, n, d, ld, metric, k, prec, rerank, rows, nq, nbr, dist, ws, ws_bytes,
                 as_stream(stream));
    });
}

extern "C" sg_status sg_rerank(const void* X, sg_dtype dtype, int64_t n, int32_t d, int64_t ld, sg_metric metric,
                               const int32_t* cand, int32_t c, int32_t k, int32_t* nbr, float* dist,
                               void* stream) {
    return guarded([&] {
        SG_REQUIRE(n >= 0 && n < (1ll << 31), "n out of range");
        SG_REQUIRE(d >= 1 && d <= 4096 && ld >= d, "bad d / ld");
        SG_REQUIRE(c >= 1 && c <= 256 && k >= 1 && k <= c, "need 1 <= k <= c <= 256");
        SG_REQUIRE(metric == SG_L2 || metric == SG_IP, "unknown metric");
        SG_REQUIRE(dtype >= SG_F32 && dtype <= SG_U8, "unknown dtype");
        if (n == 0) return;
        SG_REQUIRE(X && cand && nbr, "NULL pointer");
        hipStream_t s = as_stream(stream);
        const size_t shm = (size_t)4 * d * sizeof(float);
        const unsigned grid = (unsigned)cdiv(n, 4);
        if (c <= 64)
            knn::rerank_kernel<1, int32_t><<<grid, 256, shm, s>>>(X, dtype, n, d, ld, metric, nullptr, n, cand, c, c,
                                                                  k, nbr, dist);
        else if (c <= 128)
            knn::rerank_kernel<2, int32_t><<<grid, 256, shm, s>>>(X, dtype, n, d, ld, metric, nullptr, n, cand, c, c,
                                                                  k, nbr, dist);
        else
            knn::rerank_kernel<4, int32_t><<<grid, 256, shm, s>>>(X, dtype, n, d, ld, metric, nullptr, n, cand, c, c,
                                                                  k, nbr, dist);
        SG_LAUNCH_CHECK();
    });
}

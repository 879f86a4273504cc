// knn_impl.hpp -- device code and shared host helpers of the fused distance +
// top-k kernels: operand preparation, the register-resident and k-streamed
// distance kernels with their selection epilogue, the nearest-pivot kernel of
// the locality order, the FP32 re-rank, launch-shape variants and workspace
// layout.  Included by knn.hip (one shard) and batch.hip (many shards).
#pragma once
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <vector>

#include "common.hpp"

namespace sg {
namespace knn {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int intx8 __attribute__((ext_vector_type(8)));
typedef int intx4 __attribute__((ext_vector_type(4)));
typedef int intx16 __attribute__((ext_vector_type(16)));

constexpr int TWAVES = 8;        // waves per workgroup of the distance kernel
constexpr int TQB = 1;           // 32-query blocks per wave
constexpr int BQ = 32 * TQB * TWAVES;   // query rows per workgroup
constexpr int CB = 32;           // per-query candidate buffer (default; at most 32)
constexpr int PAD_ROWS = BQ;     // operand rows are padded to a multiple of this (>= any tile)

// ---------------------------------------------------------------------------
// operand traits: element bytes, elements per lane per MFMA step
// ---------------------------------------------------------------------------
template <int P> struct Tr;
template <> struct Tr<SG_PREC_FP32> { static constexpr int EB = 4, VEC = 1; };
template <> struct Tr<SG_PREC_F16> { static constexpr int EB = 2, VEC = 8; };
template <> struct Tr<SG_PREC_BF16> { static constexpr int EB = 2, VEC = 8; };
template <> struct Tr<SG_PREC_FP8> { static constexpr int EB = 1, VEC = 32; };
template <> struct Tr<SG_PREC_I8> { static constexpr int EB = 1, VEC = 16; };

// padded row length (elements) for a given d: two lane-halves, each a whole
// number of MFMA steps
__host__ __device__ inline int padded_d(int prec, int d) {
    int g = 2 * (prec == SG_PREC_FP32 ? 2 : prec == SG_PREC_FP8 ? 32 : prec == SG_PREC_I8 ? 16 : 8);
    return (d + g - 1) / g * g;
}
__host__ __device__ inline int elem_bytes(int prec) {
    return prec == SG_PREC_FP32 ? 4 : (prec == SG_PREC_FP8 || prec == SG_PREC_I8) ? 1 : 2;
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
//   L2, I8         key = ||c'||^2 - 2 q'.c'            dist = key + ||q'||^2
//   IP, I8         key = -128 S(c') - q'.c'             dist = key - 128 S(q') - 16384 d
// (x' = x - 128 for U8 rows, S = the sum of the elements; every term is an
// integer below 2^24, so the FP32 key is exact).  The INT8 accumulator starts
// at a = -floor(||c'||^2 / 2) (L2) or 128 S(c') (IP), so that the key is
// p - 2 acc (L2, p = ||c'||^2 mod 2) or -acc (IP): a subtile is rejected from
// the largest accumulator alone (key >= -2 acc, resp. -acc), and p is needed
// only for the candidates that pass.  A candidate's start and p travel as
// e = 2a + p (int32 bits in the start array; a = e >> 1, p = e & 1).
constexpr int32_t I8_PAD_E = -(1 << 30);   // padding rows: a = -2^29, keys near 2^30, never admitted
constexpr int32_t I8_PAD_A = I8_PAD_E >> 1;
// (x~ = the rounded operand row).  The reduced-precision IP key is the L2 key
// of the rounded rows with the exact norm put back: its rounding error scales
// with ||q - c|| instead of ||q|| ||c||, which keeps near neighbours apart.
__host__ __device__ inline bool norm_corrected_ip(int metric, int prec) {
    return metric == SG_IP && (prec == SG_PREC_BF16 || prec == SG_PREC_FP8);
}

// LPR lanes per operand row (source row rowmap[row], or row itself when
// rowmap is NULL), 64 / LPR rows per wavefront.  Writes the converted row (zero padded to DP),
// the accumulator start of the row as a candidate (ninit, NaN for padding
// rows), its output offset as a query (nout) and, for FP8, the row's scale
// exponent (ninit, nout and sexp may be NULL).
template <int LPR>
__global__ void prep_kernel(const void* __restrict__ X, int dtype, int64_t n, int d, int64_t ld,
                            const int64_t* __restrict__ rowmap, int64_t n_src, int64_t n_pad, int DP,
                            int prec, int metric, uint8_t* __restrict__ ops, float* __restrict__ ninit,
                            float* __restrict__ nout, int32_t* __restrict__ sexp) {
    const int l = threadIdx.x & (LPR - 1);
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x / LPR) + threadIdx.x / LPR;
    if (row >= n_pad) return;
    const int eb = elem_bytes(prec);
    uint8_t* out = ops + row * (int64_t)DP * eb;
    const int64_t src_row = row < n ? (rowmap ? rowmap[row] : row) : -1;
    if (src_row < 0 || src_row >= n_src) {      // padding (or an out-of-range listed row)
        for (int t = l; t < DP; t += LPR) {
            if (eb == 4) reinterpret_cast<float*>(out)[t] = 0.f;
            else if (eb == 2) reinterpret_cast<uint16_t*>(out)[t] = 0;
            else out[t] = 0;
        }
        if (l == 0) {
            // never admitted: NaN fails every comparison (INT8: a start far
            // beyond any key, turned into NaN where keys are formed)
            if (ninit) ninit[row] = prec == SG_PREC_I8 ? __builtin_bit_cast(float, I8_PAD_E) : __builtin_nanf("");
            if (nout) nout[row] = 0.f;
            if (sexp) sexp[row] = 0;
        }
        return;
    }
    const int64_t base = src_row * ld;
    int sx = 0;
    float inv = 1.0f;
    if (prec == SG_PREC_FP8) {
        float amax = 0.f;
        for (int t = l; t < d; t += LPR) amax = fmaxf(amax, fabsf(load_elem(X, dtype, base + t)));
        for (int o = LPR / 2; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
        // smallest power of two s with amax / s <= 448
        if (amax > 0.f) {
            sx = (int)ceilf(log2f(amax / 448.0f));
            while (__builtin_ldexpf(amax, -sx) > 448.0f) ++sx;
            while (sx > -126 && __builtin_ldexpf(amax, -(sx - 1)) <= 448.0f) --sx;
        }
        inv = __builtin_ldexpf(1.0f, -sx);
    }
    float ssq = 0.f, ssx = 0.f;
    // u8 rows to INT8 operands, eight elements per lane and access when rows
    // and operand rows are 8-byte aligned (every element lies in a group of
    // eight wholly below d or wholly in the padding); the sums are exact
    // integers, so their order does not matter
    const bool u8_vec = prec == SG_PREC_I8 && dtype == SG_U8 && (d & 7) == 0 && (DP & 7) == 0 && (ld & 7) == 0 &&
                        (reinterpret_cast<uintptr_t>(X) & 7) == 0 && (reinterpret_cast<uintptr_t>(ops) & 7) == 0;
    if (u8_vec) {
        const uint8_t* src = static_cast<const uint8_t*>(X) + base;
        for (int t = 8 * l; t < DP; t += 8 * LPR) {
            uint2 w = make_uint2(0x80808080u, 0x80808080u);   // padding: c = 0
            if (t < d) w = *reinterpret_cast<const uint2*>(src + t);
            // c = b - 128 as a signed byte is b with its top bit flipped
            *reinterpret_cast<uint2*>(out + t) = make_uint2(w.x ^ 0x80808080u, w.y ^ 0x80808080u);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int c = (int)(((k < 4 ? w.x : w.y) >> (8 * (k & 3))) & 0xFFu) - 128;
                ssx += (float)c;
                ssq += (float)(c * c);
            }
        }
    }
    for (int t = l; t < DP && !u8_vec; t += LPR) {
        float v = t < d ? load_elem(X, dtype, base + t) : 0.f;
        float q;
        switch (prec) {
            case SG_PREC_I8: {   // U8 rows shifted by -128 (padding elements 0)
                const int c = t < d ? (int)v - 128 : 0;
                out[t] = (uint8_t)(int8_t)c;
                q = (float)c;
                ssx += q;        // the element sum S (exact: |S| < 2^24)
                break;
            }
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
        if (prec != SG_PREC_I8) ssx += v * v;
    }
    for (int o = LPR / 2; o > 0; o >>= 1) {
        ssq += __shfl_xor(ssq, o, 64);
        ssx += __shfl_xor(ssx, o, 64);
    }
    if (l == 0) {
        float term = metric == SG_L2 ? ssq : norm_corrected_ip(metric, prec) ? ssq - ssx : 0.f;
        float oterm = term;
        if (prec == SG_PREC_I8) {
            // the accumulator start and parity of the row as a candidate (see
            // the key table above); ssq and ssx are exact integers
            const int32_t n2 = (int32_t)ssq, sx8 = (int32_t)ssx;
            const int32_t e = metric == SG_L2 ? -2 * (n2 >> 1) + (n2 & 1) : 2 * 128 * sx8;
            term = __builtin_bit_cast(float, e);
            if (metric == SG_IP) oterm = -128.f * ssx - 16384.f * (float)d;
        }
        if (ninit) ninit[row] = term;
        if (nout) nout[row] = oterm;
        if (sexp) sexp[row] = sx;
    }
}

// Operand preparation of n_pad rows with a lane count per row that suits the
// padded row length (16 lanes for rows of up to 128 elements, 32 up to 256,
// else a wavefront), so that short rows do not leave most of a wave idle.
inline void launch_prep(const void* X, int dtype, int64_t n, int d, int64_t ld, const int64_t* rowmap, int64_t n_src,
                        int64_t n_pad, int DP, int prec, int metric, uint8_t* ops, float* ninit, float* nout,
                        int32_t* sexp, hipStream_t s) {
    if (n_pad <= 0) return;
    if (DP <= 128)
        prep_kernel<16><<<(unsigned)cdiv(n_pad, 16), 256, 0, s>>>(X, dtype, n, d, ld, rowmap, n_src, n_pad, DP, prec,
                                                                   metric, ops, ninit, nout, sexp);
    else if (DP <= 256)
        prep_kernel<32><<<(unsigned)cdiv(n_pad, 8), 256, 0, s>>>(X, dtype, n, d, ld, rowmap, n_src, n_pad, DP, prec,
                                                                  metric, ops, ninit, nout, sexp);
    else
        prep_kernel<64><<<(unsigned)cdiv(n_pad, 4), 256, 0, s>>>(X, dtype, n, d, ld, rowmap, n_src, n_pad, DP, prec,
                                                                  metric, ops, ninit, nout, sexp);
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
template <int NSTEP>
struct Frag<SG_PREC_I8, NSTEP> {
    intx4 v[NSTEP];   // 16 signed bytes per MFMA step
};

// Accumulator of one 32x32 subtile: FP32, or exact INT32 for I8 operands
// (converted to the FP32 key when the subtile is selected).
template <int P>
using AccT = typename std::conditional<P == SG_PREC_I8, intx16, floatx16>::type;

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
    } else if constexpr (P == SG_PREC_I8) {
#pragma unroll
        for (int s = 0; s < NSTEP; ++s) f.v[s] = *reinterpret_cast<const intx4*>(rowp + s * 16);
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
    if constexpr (P == SG_PREC_I8) {
        (void)f;   // INT8 keys take the factor when they are converted (subtile_keys)
        (void)qmul;
    } else if constexpr (P == SG_PREC_FP8) {
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

// Largest divisor of n that is at most m.
constexpr int group_of(int n, int m) {
    for (int g = m; g > 1; --g)
        if (n % g == 0) return g;
    return 1;
}

// acc += A(32 candidate rows at arow, LDS) x Q(32 queries) over the padded
// row, in groups of steps whose A fragments are all requested before the
// group's MFMA chain starts, so that one LDS round trip covers the group
// (16-bit groups of at most GMAX steps: fewer keep fewer registers live).
template <int P, int NSTEP, int GMAX = 8>
__device__ inline floatx16 mfma_tile(const uint8_t* arow, const Frag<P, NSTEP>& q, floatx16 acc,
                                     int sa, int sb) {
    if constexpr (P == SG_PREC_FP32) {
        constexpr int G = 4 * group_of(NSTEP / 4, 4);   // floats per group
        static_assert(NSTEP % 4 == 0, "FP32 steps come in whole float4s");
#pragma unroll
        for (int g = 0; g < NSTEP; g += G) {
            floatx4 a[G / 4];
#pragma unroll
            for (int s = 0; s < G / 4; ++s) a[s] = *reinterpret_cast<const floatx4*>(arow + (g + 4 * s) * 4);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int s = 0; s < G; ++s)
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s / 4][s % 4], q.v[g + s], acc, 0, 0, 0);
        }
    } else if constexpr (P == SG_PREC_F16 || P == SG_PREC_BF16) {
        constexpr int G = group_of(NSTEP, GMAX);
#pragma unroll
        for (int g = 0; g < NSTEP; g += G) {
            intx4 a[G];
#pragma unroll
            for (int s = 0; s < G; ++s) a[s] = *reinterpret_cast<const intx4*>(arow + (g + s) * 16);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int s = 0; s < G; ++s) {
                if constexpr (P == SG_PREC_F16)
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, a[s]), q.v[g + s],
                                                                 acc, 0, 0, 0);
                else
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[s]),
                                                                  q.v[g + s], acc, 0, 0, 0);
            }
        }
    } else {
        constexpr int G = group_of(NSTEP, 4);
#pragma unroll
        for (int g = 0; g < NSTEP; g += G) {
            intx4 a[2 * G];
#pragma unroll
            for (int s = 0; s < 2 * G; ++s) a[s] = *reinterpret_cast<const intx4*>(arow + g * 32 + s * 16);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int s = 0; s < G; ++s) {
                const intx8 f = intx8{a[2 * s][0], a[2 * s][1], a[2 * s][2], a[2 * s][3],
                                      a[2 * s + 1][0], a[2 * s + 1][1], a[2 * s + 1][2], a[2 * s + 1][3]};
                acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(f, q.v[g + s], acc, 0, 0, 0, sa, 0, sb);
            }
        }
    }
    return acc;
}

// acc += A(32 candidate rows at arow, LDS) x Q(32 queries) over the padded
// row with INT8 operands: exact INT32 sums.
template <int NSTEP, int GMAX = 8>
__device__ inline intx16 mfma_tile_i8(const uint8_t* arow, const Frag<SG_PREC_I8, NSTEP>& q, intx16 acc) {
    constexpr int G = group_of(NSTEP, GMAX);
#pragma unroll
    for (int g = 0; g < NSTEP; g += G) {
        intx4 a[G];
#pragma unroll
        for (int s = 0; s < G; ++s) a[s] = *reinterpret_cast<const intx4*>(arow + (g + s) * 16);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < G; ++s) acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[s], q.v[g + s], acc, 0, 0, 0);
    }
    return acc;
}

// Exact FP32 keys of an INT8 subtile, key = p + qmul * acc (qmul = -2 for
// L2 with the rows' parities p, -1 for IP with p = 0); padding rows give NaN.
__device__ inline floatx16 i8_keys(const intx16& acc, const intx4 (&par)[4], int qmul) {
    floatx16 k;
#pragma unroll
    for (int i = 0; i < 16; ++i)
        k[i] = acc[i] == I8_PAD_A ? __builtin_nanf("") : (float)(par[i >> 2][i & 3] + qmul * acc[i]);
    return k;
}

// Largest of a lane's 16 INT8 accumulators (eight 3-input maximums).
__device__ inline int32_t max16(const intx16& a) {
    const int32_t p0 = max(max(a[0], a[1]), a[2]), p1 = max(max(a[3], a[4]), a[5]);
    const int32_t p2 = max(max(a[6], a[7]), a[8]), p3 = max(max(a[9], a[10]), a[11]);
    const int32_t p4 = max(max(a[12], a[13]), a[14]);
    return max(max(max(p0, p1), p2), max(max(p3, p4), a[15]));
}

template <int P, int NSTEP, int BCR = 0>
struct Shape {
    static constexpr int DH = NSTEP * Tr<P>::VEC;             // elements per lane-half
    static constexpr int ROW_BYTES = 2 * DH * Tr<P>::EB;      // padded operand row
    static constexpr int RS = ROW_BYTES + 16;                 // LDS row stride (bank spread)
    // candidate rows per LDS tile (BCR, or by default so that two tiles, the
    // double buffer, stay within ~70 KB)
    static constexpr int BC = BCR > 0 ? BCR : ROW_BYTES <= 256 ? 128 : ROW_BYTES <= 512 ? 64 : 32;
    static constexpr int NSUB = BC / 32;
    static_assert(BC % 32 == 0, "tiles hold whole 32-row subtiles");
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
            for (int p = 0; p < PER; ++p) v[p] = cmpx(v[p], j, (l & j) == 0);
        }
    }
}

// Merge one query's candidate buffer (c <= 32 keys in LDS) into its
// sorted top-KSEL list in the workspace, all in registers: the list's load is
// issued first; the buffer is sorted descending in lanes 0..31 and moved to
// lanes 32..63, where the element-wise minimum with the list's last 64 keys
// leaves the KSEL smallest of both as a bitonic sequence, which is then
// merged.  A fresh list (the query's first merge) is taken as empty without
// reading the workspace, which therefore needs no initialisation.  Returns the
// new admission threshold: the KSEL-th distance (+inf while the list is not
// full).
template <int KSEL>
__device__ float merge_query(uint64_t* __restrict__ gstate, const uint64_t* buf, int c, bool fresh = false) {
    constexpr int PER = KSEL >= 64 ? KSEL / 64 : 1;
    const int l = lane_id();
    uint64_t v[PER];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int e = p * 64 + l;
        v[p] = e < KSEL && !fresh ? gstate[e] : EMPTY_KEY;   // a fresh list is empty, nothing to load
    }
    uint64_t b = l < c ? buf[l] : EMPTY_KEY;
    b = low_half_to_high(half_sort_desc_u64(b));
    if (l >= 32 && b < v[PER - 1]) v[PER - 1] = b;
    bitonic_merge_multi<PER>(v);
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int e = p * 64 + l;
        if (e < KSEL) gstate[e] = v[p];
    }
    return key_dist(readlane_u64(v[(KSEL - 1) / 64], (KSEL - 1) & 63));
}

// Per-wave selection state: the admission threshold of each of the wave's
// 32*QB queries (lanes l and l+32 share query l%32 of each block), the id
// excluded as the query itself, and the LDS buffers / counters and workspace
// top-KSEL lists of those queries.
template <int KSEL, int QB, int CBQ = CB>
struct Selector {
    static_assert(CBQ <= 32, "a buffer is sorted inside one wave half");
    float thr[QB];
    // INT8 keys only (qm_int = the key's factor on the accumulator, -2 or -1;
    // 0 for other operands): the smallest subtile maximum of the accumulator
    // that can still give a key <= thr, kept beside thr so that a subtile is
    // rejected by one integer comparison
    int32_t amin[QB];
    int qm_int;
    __device__ static int32_t i8_amin(float t, int qm) {
        if (!(t < 3.0e38f)) return INT32_MIN;   // +inf: everything passes
        // qm * M <= t  <=>  M >= ceil(t / qm) (t an exact integer below 2^24)
        return (int32_t)ceilf(qm == -2 ? -0.5f * t : -t);
    }
    int64_t qself[QB];
    int64_t qlo, qhi;  // wave-uniform range of the wave's query ids
    uint64_t* state;   // state row of the wave's first query
    uint64_t* buf;     // LDS buffers of the wave's queries (32*QB*CBQ keys)
    int fill[QB];      // buffer fill of the lane's query (same in both lanes)
    uint32_t fresh[QB];  // wave-uniform: bit q set while query q's list has not been written

    // After qself is set: the smallest and largest query id of the wave, so
    // that a subtile whose candidate ids miss [qlo, qhi] skips the per-lane
    // self test with one scalar comparison (no valid query: qlo > qhi).
    __device__ void init_self_range() {
        uint64_t lo = (uint64_t)INT64_MAX, hi = 0;
#pragma unroll
        for (int b = 0; b < QB; ++b) {
            if (qself[b] >= 0) {
                lo = (uint64_t)qself[b] < lo ? (uint64_t)qself[b] : lo;
                hi = (uint64_t)qself[b] > hi ? (uint64_t)qself[b] : hi;
            }
        }
#pragma unroll
        for (int j = 1; j < 64; j <<= 1) {
            const uint64_t ol = lane_xor_u64(lo, j), oh = lane_xor_u64(hi, j);
            lo = ol < lo ? ol : lo;
            hi = oh > hi ? oh : hi;
        }
        qlo = (int64_t)readlane_u64(lo, 0);
        qhi = (int64_t)readlane_u64(hi, 0);
    }

    // Smallest of a lane's 16 distances (eight 3-input minimums; NaN only if all are).
    __device__ static float min16(const floatx16& a) {
        const float p0 = fminf(fminf(a[0], a[1]), a[2]), p1 = fminf(fminf(a[3], a[4]), a[5]);
        const float p2 = fminf(fminf(a[6], a[7]), a[8]), p3 = fminf(fminf(a[9], a[10]), a[11]);
        const float p4 = fminf(fminf(a[12], a[13]), a[14]);
        return fminf(fminf(fminf(p0, p1), p2), fminf(fminf(p3, p4), a[15]));
    }

    // Admit the candidates of one 32x32 subtile (operand rows cbase..cbase+31,
    // whose ids are tpid[0..32), or cbase.. when tpid is NULL) whose key is
    // <= the threshold, one accumulator element at a time: from the element's
    // ballot the two lanes of a query see each other's hit, so they write
    // their keys at known slots (no atomics) and both keep the query's buffer
    // fill in a register.  The 16 elements go in chunks of E (one chunk of 16
    // for CBQ = 32, two of 8 for 16 <= CBQ < 32): round 1 stops at the first element some
    // buffer cannot take; then every query whose buffer could not take two
    // keys per remaining element of the chunk is merged, and round 2 finishes
    // the chunk without checks (an emptied buffer holds the 2E <= CBQ keys a
    // chunk can add).  A merged query's lowered threshold takes effect at the
    // next chunk.  Admission is exact in any
    // candidate order: a candidate whose distance exceeds the K-th distance of
    // a subset already seen cannot be in the top K, and one that equals it is
    // admitted and ranked by (distance, id) in the merge.  The query itself
    // and padding rows are NaN, which no comparison admits.
    __device__ void admit(floatx16 (&acc)[QB], int64_t cbase, const int32_t* tpid) {
        static_assert(CBQ >= 16 && CBQ <= 32, "a chunk of E elements must fit an emptied buffer");
        const int l = lane_id();
        const int ql = l & 31;
        const int h = l >> 5;
        if (cbase <= qhi && cbase + 31 >= qlo) {
            const int32_t rel0 = (int32_t)(cbase - qlo);
#pragma unroll
            for (int b = 0; b < QB; ++b) {
                const int32_t me = qself[b] >= 0 ? (int32_t)(qself[b] - qlo) : INT32_MIN;
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    if (rel0 + out_row(i, l) == me) acc[b][i] = __builtin_nanf("");
            }
        }
        bool any = false;
#pragma unroll
        for (int b = 0; b < QB; ++b) any |= min16(acc[b]) <= thr[b];
        if (!__builtin_amdgcn_ballot_w64(any)) return;
        // the ids of this lane's 16 rows: groups of 4 consecutive rows
        int32_t ids[16];
        if (tpid) {
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const intx4 v = *reinterpret_cast<const intx4*>(tpid + g * 8 + h * 4);
#pragma unroll
                for (int e = 0; e < 4; ++e) ids[g * 4 + e] = v[e];
            }
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i) ids[i] = (int32_t)(cbase + out_row(i, l));
        }
        // chunks of E elements: a chunk adds at most 2E <= CBQ keys per query
        constexpr int E = CBQ == 32 ? 16 : 8;
#pragma unroll
        for (int b = 0; b < QB; ++b) {
            float t = thr[b];
            int c = fill[b];
            uint64_t* qbuf = buf + (b * 32 + ql) * CBQ;
#pragma unroll
            for (int c0 = 0; c0 < 16; c0 += E) {
                int stop = c0 + E;   // wave-uniform: first element round 1 left
#pragma unroll
                for (int i = c0; i < c0 + E; ++i) {
                    if (i >= stop) continue;
                    const bool hit = acc[b][i] <= t;
                    const uint64_t m = __builtin_amdgcn_ballot_w64(hit);
                    if (m == 0) continue;
                    const int pa = (int)(((uint32_t)m >> ql) & 1u);
                    const int pb = (int)(((uint32_t)(m >> 32) >> ql) & 1u);
                    if (__builtin_amdgcn_ballot_w64(c + pa + pb > CBQ)) {
                        stop = i;
                        continue;
                    }
                    if (hit) qbuf[c + (h ? pa : 0)] = make_key(acc[b][i], ids[i]);
                    c += pa + pb;
                }
                if (stop < c0 + E) {
                    const int room = 2 * (c0 + E - stop);
                    uint32_t need = (uint32_t)__builtin_amdgcn_ballot_w64(h == 0 && c + room > CBQ);
                    float tnext = t;
                    while (need) {
                        const int qi = __builtin_ctz(need);
                        need &= need - 1;
                        const int q2 = b * 32 + qi;
                        const float tq = merge_query<KSEL>(state + (int64_t)q2 * KSEL, buf + q2 * CBQ,
                                                           __builtin_amdgcn_readlane(c, qi), (fresh[b] >> qi) & 1u);
                        fresh[b] &= ~(1u << qi);
                        if (ql == qi) {
                            c = 0;
                            tnext = tq;
                        }
                    }
#pragma unroll
                    for (int i = c0; i < c0 + E; ++i) {
                        if (i < stop) continue;
                        const bool hit = acc[b][i] <= t;
                        const uint64_t m = __builtin_amdgcn_ballot_w64(hit);
                        if (m == 0) continue;
                        const int pa = (int)(((uint32_t)m >> ql) & 1u);
                        const int pb = (int)(((uint32_t)(m >> 32) >> ql) & 1u);
                        if (hit) qbuf[c + (h ? pa : 0)] = make_key(acc[b][i], ids[i]);
                        c += pa + pb;
                    }
                    t = tnext;   // a merged query's lowered threshold applies from the next chunk
                }
            }
            thr[b] = t;
            if (qm_int) amin[b] = i8_amin(t, qm_int);
            fill[b] = c;
        }
    }

    // Merge every non-empty buffer, and write the list of every query still
    // fresh (empty, or holding only the keys of its buffer), at the end of
    // the candidate stream: every list is then in the workspace.
    __device__ void drain() {
        const int l = lane_id();
#pragma unroll
        for (int b = 0; b < QB; ++b) {
            const uint64_t m = __builtin_amdgcn_ballot_w64(l < 32 && (fill[b] > 0 || ((fresh[b] >> l) & 1u)));
            uint32_t need = (uint32_t)m;
            while (need) {
                const int qi = __builtin_ctz(need);
                need &= need - 1;
                const int q2 = b * 32 + qi;
                merge_query<KSEL>(state + (int64_t)q2 * KSEL, buf + q2 * CBQ,
                                  __builtin_amdgcn_readlane(fill[b], qi), (fresh[b] >> qi) & 1u);
            }
            fresh[b] = 0;
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
};

// Arguments of one distance-kernel launch (a block of queries against one
// candidate set).  Candidate operand row j has id cpid[j] (NULL: j); query
// row q writes output row qout[q] (NULL: q) and excludes the candidate whose
// operand row is qid[q] (NULL: q; negative: none).
struct TopkArgs {
    const uint8_t* ops;      // candidate operands, padded rows
    const float* ninit;      // accumulator start per candidate (NaN: padding)
    const int32_t* sexp;     // FP8 row scale exponents (else NULL)
    const int32_t* cpid;     // candidate ids (nullable)
    int n;                   // candidate rows
    const uint8_t* qops;     // query operands (padded to whole blocks)
    const int64_t* qid;      // self row per query (nullable)
    const float* qnout;      // output term per query
    const int32_t* qsexp;
    const int64_t* qout;     // output row per query (nullable)
    int nq;                  // query rows
    float qmul, osc;
    uint64_t* state;         // sorted top-KSEL keys per query (operand order)
    int32_t* nbr;            // nullable: no lists written
    float* dist;             // nullable
    int k_out;
};

// Final lists of the wave's queries: ids and output distances.
__device__ inline void write_lists(const TopkArgs& A, int ksel, int64_t q0, int nqw) {
    const int l = lane_id();
    for (int qi = 0; qi < nqw; ++qi) {
        const int64_t q = q0 + qi;
        if (q >= A.nq) break;
        const float qn = A.qnout[q];
        const int64_t o = A.qout ? A.qout[q] : q;
        for (int t = l; t < A.k_out; t += 64) {
            const uint64_t key = A.state[q * ksel + t];
            A.nbr[o * A.k_out + t] = key_id(key);
            if (A.dist)
                A.dist[o * A.k_out + t] = key == EMPTY_KEY ? __builtin_inff() : (key_dist(key) + qn) * A.osc;
        }
    }
}

// LDS of the register-resident kernel.
template <int P, int NSTEP, int WAVES, int QB, int CBQ, int BCR>
struct TopkSmem {
    using S = Shape<P, NSTEP, BCR>;
    static constexpr int NQ = 32 * QB * WAVES;
    __align__(16) uint8_t tile[2][S::BC * S::RS];
    __align__(16) float norm[2][S::BC];
    __align__(16) int32_t pid[2][S::BC];
    int32_t sexp[2][P == SG_PREC_FP8 ? S::BC : 1];
    int32_t par[2][P == SG_PREC_I8 ? S::BC : 1];   // INT8 L2: parity of ||c'||^2
    uint64_t buf[NQ * CBQ];
};

// Candidate tile order of a query block: first the tiles of the 256-row
// group that holds the block's own rows (with rows in locality order these
// hold the queries' closest neighbours, so the thresholds tighten at once),
// then all other tiles in ascending order -- the same order for every block,
// so that concurrently running workgroups stream the same rows through L2.
struct ScanOrder {
    int t0, R;
    __device__ ScanOrder(int64_t first_row, int bc, int ntiles) {
        R = (256 + bc - 1) / bc;
        if (R > ntiles) R = ntiles;
        const int own = (int)(first_row / 256 * 256 / bc);
        t0 = own < ntiles - R ? own : ntiles - R;
    }
    __device__ int tile(int t) const {
        if (t < R) return t0 + t;
        const int g = t - R;
        return g < t0 ? g : g + R;
    }
};

// One block of NQ = 32*QB*WAVES queries (query rows qb*NQ.. of A.qops)
// against all A.n candidate rows: the fused distance tile + top-k with
// register-resident queries.  Candidate tiles (BC rows) are staged in LDS,
// double buffered, the next one or two tiles already in flight in registers
// while the current one is computed.  Within a tile the MFMAs of subtile s+1 are
// issued before the selection epilogue of subtile s so that both run at once.
// Tiles are visited in ScanOrder.
template <int P, int NSTEP, int KSEL, int WAVES, int QB, int CBQ, int BCR>
__device__ void topk_block(TopkSmem<P, NSTEP, WAVES, QB, CBQ, BCR>& sm, int64_t qb, const TopkArgs& A) {
    using S = Shape<P, NSTEP, BCR>;
    constexpr int BC = S::BC, NSUB = S::NSUB, RB = S::ROW_BYTES, RS = S::RS;
    constexpr int NT = WAVES * 64;
    constexpr int NQ = 32 * QB * WAVES;
    constexpr int CHUNKS = BC * RB / 16;                        // 16-byte chunks per tile
    constexpr int CPT = (CHUNKS + NT - 1) / NT;                 // chunks per thread
    constexpr int GMAX = CBQ < 32 ? 4 : 8;                      // A-fragment group (registers)

    const int tid = threadIdx.x;
    const int l = tid & 63;
    const int w = tid >> 6;
    const int h = l >> 5;
    const int ql = l & 31;
    const int64_t qblk0 = qb * NQ + w * 32 * QB;   // first query of this wave

    Frag<P, NSTEP> qf[QB];
    int q_scale[QB];
    Selector<KSEL, QB, CBQ> sel;
    sel.state = A.state + qblk0 * KSEL;
    sel.buf = sm.buf + w * 32 * QB * CBQ;
#pragma unroll
    for (int b = 0; b < QB; ++b) {
        const int64_t qg = qblk0 + b * 32 + ql;
        load_frag<P, NSTEP>(qf[b], A.qops + qg * RB + h * (RB / 2));
        scale_query<P, NSTEP>(qf[b], A.qmul);
        q_scale[b] = 127;
        if constexpr (P == SG_PREC_FP8) q_scale[b] = 127 + A.qsexp[qg] + 1;
        sel.thr[b] = __builtin_inff();
        sel.amin[b] = INT32_MIN;
        sel.fresh[b] = ~0u;
        sel.fill[b] = 0;
        sel.qself[b] = qg < A.nq ? (A.qid ? A.qid[qg] : qg) : -1;
    }
    sel.qm_int = P == SG_PREC_I8 ? (int)A.qmul : 0;
    sel.init_self_range();

    const int ntiles = (A.n + BC - 1) / BC;
    const ScanOrder order(qb * NQ, BC, ntiles);
    auto tile_row = [&](int t) { return order.tile(t) * BC; };

    // tile staging: global -> registers -> LDS (two buffers).  4-wave shapes
    // with 32-entry buffers, and those with more than 16 whose tile is one
    // 16-byte load per thread, keep two register sets, so that a tile's loads
    // are issued two tiles before it is committed (their tiles are short); the
    // others, whose registers are fuller, keep one (loads one tile ahead).
    constexpr int DEPTH = WAVES == 4 && (CBQ == 32 || (CBQ > 16 && CPT == 1)) ? 2 : 1;
    intx4 pre[DEPTH][CPT];
    float pre_norm[DEPTH] = {};
    int32_t pre_pid[DEPTH] = {}, pre_sexp[DEPTH] = {};
    // Every thread issues the same loads (the per-row values are read by all
    // threads, thread t taking row t % BC), so that the compiler can count the
    // loads still in flight when a register set is committed.
    auto prefetch = [&](int r, int j0) {
        const uint8_t* src = A.ops + (int64_t)j0 * RB;
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int c = tid + u * NT;
            if (CHUNKS % NT == 0 || c < CHUNKS) pre[r][u] = *reinterpret_cast<const intx4*>(src + (int64_t)c * 16);
        }
        const int rr = tid % BC;
        pre_norm[r] = A.ninit[j0 + rr];
        pre_pid[r] = A.cpid ? A.cpid[j0 + rr] : 0;
        if constexpr (P == SG_PREC_FP8) pre_sexp[r] = A.sexp[j0 + rr];
    };
    auto commit = [&](int r, int buf) {
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int c = tid + u * NT;
            if (CHUNKS % NT == 0 || c < CHUNKS) {
                const int row = c / (RB / 16), o = c % (RB / 16);
                *reinterpret_cast<intx4*>(&sm.tile[buf][row * RS + o * 16]) = pre[r][u];
            }
        }
        if (tid < BC) {
            if constexpr (P == SG_PREC_I8) {
                const int32_t e = __builtin_bit_cast(int32_t, pre_norm[r]);
                sm.norm[buf][tid] = __builtin_bit_cast(float, e >> 1);
                sm.par[buf][tid] = e & 1;
            } else {
                sm.norm[buf][tid] = pre_norm[r];
            }
            sm.pid[buf][tid] = pre_pid[r];
            if constexpr (P == SG_PREC_FP8) sm.sexp[buf][tid] = pre_sexp[r];
        }
    };
    using Acc = AccT<P>;
    // the accumulator starts of the lane's 16 candidate rows of a subtile
    auto starts = [&](floatx4 (&nv)[4], int buf, int sub) {
#pragma unroll
        for (int g = 0; g < 4; ++g)
            nv[g] = *reinterpret_cast<const floatx4*>(&sm.norm[buf][sub * 32 + g * 8 + h * 4]);
    };
    auto compute = [&](Acc (&acc)[QB], int buf, int sub) {
        const uint8_t* arow = &sm.tile[buf][(sub * 32 + ql) * RS + h * (RB / 2)];
        if constexpr (P == SG_PREC_I8) {
            // the INT8 starts are int32 words in the same LDS array (read as
            // integers: a bit cast of a vector element is not used here)
            intx4 iv[4];
#pragma unroll
            for (int g = 0; g < 4; ++g)
                iv[g] = *reinterpret_cast<const intx4*>(&sm.norm[buf][sub * 32 + g * 8 + h * 4]);
#pragma unroll
            for (int b = 0; b < QB; ++b) {
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[b][i] = iv[i >> 2][i & 3];
            }
            for (int b = 0; b < QB; ++b) acc[b] = mfma_tile_i8<NSTEP, GMAX>(arow, qf[b], acc[b]);
        } else {
            floatx4 nv[4];
            starts(nv, buf, sub);
            int a_scale = 127;
            if constexpr (P == SG_PREC_FP8) a_scale = 127 + sm.sexp[buf][sub * 32 + ql];
#pragma unroll
            for (int b = 0; b < QB; ++b) {
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[b][i] = nv[i >> 2][i & 3];
            }
            for (int b = 0; b < QB; ++b)
                acc[b] = mfma_tile<P, NSTEP, GMAX>(arow, qf[b], acc[b], a_scale, q_scale[b]);
        }
    };

    // selection of a computed subtile (INT8 sums become FP32 keys here, after
    // the next subtile's MFMAs have been issued)
    auto select = [&](Acc (&acc)[QB], int buf, int sub, int64_t cb, const int32_t* tp) {
        if constexpr (P == SG_PREC_I8) {
            // reject the subtile when even the bound -2 max(acc) (IP: -max)
            // of every lane exceeds its threshold (max(acc) < amin); else
            // form exact keys
            const int qm = (int)A.qmul;
            bool any = false;
#pragma unroll
            for (int b = 0; b < QB; ++b) any |= max16(acc[b]) >= sel.amin[b];
            if (!__builtin_amdgcn_ballot_w64(any)) return;
            intx4 par[4] = {};
            if (qm == -2) {
#pragma unroll
                for (int g = 0; g < 4; ++g)
                    par[g] = *reinterpret_cast<const intx4*>(&sm.par[buf][sub * 32 + g * 8 + h * 4]);
            }
            floatx16 kf[QB];
#pragma unroll
            for (int b = 0; b < QB; ++b) kf[b] = i8_keys(acc[b], par, qm);
            sel.admit(kf, cb, tp);
        } else {
            sel.admit(acc, cb, tp);
        }
    };
    auto body = [&](int t, int buf) {
        const int j0 = tile_row(t);
        const int32_t* tp = A.cpid ? sm.pid[buf] : nullptr;
        Acc accA[QB], accB[QB];
        compute(accA, buf, 0);
#pragma unroll
        for (int sub = 0; sub < NSUB; ++sub) {
            if (sub % 2 == 0) {
                if (sub + 1 < NSUB) compute(accB, buf, sub + 1);
                select(accA, buf, sub, j0 + sub * 32, tp ? tp + sub * 32 : nullptr);
            } else {
                if (sub + 1 < NSUB) compute(accA, buf, sub + 1);
                select(accB, buf, sub, j0 + sub * 32, tp ? tp + sub * 32 : nullptr);
            }
        }
    };
    if constexpr (DEPTH == 2) {
        // tile t sits in LDS buffer t % 2 and register set t % 2; the loop
        // takes tiles in pairs so that both indices are compile-time constants
        prefetch(0, tile_row(0));
        if (ntiles > 1) prefetch(1, tile_row(1));
        commit(0, 0);
        __syncthreads();
        if (ntiles > 2) prefetch(0, tile_row(2));
        for (int t = 0; t < ntiles; t += 2) {
            body(t, 0);
            if (t + 1 < ntiles) {
                commit(1, 1);
                if (t + 3 < ntiles) prefetch(1, tile_row(t + 3));
            }
            __syncthreads();
            if (t + 1 >= ntiles) break;
            body(t + 1, 1);
            if (t + 2 < ntiles) {
                commit(0, 0);
                if (t + 4 < ntiles) prefetch(0, tile_row(t + 4));
            }
            __syncthreads();
        }
    } else {
        prefetch(0, tile_row(0));
        commit(0, 0);
        __syncthreads();
        if (ntiles > 1) prefetch(0, tile_row(1));
        for (int t = 0; t < ntiles; ++t) {
            const int buf = t & 1;
            body(t, buf);
            if (t + 1 < ntiles) {
                commit(0, buf ^ 1);
                if (t + 2 < ntiles) prefetch(0, tile_row(t + 2));
            }
            __syncthreads();
        }
    }
    sel.drain();
    if (A.nbr) write_lists(A, KSEL, qblk0, 32 * QB);
    __syncthreads();   // LDS is reused by the next block of a persistent workgroup
}

// Workgroups per CU a launch shape aims for: 32-row tiles keep the LDS of a
// 4-wave workgroup with 32-entry buffers near 50 KB, so three fit (12 waves;
// at most 168 VGPRs); with shorter buffers (cbq_four_wgs) four fit (16 waves;
// 128 VGPRs).
constexpr int min_waves_per_simd(int waves, int bcr, int cbq = CB) {
    return waves == 4 && bcr == 32 ? (cbq < 32 ? 4 : 3) : 1;
}

// Buffer entries per query of the 4-wave, 32-row-tile shape that runs four
// workgroups per CU: the longest of 30, 28, 24, 20 whose LDS lets four share a
// CU's 160 KB, else 16.  Longer buffers mean fewer merges (for 128-byte rows
// 28 entries took the INT8 batched build from 59.8 to 53.9 ms against the
// 32-entry, three-workgroup shape, and 30 entries (40 728 bytes) 1.5% more).
template <int P, int NSTEP>
constexpr int cbq_four_wgs() {
    constexpr size_t cap = 160 * 1024 / 4;
    return sizeof(TopkSmem<P, NSTEP, 4, 1, 30, 32>) <= cap   ? 30
           : sizeof(TopkSmem<P, NSTEP, 4, 1, 28, 32>) <= cap ? 28
           : sizeof(TopkSmem<P, NSTEP, 4, 1, 24, 32>) <= cap ? 24
           : sizeof(TopkSmem<P, NSTEP, 4, 1, 20, 32>) <= cap ? 20
                                                             : 16;
}

// One query block per workgroup (blockIdx.x).
template <int P, int NSTEP, int KSEL, int WAVES, int QB, int CBQ, int BCR>
__global__ __launch_bounds__(WAVES * 64, min_waves_per_simd(WAVES, BCR, CBQ)) void dist_topk_kernel(TopkArgs A) {
    __shared__ TopkSmem<P, NSTEP, WAVES, QB, CBQ, BCR> sm;
    topk_block<P, NSTEP, KSEL, WAVES, QB, CBQ, BCR>(sm, blockIdx.x, A);
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
__global__ __launch_bounds__(KS_WAVES * 64, 1) void dist_topk_kstream_kernel(TopkArgs A, int DP) {
    const float* __restrict__ ops = reinterpret_cast<const float*>(A.ops);
    const float* __restrict__ ninit = A.ninit;
    const int n = A.n;
    const float* __restrict__ qops = reinterpret_cast<const float*>(A.qops);
    const int64_t* __restrict__ qid = A.qid;
    const int nq = A.nq;
    const float qmul = A.qmul;
    uint64_t* __restrict__ state = A.state;
    constexpr int NT = KS_WAVES * 64;
    constexpr int CPR = KS_DC / 4;                       // 16-byte chunks per row per k-chunk
    constexpr int CPT = (KS_NQ + KS_BC) * CPR / NT;      // per thread per k-chunk
    __shared__ __align__(16) float s_q[2][KS_NQ * KS_RS];
    __shared__ __align__(16) float s_c[2][KS_BC * KS_RS];
    __shared__ __align__(16) float s_norm[KS_BC];
    __shared__ uint64_t s_buf[KS_NQ * CB];

    const int tid = threadIdx.x;
    const int l = tid & 63;
    const int w = tid >> 6;
    const int h = l >> 5;
    const int ql = l & 31;
    const int64_t qb0 = (int64_t)blockIdx.x * KS_NQ;
    const int64_t qblk0 = qb0 + w * 32;

    Selector<KSEL, 1> sel;
    sel.state = state + qblk0 * KSEL;
    sel.buf = s_buf + w * 32 * CB;
    {
        const int64_t qg = qblk0 + ql;
        sel.thr[0] = __builtin_inff();
        sel.fill[0] = 0;
        sel.fresh[0] = 0;   // this kernel's workspace lists are initialised by the caller
        sel.qself[0] = qg < nq ? (qid ? qid[qg] : qg) : -1;
    }
    sel.qm_int = 0;
    sel.init_self_range();

    const int nch = DP / KS_DC;
    const int ntiles = (n + KS_BC - 1) / KS_BC;
    const int64_t total = (int64_t)ntiles * nch;
    const ScanOrder order(qb0, KS_BC, ntiles);
    intx4 pre[CPT];
    float pre_norm = 0.f;
    auto prefetch = [&](int64_t g) {
        const int t = order.tile((int)(g / nch)), kc = (int)(g % nch);
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
        const int t = order.tile((int)(g / nch)), kc = (int)(g % nch);
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
                const int64_t cb = (int64_t)t * KS_BC + sub * 32;
                sel.admit(one, cb, A.cpid ? A.cpid + cb : nullptr);
            }
        }
        if (g + 1 < total) {
            commit(g + 1, buf ^ 1);
            if (g + 2 < total) prefetch(g + 2);
        }
        __syncthreads();
    }
    sel.drain();
    if (A.nbr) write_lists(A, KSEL, qblk0, 32);
}

// Nearest candidate of every query row by (key, index): the pivot
// assignment of the locality order.  One wave per 32 register-resident
// queries; candidate tiles of 32 rows pass through LDS; each lane keeps its
// best in registers and the two lanes of a query combine at the end.  No
// self exclusion.  label[q] = label_base + index of the nearest candidate (0
// if none).  blk: the block of WAVES*32 query rows.
template <int P, int NSTEP, int WAVES>
__device__ void nearest_block(int64_t blk, const uint8_t* __restrict__ ops, const float* __restrict__ ninit,
                              const int32_t* __restrict__ sexp, int n, const uint8_t* __restrict__ qops,
                              const int32_t* __restrict__ qsexp, int nq, float qmul, int32_t* __restrict__ label,
                              int32_t label_base) {
    using S = Shape<P, NSTEP, 32>;
    constexpr int RB = S::ROW_BYTES, RS = S::RS, BC = 32;
    constexpr int NT = WAVES * 64;
    constexpr int CHUNKS = BC * RB / 16;
    __shared__ __align__(16) uint8_t tile[BC * RS];
    __shared__ __align__(16) float norm[BC];
    __shared__ int32_t tsexp[BC];
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6, h = l >> 5, ql = l & 31;
    const int64_t qg = (blk * WAVES + w) * 32 + ql;
    Frag<P, NSTEP> qf;
    load_frag<P, NSTEP>(qf, qops + qg * RB + h * (RB / 2));
    scale_query<P, NSTEP>(qf, qmul);
    const int q_scale = P == SG_PREC_FP8 ? 127 + qsexp[qg] + 1 : 127;
    float best = __builtin_inff();
    int32_t bid = INT32_MAX;
    for (int j0 = 0; j0 < n; j0 += BC) {
        __syncthreads();
        for (int c = tid; c < CHUNKS; c += NT) {
            const int r = c / (RB / 16), o = c % (RB / 16);
            *reinterpret_cast<intx4*>(&tile[r * RS + o * 16]) =
                *reinterpret_cast<const intx4*>(ops + (int64_t)(j0 + r) * RB + o * 16);
        }
        if (tid < BC) {
            norm[tid] = ninit[j0 + tid];
            if constexpr (P == SG_PREC_FP8) tsexp[tid] = sexp[j0 + tid];
        }
        __syncthreads();
        floatx16 acc;
        if constexpr (P == SG_PREC_I8) {
            intx16 ai;
            intx4 par[4];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int32_t e = __builtin_bit_cast(int32_t, norm[out_row(i, l)]);
                ai[i] = e >> 1;
                par[i >> 2][i & 3] = e & 1;
            }
            ai = mfma_tile_i8<NSTEP>(&tile[ql * RS + h * (RB / 2)], qf, ai);
            acc = i8_keys(ai, par, (int)qmul);
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[i] = norm[out_row(i, l)];
            const int a_scale = P == SG_PREC_FP8 ? 127 + tsexp[ql] : 127;
            acc = mfma_tile<P, NSTEP>(&tile[ql * RS + h * (RB / 2)], qf, acc, a_scale, q_scale);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int32_t r = j0 + out_row(i, l);
            if (acc[i] < best || (acc[i] == best && r < bid)) {
                best = acc[i];
                bid = r;
            }
        }
    }
    const float ob = __builtin_bit_cast(float, lane_xor(__builtin_bit_cast(uint32_t, best), 32));
    const int32_t oid = (int32_t)lane_xor((uint32_t)bid, 32);
    if (ob < best || (ob == best && oid < bid)) bid = oid;
    if (h == 0 && qg < nq) label[qg] = label_base + (bid < n ? bid : 0);
}

template <int P, int NSTEP, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void nearest_kernel(const uint8_t* __restrict__ ops,
                                                             const float* __restrict__ ninit,
                                                             const int32_t* __restrict__ sexp, int n,
                                                             const uint8_t* __restrict__ qops,
                                                             const int32_t* __restrict__ qsexp, int nq,
                                                             float qmul, int32_t* __restrict__ label) {
    nearest_block<P, NSTEP, WAVES>(blockIdx.x, ops, ninit, sexp, n, qops, qsexp, nq, qmul, label, 0);
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
                    const int e = p * 64 + l;
                    v[p] = cmpx(v[p], j, ((e & k) == 0) == ((l & j) == 0));
                }
            }
        }
    }
}

__device__ inline int32_t cand_id(uint64_t key) { return key_id(key); }
__device__ inline int32_t cand_id(int32_t id) { return id; }

// Sort the candidate keys of row i (element p*64 + l in lane l of v[p]),
// drop repeated ids, write the best k to output row o (SG_NONE / +inf pad;
// nothing for o < 0).
template <int PER>
__device__ void rerank_finish(uint64_t (&v)[PER], int64_t o, int k, int32_t* __restrict__ nbr,
                              float* __restrict__ dist) {
    if (o < 0) return;   // a padding slot of a batched layout (wave-uniform)
    const int l = lane_id();
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
            nbr[o * k + pos] = key_id(v[p]);
            if (dist) dist[o * k + pos] = key_dist(v[p]);
        }
        kept += __builtin_popcountll(m);
    }
    for (int e = kept + l; e < k; e += 64) {
        nbr[o * k + e] = SG_NONE;
        if (dist) dist[o * k + e] = __builtin_inff();
    }
}

template <int PER, typename CT = uint64_t>
__global__ __launch_bounds__(256) void rerank_kernel(const void* __restrict__ X, int dtype, int64_t n,
                                                     int d, int64_t ld, int metric,
                                                     const int64_t* __restrict__ rowmap,
                                                     int64_t n_src, const CT* __restrict__ cand,
                                                     int kstate,
                                                     int c, int k, int32_t* __restrict__ nbr,
                                                     float* __restrict__ dist,
                                                     const int64_t* __restrict__ orow) {
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
    rerank_finish<PER>(v, orow ? orow[i] : i, k, nbr, dist);
}

// Re-rank for wide rows (d > 128): one wave per query row; each candidate row
// is read with coalesced loads (lane l takes elements 4l..4l+3 of every
// 256-element chunk), each lane sums its elements in ascending order and the
// 64 partial sums are combined by a fixed butterfly, so the distance is
// deterministic.  Four candidates are in flight at a time.
template <int PER, typename CT, bool F32V>
__global__ __launch_bounds__(256) void rerank_wide_kernel(const void* __restrict__ X, int dtype, int64_t n, int d,
                                                          int64_t ld, int metric, const int64_t* __restrict__ rowmap,
                                                          int64_t n_src, const CT* __restrict__ cand, int kstate,
                                                          int c, int k, int32_t* __restrict__ nbr,
                                                          float* __restrict__ dist, const int64_t* __restrict__ orow) {
    constexpr int UMAX = 4;   // d <= 1024
    const int l = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const int U = (d + 255) / 256;
    int64_t self = rowmap ? rowmap[i] : i;
    const bool have_q = self >= 0 && self < n_src;
    auto load4 = [&](int64_t row, int u) {
        floatx4 r = {0.f, 0.f, 0.f, 0.f};
        const int t = u * 256 + 4 * l;
        if (F32V) {
            if (t < d) r = *reinterpret_cast<const floatx4*>(static_cast<const float*>(X) + row * ld + t);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (t + e < d) r[e] = load_elem(X, dtype, row * ld + t + e);
        }
        return r;
    };
    floatx4 q[UMAX];
#pragma unroll
    for (int u = 0; u < UMAX; ++u) q[u] = (u < U && have_q) ? load4(self, u) : floatx4{0.f, 0.f, 0.f, 0.f};
    uint64_t v[PER];
#pragma unroll
    for (int p = 0; p < PER; ++p) v[p] = EMPTY_KEY;
    for (int e0 = 0; e0 < c; e0 += 4) {
        int32_t j[4];
        bool ok[4];
        floatx4 x[4][UMAX];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int e = e0 + a;
            const int32_t jj = e < c ? cand_id(cand[i * kstate + e]) : SG_NONE;
            j[a] = __builtin_amdgcn_readfirstlane(jj);
            ok[a] = j[a] >= 0 && j[a] < n_src && j[a] != self;
#pragma unroll
            for (int u = 0; u < UMAX; ++u)
                x[a][u] = (u < U && ok[a]) ? load4(j[a], u) : floatx4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            float sum = 0.f;
#pragma unroll
            for (int u = 0; u < UMAX; ++u) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (metric == SG_L2) {
                        const float df = q[u][e] - x[a][u][e];
                        sum = fmaf(df, df, sum);
                    } else {
                        sum = fmaf(q[u][e], x[a][u][e], sum);
                    }
                }
            }
#pragma unroll
            for (int m = 32; m > 0; m >>= 1)
                sum += __builtin_bit_cast(float, lane_xor(__builtin_bit_cast(uint32_t, sum), m));
            if (metric != SG_L2) sum = -sum;
            const int e = e0 + a;
            const uint64_t key = ok[a] ? make_key(sum, j[a]) : EMPTY_KEY;
#pragma unroll
            for (int p = 0; p < PER; ++p)
                if (e < c && (e >> 6) == p && l == (e & 63)) v[p] = key;
        }
    }
    rerank_finish<PER>(v, orow ? orow[i] : i, k, nbr, dist);
}

// Launch the re-rank of n rows (rerank kernel by width and candidate count).
template <typename CT>
inline void launch_rerank(const void* X, int dtype, int64_t n, int d, int64_t ld, int metric, const int64_t* rowmap,
                          int64_t n_src, const CT* cand, int kstate, int c, int k, int32_t* nbr, float* dist,
                          const int64_t* orow, hipStream_t s) {
    const unsigned grid = (unsigned)cdiv(n, 4);
    if (d > 128) {
        const bool vec = dtype == SG_F32 && d % 4 == 0 && ld % 4 == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0;
#define SG_WIDE(PER)                                                                                                  \
        do {                                                                                                          \
            if (vec)                                                                                                  \
                rerank_wide_kernel<PER, CT, true><<<grid, 256, 0, s>>>(X, dtype, n, d, ld, metric, rowmap, n_src,     \
                                                                        cand, kstate, c, k, nbr, dist, orow);        \
            else                                                                                                      \
                rerank_wide_kernel<PER, CT, false><<<grid, 256, 0, s>>>(X, dtype, n, d, ld, metric, rowmap, n_src,    \
                                                                         cand, kstate, c, k, nbr, dist, orow);       \
        } while (0)
        if (c <= 64) SG_WIDE(1);
        else if (c <= 128) SG_WIDE(2);
        else SG_WIDE(4);
#undef SG_WIDE
    } else {
        const size_t shm = (size_t)4 * d * sizeof(float);
        if (c <= 64)
            rerank_kernel<1, CT><<<grid, 256, shm, s>>>(X, dtype, n, d, ld, metric, rowmap, n_src, cand, kstate, c, k,
                                                        nbr, dist, orow);
        else if (c <= 128)
            rerank_kernel<2, CT><<<grid, 256, shm, s>>>(X, dtype, n, d, ld, metric, rowmap, n_src, cand, kstate, c, k,
                                                        nbr, dist, orow);
        else
            rerank_kernel<4, CT><<<grid, 256, shm, s>>>(X, dtype, n, d, ld, metric, rowmap, n_src, cand, kstate, c, k,
                                                        nbr, dist, orow);
    }
    SG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
inline int ksel_for(int k) { return k <= 32 ? 32 : k <= 64 ? 64 : k <= 128 ? 128 : 256; }

// Largest resident query half-row supported: the query fragment of 32 rows
// lives in 64 VGPRs per lane at most.
inline int nstep_for(int prec, int DP) {
    int vec = prec == SG_PREC_FP32 ? 1 : prec == SG_PREC_FP8 ? 32 : prec == SG_PREC_I8 ? 16 : 8;
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

typedef void (*topk_fn)(TopkArgs);
typedef void (*near_fn)(const uint8_t*, const float*, const int32_t*, int, const uint8_t*, const int32_t*, int,
                        float, int32_t*);
constexpr int NEAR_WAVES = 4;
typedef void (*kstream_fn)(TopkArgs, int);

// A distance kernel and its launch geometry.
struct Kern {
    topk_fn fn = nullptr;         // resident-query kernel, or
    kstream_fn ks = nullptr;      // k-streamed FP32 kernel
    int DP = 0;                   // padded operand row length it expects
    int nq_block = 0;             // queries per workgroup
    int threads = 0;
    int tile_rows = 0;            // candidate rows per LDS tile (0: k-streamed)
    near_fn near = nullptr;       // nearest-candidate kernel on the same operands
};

template <int P, int NSTEP, int W, int QB, int CBQ, int BCR, int KSEL>
Kern resident() {
    Kern k;
    k.fn = dist_topk_kernel<P, NSTEP, KSEL, W, QB, CBQ, BCR>;
    k.DP = 2 * NSTEP * Tr<P>::VEC;
    k.nq_block = 32 * W * QB;
    k.threads = 64 * W;
    k.tile_rows = Shape<P, NSTEP, BCR>::BC;
    k.near = nearest_kernel<P, NSTEP, NEAR_WAVES>;
    return k;
}

// The launch shapes of a precision and padded row length, default first:
// m.template add<P, NSTEP, WAVES, QB, CBQ, BCR>() is called once per shape in
// a fixed order, so that the single-shard and the batched drivers (and the
// recorded autotuning choice, an index into this order) agree.  Resident-query
// kernels exist for the half-row lengths below (8 waves while the query
// fragment fits two waves per SIMD, 4 waves beyond); a smaller d pads up to
// the next one.  Short rows also get 4-wave shapes with 64-row tiles (two
// workgroups per CU) or 32-row tiles (three per CU), so that other workgroups
// keep the MFMA and VALU units busy while one waits at its tile barrier or on
// a merge.  Returns false if no resident kernel serves the row length (FP32
// rows wider than 128 use the k-streamed kernel).
// Each precision's table is instantiated in a translation unit of its own
// (shapes_*.hip), one per selection width, so that the kernels compile in
// parallel; the definition is in shapes.hpp.
template <int PR, class M>
bool for_shapes_p(int d, M& m);

template <class M>
bool for_shapes(int prec, int d, M& m) {
    switch (prec) {
        case SG_PREC_FP32: return for_shapes_p<SG_PREC_FP32>(d, m);
        case SG_PREC_F16: return for_shapes_p<SG_PREC_F16>(d, m);
        case SG_PREC_BF16: return for_shapes_p<SG_PREC_BF16>(d, m);
        case SG_PREC_I8: return for_shapes_p<SG_PREC_I8>(d, m);
        default: return for_shapes_p<SG_PREC_FP8>(d, m);
    }
}

template <int KSEL>
struct ResidentMaker {
    std::vector<Kern> v;
    template <int P, int NSTEP, int W, int QB, int CBQ, int BCR>
    void add() { v.push_back(resident<P, NSTEP, W, QB, CBQ, BCR, KSEL>()); }
};

// Every table slice is instantiated explicitly in its own translation unit;
// these declarations keep the other units (and each slice, for the other
// slices) from instantiating them implicitly.
#define SG_EXTERN_SLICE(PR, MAKER) extern template bool for_shapes_p<PR, MAKER>(int, MAKER&);
#define SG_EXTERN_SLICES(MAKER_T, K)                  \
    SG_EXTERN_SLICE(SG_PREC_FP32, MAKER_T<K>)         \
    SG_EXTERN_SLICE(SG_PREC_F16, MAKER_T<K>)          \
    SG_EXTERN_SLICE(SG_PREC_BF16, MAKER_T<K>)         \
    SG_EXTERN_SLICE(SG_PREC_FP8, MAKER_T<K>)          \
    SG_EXTERN_SLICE(SG_PREC_I8, MAKER_T<K>)
SG_EXTERN_SLICES(ResidentMaker, 32)
SG_EXTERN_SLICES(ResidentMaker, 64)
SG_EXTERN_SLICES(ResidentMaker, 128)
SG_EXTERN_SLICES(ResidentMaker, 256)

inline Kern kstream_kernel(int d, int ksel) {
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

// Every distance kernel for (prec, d, ksel), default first (empty if none).
inline std::vector<Kern> kernel_variants(int prec, int d, int ksel) {
    bool ok = false;
    std::vector<Kern> v;
    switch (ksel) {
        case 32: { ResidentMaker<32> m; ok = for_shapes(prec, d, m); v = m.v; break; }
        case 64: { ResidentMaker<64> m; ok = for_shapes(prec, d, m); v = m.v; break; }
        case 128: { ResidentMaker<128> m; ok = for_shapes(prec, d, m); v = m.v; break; }
        default: { ResidentMaker<256> m; ok = for_shapes(prec, d, m); v = m.v; break; }
    }
    if (ok) return v;
    if (prec == SG_PREC_FP32 && d <= 1024) return {kstream_kernel(d, ksel)};
    return {};
}

inline Kern pick_kernel(int prec, int d, int ksel) {
    const std::vector<Kern> v = kernel_variants(prec, d, ksel);
    return v.empty() ? Kern() : v[0];
}

// Process-wide record of the fastest launch shape per (precision, padded row
// length, K selection width, power-of-two bucket of n), filled by
// sg_knn_autotune; a per-thread override serves tests.  Defined in knn.hip.
struct TuneKey {
    int prec, DP, ksel, nlog;
    bool operator<(const TuneKey& o) const {
        return std::tie(prec, DP, ksel, nlog) < std::tie(o.prec, o.DP, o.ksel, o.nlog);
    }
};
extern std::mutex g_tune_mu;
extern std::map<TuneKey, int> g_tune;
extern thread_local int g_force_variant;

inline int nlog_of(int64_t n) {
    int b = 0;
    while ((int64_t(1) << (b + 1)) <= n) ++b;
    return b;
}

inline TuneKey tune_key(int prec, int d, int ksel, int64_t n) {
    return TuneKey{prec, padded_d(prec, d), ksel, nlog_of(n)};
}

// The record of a batched pass whose largest shard has n_max rows (kept apart
// from the single-shard records: the persistent launch of many shards can
// prefer another shape than one launch of its largest shard).
inline TuneKey batched_tune_key(int prec, int d, int ksel, int64_t n_max) {
    return TuneKey{prec, padded_d(prec, d), ksel, 64 + nlog_of(n_max)};
}

// Index into the shape table for a call of this shape (count entries).
int chosen_variant(int prec, int d, int ksel, int64_t n, int count);

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

inline void check_args(const void* X, int dtype, int64_t n, int d, int64_t ld, int metric, int k, int prec,
                int rerank) {
    SG_REQUIRE(n >= 0 && n <= MAX_ROWS, "n out of range (at most 2^26 - 1024 rows)");
    SG_REQUIRE(d >= 1 && d <= 1024, "d must be in 1..1024");
    SG_REQUIRE(ld >= d, "ld must be >= d");
    SG_REQUIRE(k >= 1 && k <= 256, "k must be in 1..256");
    SG_REQUIRE(metric == SG_L2 || metric == SG_IP, "unknown metric");
    SG_REQUIRE(dtype >= SG_F32 && dtype <= SG_U8, "unknown dtype");
    SG_REQUIRE(prec >= SG_PREC_FP32 && prec <= SG_PREC_I8, "unknown precision");
    SG_REQUIRE(rerank == 0 || (rerank >= k && rerank <= 256), "rerank must be 0 or in k..256");
    SG_REQUIRE(!(prec == SG_PREC_I8 && dtype != SG_U8), "SG_PREC_I8 needs U8 input");
    SG_REQUIRE(!(prec == SG_PREC_I8 && d > 256), "SG_PREC_I8 is exact on U8 input only for d <= 256");
    SG_REQUIRE(!(prec == SG_PREC_F16 && dtype != SG_F16 && dtype != SG_U8),
               "SG_PREC_F16 needs F16 or U8 input");
    SG_REQUIRE(!(prec == SG_PREC_F16 && dtype == SG_U8 && d > 128),
               "SG_PREC_F16 is exact on U8 input only for d <= 128");
    SG_REQUIRE(n == 0 || X != nullptr, "X is NULL");
}


inline int64_t pad_rows(int64_t m) { return (m + PAD_ROWS - 1) / PAD_ROWS * PAD_ROWS; }

// Locality order of a whole-shard build: rows are grouped by their nearest
// of P evenly spaced pivot rows (about 256 rows per pivot), so that a
// workgroup's queries and the candidates it scans first are close together.
// (Register-resident kernels only; the k-streamed FP32 kernel keeps the input
// order.)
constexpr int64_t LOCAL_MIN_ROWS = 4096;   // smaller shards keep their order
inline int64_t n_pivots(int64_t n) { return std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 8192); }
inline bool use_locality(int64_t n, bool subset) { return !subset && n >= LOCAL_MIN_ROWS; }

// Extra workspace of the locality order.
inline size_t locality_bytes(const Layout& L, int64_t n, int prec) {
    const int64_t P = n_pivots(n), Pp = pad_rows(P);
    return align_up((size_t)L.n_pad * 8, 256) + 2 * align_up((size_t)L.n_pad * 4, 256) +
           align_up(label_sort_tmp_bytes(n, bits_for(P)), 256) +
           align_up((size_t)Pp * L.DP * elem_bytes(prec), 256) + 3 * align_up((size_t)Pp * 4, 256) +
           align_up((size_t)P * 8, 256);
}

// Workspace of one call: candidate operands + side arrays for all n rows,
// and, for a row subset, the query operands + side arrays of its nq rows.
inline size_t total_bytes(const Layout& L, int64_t n, int64_t nq, int prec) {
    size_t t = L.total;
    if (nq >= 0) {
        const int64_t nqp = pad_rows(nq);
        t += align_up((size_t)nqp * L.DP * elem_bytes(prec), 256) + 2 * align_up((size_t)nqp * 4, 256) +
             align_up((size_t)nqp * 4, 256) + align_up((size_t)nqp * 8, 256);
        // the state then covers the query rows only
        t -= align_up(L.state_bytes, 256);
        t += align_up((size_t)nqp * L.ksel * 8, 256);
    } else if (use_locality(n, false)) {
        t += locality_bytes(L, n, prec);
    }
    return t;
}

static __global__ void iota32_kernel(int32_t* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

static __global__ void pivot_rows_kernel(int64_t* __restrict__ piv, int64_t P, int64_t n) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) piv[p] = p * n / P;
}

// The locality order as operand-row maps: position p < n holds row rows[p]
// (perm as int64, pid as int32 candidate id); padding positions get -1.
static __global__ void rows_to_perm_kernel(const int32_t* __restrict__ rows, int64_t n, int64_t n_pad,
                                           int64_t* __restrict__ perm, int32_t* __restrict__ pid) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pad;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = i < n ? rows[i] : -1;
        perm[i] = r;
        if (i >= n) pid[i] = -1;
    }
}

inline void launch_topk(const Kern& kern, const TopkArgs& A, int64_t nq_pad, int DP, hipStream_t s) {
    const unsigned grid = (unsigned)(nq_pad / kern.nq_block);
    if (kern.fn)
        kern.fn<<<grid, kern.threads, 0, s>>>(A);
    else
        kern.ks<<<grid, kern.threads, 0, s>>>(A, DP);
    SG_LAUNCH_CHECK();
}

}  // namespace knn
}  // namespace sg

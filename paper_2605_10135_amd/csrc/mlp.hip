// mlp.hip -- the learned candidate proposer: a small MLP trained and run on
// the GPU by this library's own kernels.
//
//   z = (x - mu) / sigma,  h1 = W1 z + b1,  a1 = GELU(h1) (erf form),
//   h2 = W2 a1 + b2,       f = h2 / ||h2||
//
// Training minimises the in-batch softmax cross-entropy of the logits
// l_ij = f(a_i) . f(p_j) / T (anchor i, positive j; target j = i), with Adam
// on FP32 master weights; the layer products use BF16 operands on MFMA with
// FP32 accumulation, the (small, temperature-scaled) logit products use FP32
// MFMA.  One training step is a fixed sequence of kernels whose batch is read
// from device arrays indexed by a device step counter, so a whole step can be
// captured once in a hipGraph and replayed.
#include <cmath>

#include "common.hpp"

namespace sg {
namespace mlp {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// strided GEMM: C[m][n] = alpha * sum_k A(m,k) B(k,n) + beta * C[m][n]
//   A(m,k) = A[m*sam + k*sak],  B(k,n) = B[k*sbk + n*sbn]   (FP32 in memory)
// Operands are rounded to BF16 (BF16 = true) or kept FP32 in LDS.  64 x 64
// output tile per 256-thread workgroup, 32 x 32 per wave, k in chunks of 32.
// ---------------------------------------------------------------------------
constexpr int GT = 64, GK = 32, GPAD = 4;

__device__ inline float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * __expf(-0.5f * x * x);
}

template <bool BF16>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K, float alpha,
                                                   const float* __restrict__ A, int64_t sam, int64_t sak,
                                                   const float* __restrict__ B, int64_t sbk, int64_t sbn,
                                                   float beta, float* __restrict__ C, int64_t ldc) {
    __shared__ __align__(16) float As[GT][GK + GPAD];   // (m, k)
    __shared__ __align__(16) float Bs[GT][GK + GPAD];   // (n, k)
    const int tid = threadIdx.x;
    const int l = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    floatx16 acc = {0};
    for (int k0 = 0; k0 < K; k0 += GK) {
        for (int e = tid; e < GT * GK; e += 256) {
            const int r = e / GK, c = e % GK;
            const int m = m0 + r, k = k0 + c;
            float a = (m < M && k < K) ? A[m * sam + k * sak] : 0.f;
            const int nn = n0 + r;
            float b = (nn < N && k < K) ? B[k * sbk + nn * sbn] : 0.f;
            if (BF16) {
                a = (float)(__bf16)a;
                b = (float)(__bf16)b;
            }
            As[r][c] = a;
            Bs[r][c] = b;
        }
        __syncthreads();
        const int h = l >> 5;
        const float* ar = &As[wm * 32 + (l & 31)][0];
        const float* br = &Bs[wn * 32 + (l & 31)][0];
        if (BF16) {
#pragma unroll
            for (int s = 0; s < GK / 16; ++s) {
                bf16x8 av, bv;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    av[e] = (__bf16)ar[s * 16 + h * 8 + e];
                    bv[e] = (__bf16)br[s * 16 + h * 8 + e];
                }
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int s = 0; s < GK / 2; ++s)
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[s * 2 + h], br[s * 2 + h], acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // D[i][j]: i = row (m), j = col (n); lane holds col l%32, rows 8(r/4) + 4(l/32) + r%4
    const int n = n0 + wn * 32 + (l & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm * 32 + ((r >> 2) << 3) + ((l >> 5) << 2) + (r & 3);
        if (m < M && n < N) {
            float v = alpha * acc[r];
            if (beta != 0.f) v += beta * C[m * ldc + n];
            C[m * ldc + n] = v;
        }
    }
}

template <bool BF16>
void gemm(int M, int N, int K, float alpha, const float* A, int64_t sam, int64_t sak, const float* B,
          int64_t sbk, int64_t sbn, float beta, float* C, int64_t ldc, hipStream_t s) {
    dim3 grid((unsigned)cdiv(N, GT), (unsigned)cdiv(M, GT));
    gemm_kernel<BF16><<<grid, 256, 0, s>>>(M, N, K, alpha, A, sam, sak, B, sbk, sbn, beta, C, ldc);
    SG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// elementwise / row kernels
// ---------------------------------------------------------------------------

// Z[r] = (X[rows[r]] - mu) / sigma for r < nrows (rows read from a device list)
__global__ void zscore_kernel(const float* __restrict__ X, int64_t ld, int D, const int64_t* __restrict__ rows,
                              int64_t nrows, const float* __restrict__ mu, const float* __restrict__ sigma,
                              float* __restrict__ Z) {
    const float inv = 1.0f / sigma[0];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nrows * D;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / D;
        const int t = (int)(e - r * D);
        Z[e] = (X[rows[r] * ld + t] - mu[t]) * inv;
    }
}

// H += bias (row broadcast); A = GELU(H)
__global__ void bias_gelu_kernel(float* __restrict__ H, const float* __restrict__ bias, int64_t rows, int cols,
                                 float* __restrict__ Aout) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < rows * cols;
         e += (int64_t)gridDim.x * blockDim.x) {
        const float v = H[e] + bias[e % cols];
        H[e] = v;
        Aout[e] = gelu(v);
    }
}

// one wave per row: H += bias; nrm = ||H||; F = H / nrm
__global__ void bias_norm_kernel(float* __restrict__ H, const float* __restrict__ bias, int64_t rows, int cols,
                                 float* __restrict__ F, float* __restrict__ nrm) {
    const int l = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (r >= rows) return;
    float ss = 0.f;
    for (int c = l; c < cols; c += 64) {
        const float v = H[r * cols + c] + bias[c];
        H[r * cols + c] = v;
        ss += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o, 64);
    const float nv = sqrtf(ss);
    for (int c = l; c < cols; c += 64) F[r * cols + c] = H[r * cols + c] / nv;
    if (l == 0) nrm[r] = nv;
}

// one wave per logit row: G[i][j] = (softmax_j(L[i]) - [i == j]) / B, loss_i
__global__ void softmax_ce_kernel(const float* __restrict__ Lg, int B, float* __restrict__ G,
                                  float* __restrict__ loss_rows) {
    const int l = threadIdx.x & 63;
    const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (i >= B) return;
    const float* row = Lg + (int64_t)i * B;
    float mx = -__builtin_inff();
    for (int j = l; j < B; j += 64) mx = fmaxf(mx, row[j]);
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    float se = 0.f;
    for (int j = l; j < B; j += 64) se += __expf(row[j] - mx);
    for (int o = 32; o > 0; o >>= 1) se += __shfl_xor(se, o, 64);
    const float lse = mx + __logf(se);
    for (int j = l; j < B; j += 64) {
        const float p = __expf(row[j] - lse);
        G[(int64_t)i * B + j] = (p - (i == j ? 1.f : 0.f)) / (float)B;
    }
    if (l == 0) loss_rows[i] = lse - row[i];
}

// one wave per row: dH = (dF - F (F . dF)) / nrm   (in place over dF)
__global__ void norm_bwd_kernel(const float* __restrict__ F, const float* __restrict__ nrm, int64_t rows, int cols,
                                float* __restrict__ dF) {
    const int l = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (r >= rows) return;
    float dot = 0.f;
    for (int c = l; c < cols; c += 64) dot += F[r * cols + c] * dF[r * cols + c];
    for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o, 64);
    const float inv = 1.0f / nrm[r];
    for (int c = l; c < cols; c += 64) dF[r * cols + c] = (dF[r * cols + c] - F[r * cols + c] * dot) * inv;
}

// dA *= GELU'(H)
__global__ void gelu_bwd_kernel(const float* __restrict__ H, int64_t n, float* __restrict__ dA) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        dA[e] *= gelu_grad(H[e]);
}

// out[c] = sum_r M[r][c], rows summed in order (one thread per column)
__global__ void colsum_kernel(const float* __restrict__ Mx, int64_t rows, int cols, float* __restrict__ out) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < cols; c += gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int64_t r = 0; r < rows; ++r) s += Mx[r * cols + c];
        out[c] = s;
    }
}

__global__ void sum_kernel(const float* __restrict__ v, int n, float scale, float* __restrict__ out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    float s = 0.f;
    for (int i = 0; i < n; ++i) s += v[i];
    *out = s * scale;
}

// Adam (bias corrected) on FP32 masters; the step number is read on device
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                            const int64_t* __restrict__ step_p) {
    const float t = (float)(*step_p + 1);
    const float c1 = 1.0f - powf(b1, t), c2 = 1.0f - powf(b2, t);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// batch of the current step: anchors[step*B + i], positives[step*B + i]
__global__ void pick_batch_kernel(const int64_t* __restrict__ anchors, const int64_t* __restrict__ positives,
                                  const int64_t* __restrict__ step_p, int B, int64_t* __restrict__ rows) {
    const int64_t base = *step_p * B;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < B; i += gridDim.x * blockDim.x) {
        rows[i] = anchors[base + i];
        rows[B + i] = positives[base + i];
    }
}

__global__ void step_inc_kernel(int64_t* step_p) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *step_p += 1;
}

// per-dimension mean and global standard deviation of the rows listed
__global__ void stats_mean_kernel(const float* __restrict__ X, int64_t ld, int D, const int64_t* __restrict__ rows,
                                  int64_t nrows, float* __restrict__ mu) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < D; t += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int64_t r = 0; r < nrows; ++r) s += X[rows[r] * ld + t];
        mu[t] = (float)(s / (double)nrows);
    }
}

constexpr int SIG_BLOCKS = 256;
constexpr int64_t PROJ_CHUNK = 65536;   // rows projected per pass

// partial sums of squared deviations over contiguous row ranges (fixed order)
__global__ void stats_sigma_part_kernel(const float* __restrict__ X, int64_t ld, int D,
                                        const int64_t* __restrict__ rows, int64_t nrows,
                                        const float* __restrict__ mu, double* __restrict__ part) {
    __shared__ double red[256];
    const int64_t per = (nrows + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = blockIdx.x * per, r1 = r0 + per < nrows ? r0 + per : nrows;
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r)
        for (int t = threadIdx.x; t < D; t += blockDim.x) {
            const double u = (double)X[rows[r] * ld + t] - (double)mu[t];
            s += u * u;
        }
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int i = 0; i < (int)blockDim.x; ++i) tot += red[i];
        part[blockIdx.x] = tot;
    }
}

__global__ void stats_sigma_final_kernel(const double* __restrict__ part, int nb, int64_t count,
                                         float* __restrict__ sigma) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double tot = 0.0;
    for (int b = 0; b < nb; ++b) tot += part[b];
    *sigma = (float)sqrt(tot / (double)count);
}

// ---------------------------------------------------------------------------
// one forward + backward on the rows listed in `rows` (B anchors, then B
// positives); writes the mean loss and the gradients
// ---------------------------------------------------------------------------
struct Net {
    int D, H, E;
    const float *W1, *b1, *W2, *b2, *mu, *sigma;
};

struct Scratch {
    float *Z, *H1, *A1, *H2, *F, *NR, *LG, *G, *DF, *DA1, *LR, *LOSS;
};

inline size_t scratch_floats(int64_t R2, int D, int H, int E, int B) {
    // every carved array is rounded up to 64 floats: 12 arrays
    return (size_t)R2 * D + 2 * (size_t)R2 * H + 3 * (size_t)R2 * E + R2 + 2 * (size_t)B * B + (size_t)R2 * H +
           B + 1 + 64 * 12;
}

inline Scratch carve(float* base, int64_t R2, int D, int H, int E, int B) {
    Scratch sc;
    float* p = base;
    auto take = [&](size_t n) {
        float* q = p;
        p += (n + 63) / 64 * 64;
        return q;
    };
    sc.Z = take((size_t)R2 * D);
    sc.H1 = take((size_t)R2 * H);
    sc.A1 = take((size_t)R2 * H);
    sc.H2 = take((size_t)R2 * E);
    sc.F = take((size_t)R2 * E);
    sc.DF = take((size_t)R2 * E);
    sc.NR = take(R2);
    sc.LG = take((size_t)B * B);
    sc.G = take((size_t)B * B);
    sc.DA1 = take((size_t)R2 * H);
    sc.LR = take(B);
    sc.LOSS = take(1);
    return sc;
}

inline size_t scratch_bytes(int B, int D, int H, int E) {
    const int64_t R2 = 2 * (int64_t)B;
    return scratch_floats(R2, D, H, E, B) * sizeof(float) + 4096;
}

void forward(const Net& net, const float* X, int64_t ld, const int64_t* rows, int64_t R, Scratch& sc,
             hipStream_t s) {
    const int D = net.D, H = net.H, E = net.E;
    zscore_kernel<<<(unsigned)std::min<int64_t>(cdiv(R * D, 256), 8192), 256, 0, s>>>(X, ld, D, rows, R, net.mu,
                                                                                     net.sigma, sc.Z);
    SG_LAUNCH_CHECK();
    // H1 = Z W1^T  (R x D) x (D x H): B(k,n) = W1[n][k]
    gemm<true>((int)R, H, D, 1.f, sc.Z, D, 1, net.W1, 1, D, 0.f, sc.H1, H, s);
    bias_gelu_kernel<<<(unsigned)std::min<int64_t>(cdiv(R * H, 256), 8192), 256, 0, s>>>(sc.H1, net.b1, R, H,
                                                                                       sc.A1);
    SG_LAUNCH_CHECK();
    gemm<true>((int)R, E, H, 1.f, sc.A1, H, 1, net.W2, 1, H, 0.f, sc.H2, E, s);
    bias_norm_kernel<<<(unsigned)cdiv(R, 4), 256, 0, s>>>(sc.H2, net.b2, R, E, sc.F, sc.NR);
    SG_LAUNCH_CHECK();
}

void loss_grad(const Net& net, const float* X, int64_t ld, const int64_t* rows, int B, float T, Scratch& sc,
               float* loss, float* gW1, float* gb1, float* gW2, float* gb2, hipStream_t s) {
    const int D = net.D, H = net.H, E = net.E;
    const int64_t R2 = 2 * (int64_t)B;
    forward(net, X, ld, rows, R2, sc, s);
    const float* Fa = sc.F;
    const float* Fp = sc.F + (int64_t)B * E;
    // logits L = Fa Fp^T / T (FP32 MFMA)
    gemm<false>(B, B, E, 1.f / T, Fa, E, 1, Fp, 1, E, 0.f, sc.LG, B, s);
    softmax_ce_kernel<<<(unsigned)cdiv(B, 4), 256, 0, s>>>(sc.LG, B, sc.G, sc.LR);
    SG_LAUNCH_CHECK();
    sum_kernel<<<1, 1, 0, s>>>(sc.LR, B, 1.f / (float)B, loss);
    SG_LAUNCH_CHECK();
    // dFa = G Fp / T ; dFp = G^T Fa / T
    gemm<false>(B, E, B, 1.f / T, sc.G, B, 1, Fp, E, 1, 0.f, sc.DF, E, s);
    gemm<false>(B, E, B, 1.f / T, sc.G, 1, B, Fa, E, 1, 0.f, sc.DF + (int64_t)B * E, E, s);
    norm_bwd_kernel<<<(unsigned)cdiv(R2, 4), 256, 0, s>>>(sc.F, sc.NR, R2, E, sc.DF);
    SG_LAUNCH_CHECK();
    // gW2 = dH2^T A1 (E x H), gb2 = colsum dH2
    gemm<true>(E, H, (int)R2, 1.f, sc.DF, 1, E, sc.A1, H, 1, 0.f, gW2, H, s);
    colsum_kernel<<<cdiv(E, 64), 64, 0, s>>>(sc.DF, R2, E, gb2);
    // dA1 = dH2 W2 (R2 x H)
    gemm<true>((int)R2, H, E, 1.f, sc.DF, E, 1, net.W2, H, 1, 0.f, sc.DA1, H, s);
    gelu_bwd_kernel<<<(unsigned)std::min<int64_t>(cdiv(R2 * H, 256), 8192), 256, 0, s>>>(sc.H1, R2 * H, sc.DA1);
    SG_LAUNCH_CHECK();
    // gW1 = dH1^T Z (H x D), gb1 = colsum dH1
    gemm<true>(H, D, (int)R2, 1.f, sc.DA1, 1, H, sc.Z, D, 1, 0.f, gW1, D, s);
    colsum_kernel<<<cdiv(H, 64), 64, 0, s>>>(sc.DA1, R2, H, gb1);
    SG_LAUNCH_CHECK();
}

}  // namespace mlp
}  // namespace sg

using namespace sg;

static void check_net(int D, int H, int E) {
    SG_REQUIRE(D >= 1 && D <= 4096 && H >= 1 && H <= 4096 && E >= 1 && E <= 1024, "bad network sizes");
}

extern "C" sg_status sg_mlp_stats(const float* X, int64_t n, int32_t D, int64_t ld, const int64_t* rows,
                                  int64_t nrows, float* mu, float* sigma, void* ws, size_t ws_bytes,
                                  void* stream) {
    return guarded([&] {
        SG_REQUIRE(n >= 1 && D >= 1 && ld >= D && nrows >= 1, "bad sizes");
        SG_REQUIRE(X && rows && mu && sigma, "NULL pointer");
        if (ws == nullptr || ws_bytes < mlp::SIG_BLOCKS * sizeof(double)) {
            set_error("sg_mlp_stats: workspace too small");
            throw Fail{SG_ERR_WORKSPACE};
        }
        hipStream_t s = as_stream(stream);
        double* part = static_cast<double*>(ws);
        mlp::stats_mean_kernel<<<cdiv(D, 256), 256, 0, s>>>(X, ld, D, rows, nrows, mu);
        mlp::stats_sigma_part_kernel<<<mlp::SIG_BLOCKS, 256, 0, s>>>(X, ld, D, rows, nrows, mu, part);
        mlp::stats_sigma_final_kernel<<<1, 1, 0, s>>>(part, mlp::SIG_BLOCKS, nrows * (int64_t)D, sigma);
        SG_LAUNCH_CHECK();
    });
}

extern "C" sg_status sg_mlp_workspace_size(int32_t B, int32_t D, int32_t H, int32_t E, size_t* bytes) {
    return guarded([&] {
        SG_REQUIRE(bytes != nullptr && B >= 1, "bad arguments");
        check_net(D, H, E);
        // rows + step counter + scratch + one gradient per parameter
        *bytes = align_up((size_t)2 * B * 8, 256) + 256 + align_up(mlp::scratch_bytes(B, D, H, E), 256) +
                 align_up(((size_t)H * D + H + (size_t)E * H + E) * 4, 256) + 4096;
    });
}

extern "C" sg_status sg_mlp_loss_grad(const float* X, int64_t n, int32_t D, int64_t ld, const int64_t* anchors,
                                      const int64_t* positives, int32_t B, int32_t H, int32_t E, const float* W1,
                                      const float* b1, const float* W2, const float* b2, const float* mu,
                                      const float* sigma, float T, float* loss, float* gW1, float* gb1,
                                      float* gW2, float* gb2, void* ws, size_t ws_bytes, void* stream) {
    return guarded([&] {
        check_net(D, H, E);
        SG_REQUIRE(n >= 1 && ld >= D && B >= 1 && T > 0, "bad sizes");
        size_t need = 0;
        SG_REQUIRE(sg_mlp_workspace_size(B, D, H, E, &need) == SG_OK, "size");
        if (ws == nullptr || ws_bytes < need) {
            set_error("sg_mlp_loss_grad: workspace too small");
            throw Fail{SG_ERR_WORKSPACE};
        }
        hipStream_t s = as_stream(stream);
        Carver cv(ws);
        int64_t* rows = cv.take<int64_t>(2 * (size_t)B);
        float* sbase = cv.take<float>(mlp::scratch_bytes(B, D, H, E) / 4);
        mlp::Scratch sc = mlp::carve(sbase, 2 * (int64_t)B, D, H, E, B);
        SG_HIP(hipMemcpyAsync(rows, anchors, B * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
        SG_HIP(hipMemcpyAsync(rows + B, positives, B * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
        mlp::Net net{D, H, E, W1, b1, W2, b2, mu, sigma};
        mlp::loss_grad(net, X, ld, rows, B, T, sc, loss, gW1, gb1, gW2, gb2, s);
    });
}

extern "C" sg_status sg_mlp_train(const float* X, int64_t n, int32_t D, int64_t ld, const int64_t* anchors,
                                  const int64_t* positives, int32_t B, int32_t steps, int32_t H, int32_t E,
                                  float* W1, float* b1, float* W2, float* b2, float* adam_m, float* adam_v,
                                  const float* mu, const float* sigma, float T, float lr, float beta1,
                                  float beta2, float eps, float* losses, int32_t use_graph, void* ws,
                                  size_t ws_bytes, void* stream) {
    return guarded([&] {
        check_net(D, H, E);
        SG_REQUIRE(n >= 1 && ld >= D && B >= 1 && steps >= 0 && T > 0, "bad sizes");
        SG_REQUIRE(X && anchors && positives && W1 && b1 && W2 && b2 && adam_m && adam_v && mu && sigma,
                   "NULL pointer");
        size_t need = 0;
        SG_REQUIRE(sg_mlp_workspace_size(B, D, H, E, &need) == SG_OK, "size");
        if (ws == nullptr || ws_bytes < need) {
            set_error("sg_mlp_train: workspace too small (need " + std::to_string(need) + " bytes)");
            throw Fail{SG_ERR_WORKSPACE};
        }
        if (steps == 0) return;
        hipStream_t s = as_stream(stream);
        Carver cv(ws);
        int64_t* rows = cv.take<int64_t>(2 * (size_t)B);
        int64_t* step_d = cv.take<int64_t>(1);
        float* sbase = cv.take<float>(mlp::scratch_bytes(B, D, H, E) / 4);
        const size_t nW1 = (size_t)H * D, nW2 = (size_t)E * H;
        const size_t np = nW1 + H + nW2 + E;
        float* grad = cv.take<float>(np);
        mlp::Scratch sc = mlp::carve(sbase, 2 * (int64_t)B, D, H, E, B);
        fill<int64_t>(step_d, 0, 1, s);
        // parameters are contiguous per tensor; Adam runs tensor by tensor
        float* P[4] = {W1, b1, W2, b2};
        const size_t NP[4] = {nW1, (size_t)H, nW2, (size_t)E};
        float* Gp[4] = {grad, grad + nW1, grad + nW1 + H, grad + nW1 + H + nW2};
        size_t moff[4] = {0, nW1, nW1 + H, nW1 + H + nW2};
        mlp::Net net{D, H, E, W1, b1, W2, b2, mu, sigma};
        auto one_step = [&](hipStream_t st, float* loss_slot) {
            mlp::pick_batch_kernel<<<cdiv(B, 256), 256, 0, st>>>(anchors, positives, step_d, B, rows);
            SG_LAUNCH_CHECK();
            mlp::loss_grad(net, X, ld, rows, B, T, sc, loss_slot, Gp[0], Gp[1], Gp[2], Gp[3], st);
            for (int t = 0; t < 4; ++t) {
                mlp::adam_kernel<<<(unsigned)std::min<size_t>(cdiv((int64_t)NP[t], 256), 4096), 256, 0, st>>>(
                    P[t], Gp[t], adam_m + moff[t], adam_v + moff[t], (int64_t)NP[t], lr, beta1, beta2, eps, step_d);
                SG_LAUNCH_CHECK();
            }
            mlp::step_inc_kernel<<<1, 1, 0, st>>>(step_d);
            SG_LAUNCH_CHECK();
        };
        if (use_graph) {
            // capture one step (losses written to a per-step slot selected on replay by a copy)
            float* loss_slot = sc.LOSS;
            hipStream_t cs;
            SG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            hipEvent_t ready;
            SG_HIP(hipEventCreate(&ready));
            SG_HIP(hipEventRecord(ready, s));
            SG_HIP(hipStreamWaitEvent(cs, ready, 0));
            hipGraph_t g;
            SG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            one_step(cs, loss_slot);
            SG_HIP(hipStreamEndCapture(cs, &g));
            hipGraphExec_t ge;
            SG_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
            for (int it = 0; it < steps; ++it) {
                SG_HIP(hipGraphLaunch(ge, cs));
                if (losses) SG_HIP(hipMemcpyAsync(losses + it, loss_slot, sizeof(float), hipMemcpyDeviceToDevice, cs));
            }
            hipEvent_t done;
            SG_HIP(hipEventCreate(&done));
            SG_HIP(hipEventRecord(done, cs));
            SG_HIP(hipStreamWaitEvent(s, done, 0));
            SG_HIP(hipStreamSynchronize(cs));
            hipGraphExecDestroy(ge);
            hipGraphDestroy(g);
            hipEventDestroy(ready);
            hipEventDestroy(done);
            hipStreamDestroy(cs);
        } else {
            for (int it = 0; it < steps; ++it) one_step(s, losses ? losses + it : sc.LOSS);
        }
    });
}

extern "C" sg_status sg_mlp_project_workspace_size(int32_t D, int32_t H, int32_t E, size_t* bytes) {
    return guarded([&] {
        SG_REQUIRE(bytes != nullptr, "bytes is NULL");
        check_net(D, H, E);
        const size_t CH = mlp::PROJ_CHUNK;
        *bytes = CH * 8 + (CH * D + 2 * CH * H + CH * E + CH) * 4 + 8 * 256 + 4096;
    });
}

extern "C" sg_status sg_mlp_project(const float* X, int64_t n, int32_t D, int64_t ld, int32_t H, int32_t E,
                                    const float* W1, const float* b1, const float* W2, const float* b2,
                                    const float* mu, const float* sigma, float* F, void* ws, size_t ws_bytes,
                                    void* stream) {
    return guarded([&] {
        check_net(D, H, E);
        SG_REQUIRE(n >= 0 && n <= MAX_ROWS && ld >= D, "bad sizes (at most 2^26 - 1024 rows)");
        if (n == 0) return;
        SG_REQUIRE(X && F && W1 && b1 && W2 && b2 && mu && sigma, "NULL pointer");
        const int64_t CH = mlp::PROJ_CHUNK;
        size_t need = 0;
        SG_REQUIRE(sg_mlp_project_workspace_size(D, H, E, &need) == SG_OK, "size");
        if (ws == nullptr || ws_bytes < need) {
            set_error("sg_mlp_project: workspace too small (need " + std::to_string(need) + " bytes)");
            throw Fail{SG_ERR_WORKSPACE};
        }
        hipStream_t s = as_stream(stream);
        Carver cv(ws);
        int64_t* rows = cv.take<int64_t>(CH);
        mlp::Scratch sc;
        sc.Z = cv.take<float>((size_t)CH * D);
        sc.H1 = cv.take<float>((size_t)CH * H);
        sc.A1 = cv.take<float>((size_t)CH * H);
        sc.H2 = cv.take<float>((size_t)CH * E);
        sc.NR = cv.take<float>(CH);
        mlp::Net net{D, H, E, W1, b1, W2, b2, mu, sigma};
        for (int64_t r0 = 0; r0 < n; r0 += CH) {
            const int64_t R = std::min<int64_t>(CH, n - r0);
            sg::fill_iota(rows, r0, R, s);
            sc.F = F + r0 * E;
            mlp::forward(net, X, ld, rows, R, sc, s);
        }
    });
}

// batch_impl.hpp -- device code of the batched build shared by batch.hip and
// the shapes_*.hip translation units: the shard table, the batched
// nearest-pivot and persistent distance kernels, and the launch-shape maker.
#pragma once
#include "knn_impl.hpp"

namespace sg {
namespace batch {

using namespace knn;

constexpr int MAXS = 64;

// The shard table, passed by value to the batched kernels.  Shard s holds
// input / output rows [row0[s], row0[s+1]) (row0[0] = 0), operand rows
// [pad0[s], pad0[s] + n_s) of a layout padded per shard to PAD_ROWS, pivot
// labels [piv0[s], piv0[s+1]) and pivot operand rows from ppad0[s].  Work
// items: the k-th largest shard, order[k], owns items [item0[k], item0[k+1]).
struct Shards {
    int S;
    int64_t row0[MAXS + 1];
    int64_t pad0[MAXS + 1];
    int64_t piv0[MAXS + 1];
    int64_t ppad0[MAXS + 1];
    int32_t item0[MAXS + 1];
    int32_t order[MAXS];
};

// largest s in [0, S) with b[s] <= x
__device__ inline int shard_of(const int64_t* b, int S, int64_t x) {
    int lo = 0, hi = S - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b[mid] <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}


// Nearest pivot of every row, each shard against its own pivots; labels are
// global (shard s owns labels piv0[s]..).
template <int P, int NSTEP>
__global__ __launch_bounds__(NEAR_WAVES * 64) void near_batched_kernel(Shards sh, const uint8_t* __restrict__ pops,
                                                                       const float* __restrict__ pinit,
                                                                       const int32_t* __restrict__ psexp,
                                                                       const uint8_t* __restrict__ ops,
                                                                       const int32_t* __restrict__ sexp, float qmul,
                                                                       int32_t* __restrict__ lab) {
    constexpr int RB = Shape<P, NSTEP, 32>::ROW_BYTES;
    constexpr int QR = NEAR_WAVES * 32;   // query rows per block; PAD_ROWS is a multiple
    const int64_t r = (int64_t)blockIdx.x * QR;
    const int s = shard_of(sh.pad0, sh.S, r);
    const int64_t p0 = sh.pad0[s], pp0 = sh.ppad0[s];
    nearest_block<P, NSTEP, NEAR_WAVES>((r - p0) / QR, pops + pp0 * RB, pinit + pp0, psexp ? psexp + pp0 : nullptr,
                                        (int)(sh.piv0[s + 1] - sh.piv0[s]), ops + p0 * RB, sexp ? sexp + p0 : nullptr,
                                        (int)(sh.row0[s + 1] - sh.row0[s]), qmul, lab + p0, (int32_t)sh.piv0[s]);
}



// Persistent distance + top-k over all shards.  A holds the base pointers of
// the whole batch (operand-layout arrays and the output lists); each item
// narrows them to one shard.  Candidate ids and output rows are batch rows
// (row0-based); every workgroup leaves once the counter passes the last item.
template <int P, int NSTEP, int KSEL, int WAVES, int QB, int CBQ, int BCR>
__global__ __launch_bounds__(WAVES * 64, min_waves_per_simd(WAVES, BCR, CBQ)) void dist_topk_batched_kernel(
    TopkArgs A, Shards sh, unsigned int* __restrict__ counter, int nitems) {
    __shared__ TopkSmem<P, NSTEP, WAVES, QB, CBQ, BCR> sm;
    __shared__ int s_item;
    constexpr int RB = Shape<P, NSTEP, BCR>::ROW_BYTES;
    while (true) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= nitems) break;
        int k = 0;
        while (k + 1 < sh.S && sh.item0[k + 1] <= it) ++k;
        const int s = sh.order[k];
        const int64_t p0 = sh.pad0[s];
        TopkArgs B = A;
        B.ops = A.ops + p0 * RB;
        B.ninit = A.ninit + p0;
        B.sexp = A.sexp ? A.sexp + p0 : nullptr;
        B.cpid = A.cpid + p0;
        B.n = (int)(sh.row0[s + 1] - sh.row0[s]);
        B.qops = B.ops;
        B.qid = nullptr;
        B.qnout = A.qnout + p0;
        B.qsexp = B.sexp;
        B.qout = A.qout + p0;
        B.nq = B.n;
        B.state = A.state + p0 * KSEL;
        topk_block<P, NSTEP, KSEL, WAVES, QB, CBQ, BCR>(sm, it - sh.item0[k], B);
    }
}


typedef void (*bfn)(TopkArgs, Shards, unsigned int*, int);
typedef void (*bnear_fn)(Shards, const uint8_t*, const float*, const int32_t*, const uint8_t*, const int32_t*, float,
                         int32_t*);

struct BKern {
    bfn fn = nullptr;
    bnear_fn near = nullptr;
    int DP = 0, nq_block = 0, threads = 0;
};

template <int KSEL>
struct BatchedMaker {
    std::vector<BKern> v;
    template <int P, int NSTEP, int W, int QB, int CBQ, int BCR>
    void add() {
        BKern k;
        k.fn = dist_topk_batched_kernel<P, NSTEP, KSEL, W, QB, CBQ, BCR>;
        k.near = near_batched_kernel<P, NSTEP>;
        k.DP = 2 * NSTEP * Tr<P>::VEC;
        k.nq_block = 32 * W * QB;
        k.threads = 64 * W;
        v.push_back(k);
    }
};

}  // namespace batch
namespace knn {
SG_EXTERN_SLICES(batch::BatchedMaker, 64)
SG_EXTERN_SLICES(batch::BatchedMaker, 128)
SG_EXTERN_SLICES(batch::BatchedMaker, 256)
}  // namespace knn
namespace batch {

// The launch shapes of a batched call with selection width ksel (64, 128 or 256).
inline bool batched_shapes(int prec, int d, int ksel, std::vector<BKern>& v) {
    bool ok;
    if (ksel <= 64) {
        BatchedMaker<64> m;
        ok = for_shapes(prec, d, m);
        v = m.v;
    } else if (ksel <= 128) {
        BatchedMaker<128> m;
        ok = for_shapes(prec, d, m);
        v = m.v;
    } else {
        BatchedMaker<256> m;
        ok = for_shapes(prec, d, m);
        v = m.v;
    }
    return ok;
}

}  // namespace batch
}  // namespace sg

"""GPU parity of the exact INT8 path (SG_PREC_I8) for uint8 rows.

Rows are shifted by -128 into INT8 and contracted on the INT8 matrix cores
with exact INT32 sums; the L2 and IP keys are integers below 2^24, so the
lists and distances must equal the FP64 oracle bit for bit (ties included),
for every launch shape, with and without the locality order, in the
single-shard, row-subset and batched builds, up to d = 256."""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_10135_amd as sg
import synthdata

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _u8(n, d, seed, levels=256):
    rng = np.random.default_rng(seed)
    if levels < 256:
        return rng.integers(0, levels, size=(n, d)).astype(np.uint8)
    return synthdata.sift_like_u8(n=n, d=d, seed=seed, n_comp=max(2, n // 50))


def _extremes(n, d, seed):
    """Rows of 0 and 255 only (the largest |x - 128| products and sums)."""
    rng = np.random.default_rng(seed)
    return (rng.integers(0, 2, size=(n, d)) * 255).astype(np.uint8)


@pytest.mark.parametrize("metric", ["l2", "ip"])
@pytest.mark.parametrize("n,d,K", [(1, 128, 4), (5, 128, 8), (33, 16, 32), (200, 128, 64),
                                   (1000, 96, 32), (2100, 128, 64), (700, 24, 100), (300, 8, 256),
                                   (800, 200, 64), (600, 256, 32)])
def test_i8_bit_exact(metric, n, d, K):
    X = _u8(n, d, seed=n * 7 + d)
    m = oracle.IP if metric == "ip" else oracle.L2
    nbr, dist = sg.sg_knn_graph(torch.from_numpy(X).to(DEV), K, metric, "i8")
    torch.cuda.synchronize()
    onbr, odist = oracle.knn(oracle.widen(X), K, m)
    np.testing.assert_array_equal(nbr.cpu().numpy(), onbr)
    np.testing.assert_array_equal(dist.cpu().numpy(), odist.astype(np.float32))


@pytest.mark.parametrize("metric", ["l2", "ip"])
@pytest.mark.parametrize("d", [128, 256])
def test_i8_extreme_values_bit_exact(metric, d):
    # accumulators near their largest magnitude (the subtile bound is an
    # integer comparison of the largest accumulator): every launch shape
    X = _extremes(500, d, seed=d)
    m = oracle.IP if metric == "ip" else oracle.L2
    Xg = torch.from_numpy(X).to(DEV)
    onbr, odist = oracle.knn(oracle.widen(X), 48, m)
    try:
        for v in range(sg.sg_knn_variant_count(d, 48, "i8")):
            sg.sg_knn_force_variant(v)
            nbr, dist = sg.sg_knn_graph(Xg, 48, metric, "i8")
            torch.cuda.synchronize()
            np.testing.assert_array_equal(nbr.cpu().numpy(), onbr, err_msg="variant %d" % v)
            np.testing.assert_array_equal(dist.cpu().numpy(), odist.astype(np.float32))
    finally:
        sg.sg_knn_force_variant(-1)


def test_i8_heavy_ties():
    X = _u8(900, 6, seed=3, levels=4)
    nbr, dist = sg.sg_knn_graph(torch.from_numpy(X).to(DEV), 40, "l2", "i8")
    onbr, odist = oracle.knn(oracle.widen(X), 40)
    np.testing.assert_array_equal(nbr.cpu().numpy(), onbr)
    np.testing.assert_array_equal(dist.cpu().numpy(), odist.astype(np.float32))


@pytest.mark.parametrize("n,d,K", [(2100, 128, 64), (1300, 64, 32), (700, 128, 256), (900, 256, 64)])
def test_i8_every_variant_bit_exact(n, d, K):
    X = _u8(n, d, seed=n + d + K)
    Xg = torch.from_numpy(X).to(DEV)
    onbr, odist = oracle.knn(oracle.widen(X), K)
    nv = sg.sg_knn_variant_count(d, K, "i8")
    assert nv >= 1
    try:
        for v in range(nv):
            sg.sg_knn_force_variant(v)
            nbr, dist = sg.sg_knn_graph(Xg, K, "l2", "i8")
            torch.cuda.synchronize()
            np.testing.assert_array_equal(nbr.cpu().numpy(), onbr, err_msg="variant %d" % v)
            np.testing.assert_array_equal(dist.cpu().numpy(), odist.astype(np.float32))
    finally:
        sg.sg_knn_force_variant(-1)


@pytest.mark.parametrize("n,d,K,levels", [(5000, 32, 64, 256), (4500, 6, 40, 4), (6100, 128, 32, 256)])
def test_i8_locality_order_bit_exact(n, d, K, levels):
    X = _u8(n, d, seed=n + levels, levels=levels)
    nbr, dist = sg.sg_knn_graph(torch.from_numpy(X).to(DEV), K, "l2", "i8")
    torch.cuda.synchronize()
    onbr, odist = oracle.knn(oracle.widen(X), K)
    np.testing.assert_array_equal(nbr.cpu().numpy(), onbr)
    np.testing.assert_array_equal(dist.cpu().numpy(), odist.astype(np.float32))


def test_i8_many_merges_sampled_exact():
    X = synthdata.sift_like_u8(n=20000, d=128, seed=5, n_comp=40)
    Xg = torch.from_numpy(X).to(DEV)
    rows = np.random.default_rng(2).choice(20000, size=96, replace=False)
    onbr, odist = oracle.knn(oracle.widen(X), 64, rows=rows)
    nbr, dist = sg.sg_knn_graph(Xg, 64, "l2", "i8")
    torch.cuda.synchronize()
    np.testing.assert_array_equal(nbr.cpu().numpy()[rows], onbr)
    np.testing.assert_array_equal(dist.cpu().numpy()[rows], odist.astype(np.float32))


def test_i8_rows_subset_bit_exact():
    X = _u8(3000, 128, seed=77)
    rows = np.random.default_rng(1).choice(3000, size=300, replace=False)
    nbr, dist = sg.sg_knn_rows(torch.from_numpy(X).to(DEV), rows, 64, "l2", "i8")
    onbr, odist = oracle.knn(oracle.widen(X), 64, rows=rows)
    np.testing.assert_array_equal(nbr.cpu().numpy(), onbr)
    np.testing.assert_array_equal(dist.cpu().numpy(), odist.astype(np.float32))


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_i8_batched_equals_per_shard_and_oracle(metric):
    sizes = [3000, 0, 700, 4500, 40, 1]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    X = synthdata.sift_like_u8(n=int(offs[-1]), d=128, seed=31, n_comp=60)
    Xg = torch.from_numpy(X).to(DEV)
    k, R = 32, 16
    graphs, knn = sg.sg_knn_graph_batched(Xg, offs, k, R, metric, "i8")
    torch.cuda.synchronize()
    m = oracle.IP if metric == "ip" else oracle.L2
    knn_h, g_h = knn.cpu().numpy(), graphs.cpu().numpy()
    for s in range(len(sizes)):
        a, b = offs[s], offs[s + 1]
        if b - a < 2:
            continue
        onbr, _ = oracle.knn(oracle.widen(X[a:b]), k, m)
        np.testing.assert_array_equal(knn_h[a:b], onbr, err_msg="shard %d" % s)
        np.testing.assert_array_equal(g_h[a:b], oracle.prune(onbr, R), err_msg="shard %d" % s)


def test_i8_operands_and_norms():
    X = _u8(300, 100, seed=4)
    q, sexp, sq = sg.sg_quantize_rows(torch.from_numpy(X).to(DEV), "i8", ldo=128)
    torch.cuda.synchronize()
    got = q.cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(got[:, :100], X.astype(np.int64) - 128)
    assert (got[:, 100:] == 0).all()
    assert sexp is None
    np.testing.assert_array_equal(sq.cpu().numpy().astype(np.int64), ((X.astype(np.int64) - 128) ** 2).sum(1))


def test_i8_refuses_other_inputs():
    with pytest.raises(sg.SgError):
        sg.sg_knn_graph(torch.zeros((100, 16), dtype=torch.float32, device=DEV), 8, "l2", "i8")
    with pytest.raises(sg.SgError):
        sg.sg_knn_graph(torch.zeros((100, 300), dtype=torch.uint8, device=DEV), 8, "l2", "i8")

"""GPU parity of sg_knn_graph against the FP64 oracle (through the C ABI).

Integer-valued rows (uint8, d <= 128) make every FP32 product and partial sum
exact, so the FP32-MFMA and FP16-MFMA builds must equal the oracle bit for bit,
ties included.  Float rows are compared under the FP32 rounding-bound rule in
parity.py, with no row allowance.
Reduced-precision keys (BF16, FP8) with the FP32 re-rank are judged by recall
and by the exactness of the re-ranked distances they return.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_10135_amd as sg
import synthdata
from parity import check_rows, recall

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _u8(n, d, seed, levels=256):
    rng = np.random.default_rng(seed)
    if levels < 256:
        return rng.integers(0, levels, size=(n, d)).astype(np.uint8)
    return synthdata.sift_like_u8(n=n, d=d, seed=seed, n_comp=max(2, n // 50))


@pytest.mark.parametrize("prec", ["fp32", "f16"])
@pytest.mark.parametrize("n,d,K", [(1, 128, 4), (5, 128, 8), (33, 16, 32), (200, 128, 64),
                                   (1000, 96, 32), (2100, 128, 64), (700, 24, 100), (300, 8, 256)])
def test_knn_u8_bit_exact(prec, n, d, K):
    X = _u8(n, d, seed=n * 7 + d)
    nbr, dist = sg.sg_knn_graph(torch.from_numpy(X).to(DEV), K, "l2", prec)
    torch.cuda.synchronize()
    onbr, odist = oracle.knn(oracle.widen(X), K)
    np.testing.assert_array_equal(nbr.cpu().numpy(), onbr)
    np.testing.assert_array_equal(dist.cpu().numpy(), odist.astype(np.float32))


@pytest.mark.parametrize("prec", ["fp32", "f16"])
def test_knn_u8_heavy_ties(prec):
    # 4 levels in 6 dims: huge numbers of exactly equal distances -> the id rule decides
    X = _u8(900, 6, seed=3, levels=4)
    nbr, dist = sg.sg_knn_graph(torch.from_numpy(X).to(DEV), 40, "l2", prec)
    onbr, odist = oracle.knn(oracle.widen(X), 40)
    np.testing.assert_array_equal(nbr.cpu().numpy(), onbr)
    np.testing.assert_array_equal(dist.cpu().numpy(), odist.astype(np.float32))


def test_knn_u8_ip_bit_exact():
    X = _u8(600, 32, seed=11, levels=16)
    nbr, dist = sg.sg_knn_graph(torch.from_numpy(X).to(DEV), 24, "ip", "fp32")
    onbr, odist = oracle.knn(oracle.widen(X), 24, oracle.IP)
    np.testing.assert_array_equal(nbr.cpu().numpy(), onbr)
    np.testing.assert_array_equal(dist.cpu().numpy(), odist.astype(np.float32))


@pytest.mark.parametrize("n,d,K", [(2048, 96, 32), (1500, 100, 64), (333, 7, 16)])
def test_knn_f32_tie_rule(n, d, K):
    X = synthdata.mixture(n, d, 16, 0.3, seed=n + d)
    nbr, dist = sg.sg_knn_graph(torch.from_numpy(X).to(DEV), K, "l2", "fp32")
    X64 = oracle.widen(X)
    onbr, odist = oracle.knn(X64, K)
    bad = check_rows(X64, np.arange(n), nbr.cpu().numpy(), dist.cpu().numpy(), onbr, odist)
    assert not bad, bad[:5]


def test_knn_ip_unit_tie_rule():
    X = synthdata.unit_rows(synthdata.mixture(1200, 64, 20, 0.15, seed=4))
    nbr, dist = sg.sg_knn_graph(torch.from_numpy(X).to(DEV), 48, "ip", "fp32")
    X64 = oracle.widen(X)
    onbr, odist = oracle.knn(X64, 48, oracle.IP)
    bad = check_rows(X64, np.arange(len(X)), nbr.cpu().numpy(), dist.cpu().numpy(), onbr, odist,
                     oracle.IP)
    assert not bad, bad[:5]


def test_knn_f16_input_tie_rule():
    X = synthdata.unit_rows(synthdata.mixture(1000, 96, 10, 0.15, seed=8)).astype(np.float16)
    nbr, dist = sg.sg_knn_graph(torch.from_numpy(X).to(DEV), 32, "ip", "f16")
    X64 = oracle.widen(X)
    onbr, odist = oracle.knn(X64, 32, oracle.IP)
    bad = check_rows(X64, np.arange(len(X)), nbr.cpu().numpy(), dist.cpu().numpy(), onbr, odist,
                     oracle.IP)
    assert not bad, bad[:5]


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("metric", ["ip", "l2"])
def test_knn_reduced_precision_with_rerank(prec, metric):
    X = synthdata.unit_rows(synthdata.mixture(3000, 96, 40, 0.15, seed=21))
    K, c = 32, 64
    nbr, dist = sg.sg_knn_graph(torch.from_numpy(X).to(DEV), K, metric, prec, rerank=c)
    X64 = oracle.widen(X)
    m = oracle.IP if metric == "ip" else oracle.L2
    onbr, odist = oracle.knn(X64, K, m)
    g = nbr.cpu().numpy()
    assert recall(g, onbr) >= 0.99
    # the re-ranked distances are the FP32 distances of the returned pairs
    d64 = oracle.pair_dist(X64, np.repeat(np.arange(len(X))[:, None], K, 1), g, m)
    gd = dist.cpu().numpy()
    scale = np.maximum(np.abs(d64), 1e-3)
    assert np.max(np.abs(gd - d64) / scale) < 1e-5
    for row in g[:50]:
        assert len(set(row.tolist())) == K


def test_knn_deterministic():
    X = synthdata.mixture(1500, 64, 8, 0.5, seed=2)
    Xg = torch.from_numpy(X).to(DEV)
    a = sg.sg_knn_graph(Xg, 32, "l2", "fp32")
    b = sg.sg_knn_graph(Xg, 32, "l2", "fp32")
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


@pytest.mark.parametrize("prec", ["fp32", "f16"])
def test_knn_rows_u8_bit_exact(prec):
    X = _u8(3000, 128, seed=77)
    rows = np.random.default_rng(1).choice(3000, size=300, replace=False)
    nbr, dist = sg.sg_knn_rows(torch.from_numpy(X).to(DEV), rows, 64, "l2", prec)
    onbr, odist = oracle.knn(oracle.widen(X), 64, rows=rows)
    np.testing.assert_array_equal(nbr.cpu().numpy(), onbr)
    np.testing.assert_array_equal(dist.cpu().numpy(), odist.astype(np.float32))


def test_knn_rows_rerank_and_full_agree():
    X = synthdata.unit_rows(synthdata.mixture(2500, 96, 30, 0.15, seed=3))
    Xg = torch.from_numpy(X).to(DEV)
    rows = np.arange(0, 2500, 7)
    full, _ = sg.sg_knn_graph(Xg, 32, "ip", "bf16", rerank=64)
    sub, _ = sg.sg_knn_rows(Xg, rows, 32, "ip", "bf16", rerank=64)
    np.testing.assert_array_equal(sub.cpu().numpy(), full.cpu().numpy()[rows])


@pytest.mark.parametrize("n,d,K", [(700, 960, 64), (1030, 200, 32), (300, 129, 16)])
def test_knn_wide_fp32_kstream_exact(n, d, K):
    # small integers: every FP32 product and partial sum is exact at d = 960
    X = _u8(n, d, seed=d, levels=16).astype(np.float32)
    nbr, dist = sg.sg_knn_graph(torch.from_numpy(X).to(DEV), K, "l2", "fp32")
    onbr, odist = oracle.knn(oracle.widen(X), K)
    np.testing.assert_array_equal(nbr.cpu().numpy(), onbr)
    np.testing.assert_array_equal(dist.cpu().numpy(), odist.astype(np.float32))


@pytest.mark.parametrize("d", [768, 300])
def test_knn_wide_f16_four_wave_exact(d):
    X = _u8(900, d, seed=d + 1, levels=12).astype(np.float16)
    nbr, dist = sg.sg_knn_graph(torch.from_numpy(X).to(DEV), 64, "ip", "f16")
    onbr, odist = oracle.knn(oracle.widen(X), 64, oracle.IP)
    np.testing.assert_array_equal(nbr.cpu().numpy(), onbr)
    np.testing.assert_array_equal(dist.cpu().numpy(), odist.astype(np.float32))


def test_knn_rows_wide_fp32_exact():
    X = _u8(1500, 960, seed=5, levels=16).astype(np.float32)
    rows = np.arange(3, 1500, 11)
    nbr, _ = sg.sg_knn_rows(torch.from_numpy(X).to(DEV), rows, 64, "l2", "fp32")
    onbr, _ = oracle.knn(oracle.widen(X), 64, rows=rows)
    np.testing.assert_array_equal(nbr.cpu().numpy(), onbr)


def test_knn_fp8_wide_rerank_recall():
    X = synthdata.l1_nonneg(2000, d=512, seed=9, n_comp=20)
    nbr, _ = sg.sg_knn_graph(torch.from_numpy(X).to(DEV), 32, "l2", "fp8", rerank=128)
    onbr, _ = oracle.knn(oracle.widen(X), 32)
    assert recall(nbr.cpu().numpy(), onbr) >= 0.95


@pytest.mark.parametrize("prec", ["fp32", "f16"])
@pytest.mark.parametrize("n,d,K", [(2100, 128, 64), (1300, 64, 32), (900, 96, 128), (700, 128, 256)])
def test_knn_every_variant_bit_exact(prec, n, d, K):
    """Each launch-shape variant of the distance kernel gives the oracle's lists."""
    X = _u8(n, d, seed=n + d + K)
    Xg = torch.from_numpy(X).to(DEV)
    onbr, odist = oracle.knn(oracle.widen(X), K)
    nv = sg.sg_knn_variant_count(d, K, prec)
    assert nv >= 1
    try:
        for v in range(nv):
            sg.sg_knn_force_variant(v)
            nbr, dist = sg.sg_knn_graph(Xg, K, "l2", prec)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(nbr.cpu().numpy(), onbr, err_msg="variant %d" % v)
            np.testing.assert_array_equal(dist.cpu().numpy(), odist.astype(np.float32))
    finally:
        sg.sg_knn_force_variant(-1)


@pytest.mark.parametrize("prec,d", [("bf16", 96), ("fp8", 64), ("bf16", 128)])
def test_knn_reduced_variants_agree(prec, d):
    X = synthdata.unit_rows(synthdata.mixture(3000, d, 30, 0.3, seed=d))
    Xg = torch.from_numpy(X).to(DEV)
    nv = sg.sg_knn_variant_count(d, 64, prec)
    outs = []
    try:
        for v in range(nv):
            sg.sg_knn_force_variant(v)
            nbr, dist = sg.sg_knn_graph(Xg, 64, "ip", prec, rerank=128)
            torch.cuda.synchronize()
            outs.append((nbr.cpu().numpy(), dist.cpu().numpy()))
    finally:
        sg.sg_knn_force_variant(-1)
    for v in range(1, nv):
        np.testing.assert_array_equal(outs[v][0], outs[0][0])
        np.testing.assert_array_equal(outs[v][1], outs[0][1])


def test_knn_many_merges_sampled_exact():
    """A shard large enough that every query merges its buffer many times
    (and subtiles overflow mid-way): sampled rows equal the oracle."""
    X = synthdata.sift_like_u8(n=20000, d=128, seed=5, n_comp=40)
    Xg = torch.from_numpy(X).to(DEV)
    rows = np.random.default_rng(2).choice(20000, size=96, replace=False)
    onbr, odist = oracle.knn(oracle.widen(X), 64, rows=rows)
    nv = sg.sg_knn_variant_count(128, 64, "f16")
    try:
        for v in range(nv):
            sg.sg_knn_force_variant(v)
            for prec in ("f16", "fp32"):
                nbr, dist = sg.sg_knn_graph(Xg, 64, "l2", prec)
                torch.cuda.synchronize()
                np.testing.assert_array_equal(nbr.cpu().numpy()[rows], onbr, err_msg="%s v%d" % (prec, v))
                np.testing.assert_array_equal(dist.cpu().numpy()[rows], odist.astype(np.float32))
    finally:
        sg.sg_knn_force_variant(-1)


def test_knn_autotune_records_a_valid_choice():
    X = _u8(5000, 128, seed=77)
    Xg = torch.from_numpy(X).to(DEV)
    ref, _ = sg.sg_knn_graph(Xg, 64, "l2", "f16")
    chosen, times = sg.sg_knn_autotune(Xg, 64, "l2", "f16")
    assert 0 <= chosen < len(times) == sg.sg_knn_variant_count(128, 64, "f16")
    assert all(t > 0 for t in times) and times[chosen] == min(times)
    nbr, _ = sg.sg_knn_graph(Xg, 64, "l2", "f16")
    torch.cuda.synchronize()
    assert torch.equal(nbr, ref)


@pytest.mark.parametrize("prec", ["fp32", "f16"])
@pytest.mark.parametrize("n,d,K,levels", [(5000, 32, 64, 256), (4500, 6, 40, 4), (6100, 128, 32, 256)])
def test_knn_locality_order_bit_exact(prec, n, d, K, levels):
    """Shards of >= 4096 rows are scanned in pivot order; every row's list
    (ties included) still equals the oracle's."""
    X = _u8(n, d, seed=n + levels, levels=levels)
    nbr, dist = sg.sg_knn_graph(torch.from_numpy(X).to(DEV), K, "l2", prec)
    torch.cuda.synchronize()
    onbr, odist = oracle.knn(oracle.widen(X), K)
    np.testing.assert_array_equal(nbr.cpu().numpy(), onbr)
    np.testing.assert_array_equal(dist.cpu().numpy(), odist.astype(np.float32))


def test_knn_locality_order_f32_and_rerank():
    X = synthdata.unit_rows(synthdata.mixture(5200, 48, 40, 0.3, seed=9))
    Xg = torch.from_numpy(X).to(DEV)
    X64 = oracle.widen(X)
    onbr, odist = oracle.knn(X64, 32, oracle.IP)
    nbr, dist = sg.sg_knn_graph(Xg, 32, "ip", "fp32")
    torch.cuda.synchronize()
    bad = check_rows(X64, np.arange(len(X)), nbr.cpu().numpy(), dist.cpu().numpy(), onbr, odist, oracle.IP)
    assert not bad, bad[:5]
    nb2, d2 = sg.sg_knn_graph(Xg, 32, "ip", "bf16", rerank=64)
    torch.cuda.synchronize()
    assert recall(nb2.cpu().numpy(), onbr) >= 0.99


@pytest.mark.parametrize("n,levels", [(6000, 256), (5000, 4)])
def test_knn_order_is_deterministic_and_a_permutation(n, levels):
    """The locality order sg_knn_graph returns is a stable sort by pivot: the
    same call gives the same order, bit for bit, and it is a permutation."""
    X = _u8(n, 32, seed=n, levels=levels)
    Xg = torch.from_numpy(X).to(DEV)
    o1 = torch.empty(n, dtype=torch.int32, device=DEV)
    o2 = torch.empty(n, dtype=torch.int32, device=DEV)
    a, _ = sg.sg_knn_graph(Xg, 16, "l2", "f16", order_out=o1)
    b, _ = sg.sg_knn_graph(Xg, 16, "l2", "f16", order_out=o2)
    torch.cuda.synchronize()
    assert torch.equal(o1, o2)
    assert torch.equal(a, b)
    assert np.array_equal(np.sort(o1.cpu().numpy()), np.arange(n))

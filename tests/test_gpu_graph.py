"""GPU parity of the integer passes (sg_prune, sg_merge) against the oracle:
bit-exact on the hand-worked examples, on exact kNN graphs of seeded data and
on seeded random graphs (with padding, odd R, K = R, high in-degree)."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2605_10135_amd as sg
import synthdata

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _prune_gpu(knn, R):
    out = sg.sg_prune(torch.from_numpy(np.ascontiguousarray(knn, np.int32)).to(DEV), R)
    return out.cpu().numpy()


def test_prune_worked_example():
    g = _gold("detour_prune_5.json")
    knn = np.array(g["knn"], np.int32)
    # the worked example fixes P; the reverse pass then adds nothing at R = 2
    assert _prune_gpu(knn, g["R"]).tolist() == oracle.prune(knn, g["R"]).tolist()
    assert oracle.detour_prune(knn, g["R"]).tolist() == g["expected_P"]


def test_reverse_combine_worked_example_through_prune():
    # a K = R input makes the detour step a permutation; compare the whole pass
    g = _gold("reverse_combine_7.json")
    P = np.array(g["P"], np.int32)
    exp = oracle.reverse_combine(oracle.detour_prune(P, P.shape[1]))
    assert _prune_gpu(P, P.shape[1]).tolist() == exp.tolist()


@pytest.mark.parametrize("n,K,R", [(300, 32, 16), (1000, 64, 32), (257, 64, 64), (500, 20, 7),
                                   (130, 128, 64), (600, 256, 33), (700, 128, 65), (900, 256, 128),
                                   (300, 96, 96), (1100, 256, 99), (1800, 64, 64), (1800, 64, 32)])
def test_prune_on_random_graphs(n, K, R):
    knn = synthdata.local_graph(n, K, seed=n + K + R) if n > 2 * K + 2 else synthdata.random_graph(n, K, seed=n)
    np.testing.assert_array_equal(_prune_gpu(knn, R), oracle.prune(knn, R))


def test_prune_with_padding():
    knn = synthdata.random_graph(400, 24, seed=5, n_none=5)
    np.testing.assert_array_equal(_prune_gpu(knn, 12), oracle.prune(knn, 12))


@pytest.mark.parametrize("n,d,K,R", [(2000, 128, 64, 32), (3000, 96, 32, 16), (40, 8, 64, 32),
                                     (2500, 128, 128, 64), (2500, 128, 256, 128), (200, 16, 256, 128)])
def test_prune_on_exact_knn(n, d, K, R):
    X = synthdata.sift_like_u8(n=n, d=d, seed=n, n_comp=max(2, n // 100))
    knn, _ = oracle.knn(oracle.widen(X), K)
    np.testing.assert_array_equal(_prune_gpu(knn, R), oracle.prune(knn, R))


@pytest.mark.parametrize("K,R", [(16, 8), (160, 100)])
def test_prune_hub_in_degree(K, R):
    # many rows point at a few hubs: in-degree >> 64 (>> 128 for R > 64)
    # exercises the chunked selection of the smallest reverse keys
    rng = np.random.default_rng(0)
    n = 3000
    knn = np.empty((n, K), np.int32)
    for i in range(n):
        hubs = [h for h in range(8) if h != i][:4]
        rest = rng.choice([j for j in range(n) if j != i and j not in hubs][:max(200, 2 * K)], K - 4,
                          replace=False)
        knn[i] = np.concatenate([hubs, rest])
    np.testing.assert_array_equal(_prune_gpu(knn, R), oracle.prune(knn, R))


@pytest.mark.parametrize("n,half,R", [(500, 8, 8), (500, 8, 16), (130, 32, 21), (70, 32, 64),
                                      (400, 64, 128), (300, 64, 77), (260, 128, 128)])
def test_prune_symmetric_graph(n, half, R):
    # circulant graph, offsets +-1..+-half by |offset|: every edge is mutual, so
    # Rev(y) repeats most of P(y) and the in-order deduplication decides F(y)
    offs = [s * o for o in range(1, half + 1) for s in (1, -1)]
    knn = (np.arange(n)[:, None] + np.array(offs)[None, :]) % n
    np.testing.assert_array_equal(_prune_gpu(knn.astype(np.int32), R), oracle.prune(knn.astype(np.int32), R))


def _cuckoo_slots(z, ct=256):
    """The two table slots the detour kernel's row hash gives id z (K <= 64):
    bits 8.. and 20.. of the low 32 bits of (low 24 bits of z) * 0x9E3779."""
    z = np.asarray(z, np.uint64) & np.uint64(0xFFFFFF)
    p = (z * np.uint64(0x9E3779)) & np.uint64(0xFFFFFFFF)
    return (p >> np.uint64(8)) & np.uint64(ct - 1), (p >> np.uint64(20)) & np.uint64(ct - 1)


def test_prune_rows_whose_table_cannot_settle():
    # four ids that share both table slots cannot all be placed: rows holding
    # them take the kernel's compare-with-every-entry path, with the same result
    n, K, R = 300_000, 32, 12
    h0, h1 = _cuckoo_slots(np.arange(n))
    key = h0 * np.uint64(256) + h1
    vals, first, counts = np.unique(key, return_index=True, return_counts=True)
    clash = np.nonzero(key == vals[np.argmax(counts >= 4)])[0][:4]
    assert len(clash) == 4
    rng = np.random.default_rng(11)
    active = np.unique(np.concatenate([clash, rng.choice(n, 600, replace=False)]))
    knn = np.full((n, K), -1, np.int32)
    for x in active:
        pool = active[active != x]
        if rng.random() < 0.5:           # rows holding the clashing ids (distinct ids per row)
            c = clash[clash != x]
            pick = np.concatenate([c, rng.choice(pool[~np.isin(pool, c)], K - len(c), replace=False)])
        else:
            pick = rng.choice(pool, K, replace=False)
        knn[x] = pick
    np.testing.assert_array_equal(_prune_gpu(knn, R), oracle.prune(knn, R))


def test_prune_rejects_more_rows_than_one_call_takes():
    # wavefront-per-row launches hold 64 work-items per row and a dispatch
    # fewer than 2^32: the entry point refuses 2^26 rows before any launch
    knn = torch.full((1 << 26, 1), -1, dtype=torch.int32, device=DEV)
    with pytest.raises(sg.SgError, match="n out of range"):
        sg.sg_prune(knn, 1)
    del knn
    torch.cuda.empty_cache()


def _merge_gpu(off, mem, graphs, R, n_global, cap):
    out, deg = sg.sg_merge(off, torch.from_numpy(np.asarray(mem, np.int32)).to(DEV),
                           torch.from_numpy(np.asarray(graphs, np.int32)).to(DEV), R, n_global, cap)
    return out.cpu().numpy(), deg.cpu().numpy()


@pytest.mark.parametrize("cap", [4, 3, 2])
def test_merge_worked_example(cap):
    g = _gold("merge_2shards.json")
    out, deg = _merge_gpu(g["offsets"], g["member_ids"], g["graphs_local"], g["R"], g["n_global"], cap)
    assert out.tolist() == g["expected"][str(cap)]["out"]
    assert deg.tolist() == g["expected"][str(cap)]["degree"]


@pytest.mark.parametrize("overlap,R", [(0.25, 8), (0.5, 16), (0.0, 5)])
def test_merge_overlapping_windows(overlap, R):
    sizes = synthdata.batched_shard_sizes(12, seed=3, mu=np.log(400), sigma=0.5, lo=100, hi=900)
    N, off, mem = synthdata.overlapping_windows(sizes, overlap)
    graphs = np.concatenate([synthdata.random_graph(int(s), R, seed=t, n_none=2) for t, s in enumerate(sizes)])
    for cap in (R, 2 * R, 3 * R):
        out, deg = _merge_gpu(off, mem, graphs, R, N, cap)
        oout, odeg = oracle.merge(off, mem, graphs, R, N, cap)
        np.testing.assert_array_equal(out, oout)
        np.testing.assert_array_equal(deg, odeg)


def test_merge_identity_and_absent_ids():
    n, R = 500, 12
    g = synthdata.random_graph(n, R, seed=9)
    off = [0, n, 2 * n]
    mem = np.concatenate([np.arange(n), np.arange(n)])
    out, deg = _merge_gpu(off, mem, np.concatenate([g, g]), R, n + 7, 2 * R)
    oout, odeg = oracle.merge(off, mem, np.concatenate([g, g]), R, n + 7, 2 * R)
    np.testing.assert_array_equal(out, oout)
    np.testing.assert_array_equal(deg, odeg)
    assert (deg[n:] == 0).all()


def test_prune_merge_deterministic():
    knn = synthdata.local_graph(2000, 32, seed=1)
    a = _prune_gpu(knn, 16)
    b = _prune_gpu(knn, 16)
    np.testing.assert_array_equal(a, b)


def test_knn_order_is_permutation_and_prune_order_free():
    """sg_knn_graph's row order is a permutation (the locality order for large
    shards); pruning in that order gives the same graph as in row order."""
    import synthdata
    X = synthdata.sift_like_u8(n=6000, d=32, seed=77, n_comp=40)
    Xg = torch.from_numpy(X).to(DEV)
    order = torch.empty(6000, dtype=torch.int32, device=DEV)
    nbr, _ = sg.sg_knn_graph(Xg, 32, "l2", "f16", dist=False, order_out=order)
    o = order.cpu().numpy()
    assert np.array_equal(np.sort(o), np.arange(6000))
    assert not np.array_equal(o, np.arange(6000))      # >= 4096 rows: reordered
    g0 = sg.sg_prune(nbr, 16)
    g1 = sg.sg_prune(nbr, 16, order=order)
    assert torch.equal(g0, g1)
    small = torch.empty(500, dtype=torch.int32, device=DEV)
    sg.sg_knn_graph(Xg[:500], 16, "l2", "f16", dist=False, order_out=small)
    assert np.array_equal(small.cpu().numpy(), np.arange(500))


def test_prune_order_that_is_not_a_permutation_is_ignored():
    """sg_prune visits rows in the caller's order only when it is a
    permutation; repeated, missing or out-of-range entries are detected on the
    device and the rows are visited in row order: the result is unchanged."""
    n, K, R = 900, 32, 16
    knn = synthdata.local_graph(n, K, seed=41)
    ref = oracle.prune(knn, R)
    kd = torch.from_numpy(knn).to(DEV)
    rng = np.random.default_rng(3)
    perm = rng.permutation(n).astype(np.int32)
    dup = perm.copy()
    dup[10] = dup[11]                       # a repeat (and so a missing row)
    oob = perm.copy()
    oob[5] = n + 7                          # out of range
    neg = perm.copy()
    neg[0] = -3
    for order in (perm, dup, oob, neg, np.zeros(n, np.int32)):
        out = sg.sg_prune(kd, R, order=torch.from_numpy(order).to(DEV))
        np.testing.assert_array_equal(out.cpu().numpy(), ref)

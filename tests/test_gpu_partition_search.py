"""GPU parity of sg_partition and sg_search against the oracle.

Partition: with zero Lloyd iterations the centroids are rows of integer data,
so every FP32 distance is exact and centroids, primaries, replicas and the
membership must equal the oracle bit for bit (including the Fig. 2 example).
After one iteration the FP64 sums of integers are exact, so the centroids must
again be identical.  Longer runs on float data agree up to near-ties.
Search: integer data makes every distance exact, so beam search on the same
graph from the same entry must return the oracle's ids exactly.
"""
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


def test_partition_fig2_example():
    with open(os.path.join(GOLD, "fig2_assignment.json")) as f:
        g = json.load(f)
    X = np.array(g["centroids"] + g["vectors"], np.float32)
    # the library takes epsilon as FP32; give the oracle that same value
    for eps in (float(np.float32(g["epsilon"])), float("inf")):
        C, prim, off, mem = sg.sg_partition(torch.from_numpy(X).to(DEV), 3, 2, 0, [0, 1, 2], eps)
        oC, oprim, ooff, omem = oracle.partition(oracle.widen(X), 3, 2, 0, [0, 1, 2], eps)
        np.testing.assert_array_equal(C.cpu().numpy(), oC)
        np.testing.assert_array_equal(prim.cpu().numpy(), oprim)
        np.testing.assert_array_equal(off.numpy(), ooff)
        np.testing.assert_array_equal(mem.cpu().numpy(), omem)
        if eps != float("inf"):
            # rows 3..5 are v1..v3: v1 joins c1 and c3, v2 only c2, v3 only c3
            members = [set(omem[ooff[s]:ooff[s + 1]].tolist()) for s in range(3)]
            assert members == [{0, 3}, {1, 4}, {2, 3, 5}]


@pytest.mark.parametrize("iters", [0, 1])
@pytest.mark.parametrize("S,omega,eps", [(4, 2, float("inf")), (6, 3, float(np.float32(1.2))),
                                         (5, 1, float("inf"))])
def test_partition_u8_exact(iters, S, omega, eps):
    X = synthdata.sift_like_u8(n=3000, d=16, seed=S * 10 + omega, n_comp=12)
    init = synthdata.init_rows(3000, S, seed=S)
    C, prim, off, mem = sg.sg_partition(torch.from_numpy(X).to(DEV), S, omega, iters, init, eps)
    X64 = oracle.widen(X)
    oC, oprim = oracle.kmeans(X64, S, iters, init)
    np.testing.assert_array_equal(C.cpu().numpy(), oC)
    if iters == 0:
        oassign, _ = oracle.assign_replicas(X64, oC, oprim, omega, eps)
        ooff, omem = oracle.membership(oassign, S)
        np.testing.assert_array_equal(prim.cpu().numpy(), oprim)
        np.testing.assert_array_equal(off.numpy(), ooff)
        np.testing.assert_array_equal(mem.cpu().numpy(), omem)


def test_partition_float_many_iterations_close():
    X = synthdata.mixture(5000, 24, 10, 0.4, seed=5)
    init = synthdata.init_rows(5000, 8, seed=1)
    C, prim, off, mem = sg.sg_partition(torch.from_numpy(X).to(DEV), 8, 2, 20, init)
    oC, oprim = oracle.kmeans(oracle.widen(X), 8, 20, init)
    agree = (prim.cpu().numpy() == oprim).mean()
    assert agree > 0.999
    np.testing.assert_allclose(C.cpu().numpy(), oC, rtol=1e-4, atol=1e-5)
    o = off.numpy()
    m = mem.cpu().numpy()
    assert o[-1] == 2 * 5000
    for s in range(8):
        assert np.all(np.diff(m[o[s]:o[s + 1]]) > 0)


@pytest.mark.parametrize("L", [16, 64, 200])
def test_search_u8_exact(L):
    X = synthdata.sift_like_u8(n=3000, d=32, seed=1, n_comp=30)
    Q = synthdata.sift_like_u8(n=100, d=32, seed=1, stream=1, n_comp=30)
    X64 = oracle.widen(X)
    knn, _ = oracle.knn(X64, 32)
    graph = oracle.prune(knn, 16)
    entry = oracle.medoid(X64)
    ids, dist = sg.sg_search(torch.from_numpy(X).to(DEV), torch.from_numpy(graph).to(DEV),
                             torch.from_numpy(Q).to(DEV), 10, L, entry=entry)
    oids, odist = oracle.search(X64, graph, oracle.widen(Q), 10, L, entry=entry)
    np.testing.assert_array_equal(ids.cpu().numpy(), oids)
    np.testing.assert_array_equal(dist.cpu().numpy(), odist.astype(np.float32))


def test_search_medoid_entry_and_wide_graph():
    X = synthdata.sift_like_u8(n=2500, d=24, seed=2, n_comp=20)
    Q = synthdata.sift_like_u8(n=64, d=24, seed=2, stream=1, n_comp=20)
    X64 = oracle.widen(X)
    knn, _ = oracle.knn(X64, 96)
    graph = oracle.prune(knn, 64)
    # merged-style wide lists: two copies of the degree with padding
    wide = np.concatenate([graph, np.full((len(X), 70), -1, np.int32)], 1)
    ids, dist = sg.sg_search(torch.from_numpy(X).to(DEV), torch.from_numpy(wide).to(DEV),
                             torch.from_numpy(Q).to(DEV), 10, 40, entry=-1)
    # the GPU medoid may differ from the FP64 one only at a near-tie; with the
    # oracle's entry the result must then be identical
    ent = oracle.medoid(X64)
    oids, _ = oracle.search(X64, wide, oracle.widen(Q), 10, 40, entry=ent)
    g = ids.cpu().numpy()
    if not np.array_equal(g, oids):
        ids2, _ = sg.sg_search(torch.from_numpy(X).to(DEV), torch.from_numpy(wide).to(DEV),
                               torch.from_numpy(Q).to(DEV), 10, 40, entry=ent)
        np.testing.assert_array_equal(ids2.cpu().numpy(), oids)

"""Pins of the oracle's integer passes: detour prune, reverse + combine, merge.

Pinned by hand-worked examples under tests/golden/ (each with its derivation),
by closed forms (K = R gives a permutation of N(x); detour(x,0) = 0 so the
nearest neighbour always survives; F(y)[0:h] = P(y)[0:h]; merge of a graph with
itself is the graph; a single-shard id copies through) and by invariants
(degree bound, no self, no duplicates, every reverse entry traces to a forward
edge, the union covers every shard list up to the cap).
"""
import json
import os

import numpy as np
import pytest

import oracle
import synthdata

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_detour_prune_worked_example():
    g = _gold("detour_prune_5.json")
    P = oracle.detour_prune(np.array(g["knn"], np.int32), g["R"])
    assert P.tolist() == g["expected_P"]


def test_reverse_combine_worked_example():
    g = _gold("reverse_combine_7.json")
    F = oracle.reverse_combine(np.array(g["P"], np.int32))
    assert F.tolist() == g["expected_F"]


@pytest.mark.parametrize("max_degree", [4, 3, 2])
def test_merge_worked_example(max_degree):
    g = _gold("merge_2shards.json")
    out, deg = oracle.merge(g["offsets"], g["member_ids"], np.array(g["graphs_local"], np.int32),
                            g["R"], g["n_global"], max_degree)
    assert out.tolist() == g["expected"][str(max_degree)]["out"]
    assert deg.tolist() == g["expected"][str(max_degree)]["degree"]


def test_prune_K_equals_R_is_permutation():
    knn = synthdata.local_graph(300, 12, seed=1)
    P = oracle.detour_prune(knn, 12)
    for a, b in zip(P, knn):
        assert sorted(a.tolist()) == sorted(b.tolist())


@pytest.mark.parametrize("K,R", [(16, 8), (32, 16), (12, 5)])
def test_prune_closed_forms(K, R):
    knn = synthdata.local_graph(400, K, seed=K + R)
    P = oracle.detour_prune(knn, R)
    assert (P[:, 0] == knn[:, 0]).all()            # detour(x, 0) = 0
    for a, b in zip(P, knn):
        assert len(set(a.tolist())) == R
        assert set(a.tolist()) <= set(b.tolist())


def test_prune_skips_none():
    knn = np.array([[1, 2, -1, -1], [0, 2, 3, -1], [1, 0, 3, -1], [2, 1, 0, -1]], np.int32)
    P = oracle.detour_prune(knn, 3)
    for x in range(4):
        assert x not in P[x]
        valid = [v for v in knn[x] if v >= 0]
        kept = [v for v in P[x] if v >= 0]
        assert kept == [v for v in kept if v in valid]
        assert len(kept) == min(3, len(valid))
    assert P[0].tolist()[2] == -1


@pytest.mark.parametrize("R", [4, 5, 16])
def test_reverse_combine_invariants(R):
    P = synthdata.random_graph(500, R, seed=R, n_none=1)
    F = oracle.reverse_combine(P)
    h = (R + 1) // 2
    n = len(P)
    fwd = {(x, int(y)) for x in range(n) for y in P[x] if y >= 0}
    for y in range(n):
        row = [v for v in F[y].tolist() if v >= 0]
        assert y not in row
        assert len(row) == len(set(row))
        # the first h valid forward entries lead
        lead = [v for v in P[y, :h].tolist() if v >= 0]
        assert row[:len(lead)] == lead
        for v in row:
            assert (y, v) in fwd or (v, y) in fwd     # forward or reverse of a forward edge
        nvalid = int((P[y] >= 0).sum())
        assert len(row) >= min(R, nvalid)


def test_merge_of_identical_shards_is_identity():
    n, R = 60, 6
    g = synthdata.random_graph(n, R, seed=4)
    off = [0, n, 2 * n]
    mem = np.concatenate([np.arange(n), np.arange(n)]).astype(np.int32)
    graphs = np.concatenate([g, g])
    out, deg = oracle.merge(off, mem, graphs, R, n, 2 * R)
    np.testing.assert_array_equal(out[:, :R], g)
    assert (out[:, R:] == -1).all()
    assert (deg == R).all()


def test_merge_invariants_overlapping_windows():
    sizes = np.array([40, 55, 30, 70], np.int64)
    N, off, mem = synthdata.overlapping_windows(sizes, overlap=0.25)
    R = 5
    graphs = np.concatenate([synthdata.random_graph(int(s), R, seed=10 + t, n_none=1)
                             for t, s in enumerate(sizes)])
    for cap in (R, 2 * R, 3 * R):
        out, deg = oracle.merge(off, mem, graphs, R, N, cap)
        assert (deg <= cap).all()
        for gid in range(N):
            row = out[gid, :deg[gid]].tolist()
            assert gid not in row and len(set(row)) == len(row)
            assert (out[gid, deg[gid]:] == -1).all()
            shards = [t for t in range(len(sizes)) if gid in mem[off[t]:off[t + 1]]]
            union = []
            for t in shards:
                r = int(np.nonzero(mem[off[t]:off[t + 1]] == gid)[0][0])
                lst = [int(mem[off[t] + v]) for v in graphs[off[t] + r] if v >= 0]
                union += [v for v in lst if v not in union and v != gid]
                if len(shards) == 1:
                    assert row == lst[:cap]
            assert set(row) <= set(union)
            if cap >= len(union):
                assert set(row) == set(union)


def test_merge_drops_self_and_duplicates_from_malformed_lists():
    # a shard list naming the row's own local index, and a repeated id
    off = [0, 3]
    mem = np.array([0, 1, 2], np.int32)
    graphs = np.array([[0, 1, 1], [2, 0, -1], [1, 1, 0]], np.int32)
    out, deg = oracle.merge(off, mem, graphs, 3, 3, 3)
    assert out.tolist() == [[1, -1, -1], [2, 0, -1], [1, 0, -1]]
    assert deg.tolist() == [1, 2, 2]

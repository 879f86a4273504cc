"""Pins of the oracle's k-means partition, selective replication and search.

Pinned by: the Fig. 2 outcome of Sec. V-B (coordinates chosen to reproduce
it, tests/golden/fig2_assignment.json), the closed forms eps <= 1 => no
replicas and eps = inf, omega = 2 => nearest + second nearest, a hand-worked
1-D Lloyd run with an exact tie, two separated blobs with known means, the
non-increasing k-means objective, and for search: a hand-worked beam trace and
the reduction to brute force when the beam holds every vector.
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


def test_fig2_selective_replication():
    g = _gold("fig2_assignment.json")
    X = np.array(g["vectors"], np.float64)
    Cc = np.array(g["centroids"], np.float64)
    primary = np.array([0, 1, 2], np.int32)
    sel, counts = oracle.assign_replicas(X, Cc, primary, g["omega"], g["epsilon"], g["tau"])
    assert sel.tolist() == g["expected_selective"]
    assert counts.tolist() == [1, 1, 2]
    uni, counts = oracle.assign_replicas(X, Cc, primary, g["omega"], float("inf"), g["tau"])
    assert uni.tolist() == g["expected_replicate_once"]
    assert counts.tolist() == [2, 1, 3]


@pytest.mark.parametrize("eps", [0.5, 1.0])
def test_eps_at_most_one_gives_no_replicas(eps):
    X = synthdata.mixture(500, 6, 5, 0.6, seed=2).astype(np.float64)
    Cc, lab = oracle.kmeans(X, 5, 4, synthdata.init_rows(500, 5, 3))
    assign, counts = oracle.assign_replicas(X, Cc, lab, 3, eps)
    assert (assign[:, 1:] == -1).all()
    assert counts.sum() == 500


def test_eps_inf_omega2_is_second_nearest():
    X = synthdata.mixture(400, 5, 6, 0.5, seed=4).astype(np.float64)
    S = 6
    Cc, lab = oracle.kmeans(X, S, 5, synthdata.init_rows(400, S, 1))
    assign, _ = oracle.assign_replicas(X, Cc, lab, 2, float("inf"))
    D = ((X[:, None, :] - Cc[None, :, :]) ** 2).sum(-1)
    order = np.argsort(D, axis=1, kind="stable")
    np.testing.assert_array_equal(assign[:, 0], order[:, 0])
    np.testing.assert_array_equal(assign[:, 1], order[:, 1])


def test_kmeans_worked_example():
    g = _gold("kmeans_1d.json")
    X = np.array(g["points"], np.float64)
    for it, cent in enumerate(g["per_iteration_centroids"], start=1):
        Cc, lab = oracle.kmeans(X, 2, it, g["init_idx"])
        np.testing.assert_array_equal(Cc, np.array(cent))
    assert lab.tolist() == g["final_labels"]


def test_kmeans_two_blobs_exact_means():
    X = np.array([[0.0], [1.0], [2.0], [10.0], [11.0], [12.0]])
    Cc, lab = oracle.kmeans(X, 2, 3, [0, 3])
    assert Cc.ravel().tolist() == [1.0, 11.0]
    assert lab.tolist() == [0, 0, 0, 1, 1, 1]


def test_kmeans_objective_non_increasing_and_empty_cluster_kept():
    X = synthdata.mixture(600, 4, 8, 0.7, seed=8).astype(np.float64)
    init = synthdata.init_rows(600, 8, 2)
    prev = np.inf
    for it in range(0, 8):
        Cc, lab = oracle.kmeans(X, 8, it, init)
        obj = ((X - Cc[lab]) ** 2).sum()
        assert obj <= prev + 1e-9
        prev = obj
    # a centroid far from every point never gains members and stays put
    X2 = np.concatenate([X, [[1e6, 1e6, 1e6, 1e6]]])
    Cc, lab = oracle.kmeans(X2, 2, 3, [0, 600])
    assert Cc[1].tolist() == [1e6] * 4


def test_membership_sorted_and_counts():
    X = synthdata.mixture(300, 3, 4, 0.8, seed=6).astype(np.float64)
    Cc, prim, off, mem = oracle.partition(X, 4, 2, 5, synthdata.init_rows(300, 4, 0))
    assert off[-1] == len(mem) == 600
    for s in range(4):
        seg = mem[off[s]:off[s + 1]]
        assert (np.diff(seg) > 0).all()
        assert set(np.nonzero(prim == s)[0].tolist()) <= set(seg.tolist())


def test_search_worked_example():
    g = _gold("search_path.json")
    X = np.array(g["points"], np.float64)
    ids, dist = oracle.search(X, np.array(g["graph"], np.int32), np.array([g["query"]]),
                              g["topk"], g["L"], entry=g["entry"])
    assert ids[0].tolist() == g["expected_ids"]
    np.testing.assert_allclose(dist[0], g["expected_dist"], rtol=1e-12)


def test_search_full_beam_is_bruteforce():
    X = synthdata.mixture(200, 6, 4, 0.5, seed=12).astype(np.float64)
    knn, _ = oracle.knn(X, 8)
    graph = oracle.prune(knn, 6)
    Q = synthdata.mixture(20, 6, 4, 0.5, seed=12, stream=1).astype(np.float64)
    ids, dist = oracle.search(X, graph, Q, 10, 256)
    D = ((Q[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    # the pruned graph of a clustered set may be disconnected: compare within
    # the ids reachable from the medoid
    med = oracle.medoid(X)
    reach, stack = {med}, [med]
    while stack:
        v = stack.pop()
        for u in graph[v]:
            if u >= 0 and u not in reach:
                reach.add(int(u))
                stack.append(int(u))
    reach = np.array(sorted(reach))
    for q in range(len(Q)):
        order = reach[np.lexsort((reach, D[q, reach]))][:10]
        assert ids[q].tolist() == order.tolist()


def test_medoid_closed_form():
    X = np.array([[0.0, 0.0], [10.0, 0.0], [0.0, 10.0], [4.0, 4.0], [3.0, 3.0]])
    # mean = (3.4, 3.4): nearest row is (3,3)
    assert oracle.medoid(X) == 4


def test_radius_constraint_decides():
    g = _gold("fig2_assignment.json")["radius_case"]
    Cc = np.array(g["centroids"])
    for key in ("small_radius", "large_radius"):
        X = np.array(g["vectors_" + key])
        prim = np.array([0] + [1] * (len(X) - 1), np.int32)
        a, _ = oracle.assign_replicas(X, Cc, prim, 2, 1.2)
        assert a.tolist() == g["expected_" + key]


def test_search_beats_lth_not_first():
    g = _gold("search_path.json")
    X = np.array(g["points"], np.float64)
    ids, dist = oracle.search(X, np.array(g["graph"], np.int32), np.array([g["query2"]]),
                              g["topk"], g["L"], entry=g["entry"])
    assert ids[0].tolist() == g["expected_ids2"]
    np.testing.assert_allclose(dist[0], g["expected_dist2"], rtol=1e-12)

"""Pins of the oracle's exact kNN and re-rank (CPU only).

Pinned by: exact integer brute force in Python integers (no rounding at all),
the closed-form neighbour order of points on a line (including the tie rule),
scipy's cdist + lexsort, and invariants (no self, sorted rows, symmetric
distances, the K-th-distance bound, padding when the shard is smaller than K).
"""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
import synthdata


def _exact_int_knn(Xi, K, metric):
    """Brute force with Python integers: exact distances, (dist, id) order."""
    n = len(Xi)
    out = []
    for i in range(n):
        cand = []
        for j in range(n):
            if j == i:
                continue
            if metric == oracle.L2:
                dist = sum((a - b) * (a - b) for a, b in zip(Xi[i], Xi[j]))
            else:
                dist = -sum(a * b for a, b in zip(Xi[i], Xi[j]))
            cand.append((dist, j))
        cand.sort()
        row = [j for _, j in cand[:K]] + [-1] * max(0, K - len(cand))
        out.append(row)
    return np.array(out, np.int32)


@pytest.mark.parametrize("metric", [oracle.L2, oracle.IP])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_knn_matches_exact_integer_bruteforce(metric, seed):
    rng = np.random.default_rng(seed)
    n, d, K = 40, 5, 7
    # few distinct values -> many exact distance ties, decided by the id rule
    Xi = rng.integers(0, 4, size=(n, d))
    X64 = oracle.widen(Xi.astype(np.uint8))
    nbr, dist = oracle.knn(X64, K, metric)
    exp = _exact_int_knn(Xi.tolist(), K, metric)
    np.testing.assert_array_equal(nbr, exp)


def test_knn_line_closed_form():
    """Points i*e_0 on a line: neighbours of i are i-1, i+1, i-2, i+2, ...
    (equal distances go to the lower id), clipped at the ends."""
    n, d, K = 30, 3, 6
    X = np.zeros((n, d), np.float32)
    X[:, 0] = np.arange(n)
    nbr, dist = oracle.knn(oracle.widen(X), K, oracle.L2)
    for i in range(n):
        order = sorted((j for j in range(n) if j != i), key=lambda j: (abs(i - j), j))[:K]
        assert nbr[i].tolist() == order
        assert dist[i].tolist() == [float((i - j) ** 2) for j in order]


def test_knn_matches_scipy_lexsort():
    X = synthdata.mixture(300, 12, 4, 0.5, seed=5)
    X64 = oracle.widen(X)
    K = 10
    nbr, dist = oracle.knn(X64, K, oracle.L2)
    D = cdist(X64, X64, "sqeuclidean")
    for i in range(len(X)):
        ids = np.arange(len(X))
        m = ids != i
        order = np.lexsort((ids[m], D[i, m]))[:K]
        np.testing.assert_array_equal(nbr[i], ids[m][order])
        np.testing.assert_allclose(dist[i], D[i, m][order], rtol=1e-12, atol=1e-12)
    Dip = -(X64 @ X64.T)
    nbr2, _ = oracle.knn(X64, K, oracle.IP)
    for i in range(0, len(X), 7):
        ids = np.arange(len(X))
        m = ids != i
        order = np.lexsort((ids[m], Dip[i, m]))[:K]
        np.testing.assert_array_equal(nbr2[i], ids[m][order])


def test_knn_invariants_small_workload():
    X = synthdata.small_f32(n=1024)
    X64 = oracle.widen(X)
    K = 32
    nbr, dist = oracle.knn(X64, K, oracle.L2)
    n = len(X)
    for i in range(0, n, 37):
        row = nbr[i]
        assert i not in row
        assert len(set(row.tolist())) == K
        assert np.all(np.diff(dist[i]) >= 0)
        # symmetric distance, bit for bit
        j = int(row[3])
        d_ij = ((X64[i] - X64[j]) ** 2).sum()
        rows_j, dist_j = oracle.knn(X64, n - 1, oracle.L2, rows=[j])
        k = int(np.nonzero(rows_j[0] == i)[0][0])
        assert dist_j[0, k] == dist[i, 3]
        assert abs(d_ij - dist[i, 3]) <= 1e-12 * max(1.0, d_ij)
        # everything not selected is at or beyond the K-th (dist, id)
        full_ids, full_d = oracle.knn(X64, n - 1, oracle.L2, rows=[i])
        kth = (dist[i, K - 1], nbr[i, K - 1])
        for dd, jj in zip(full_d[0, K:], full_ids[0, K:]):
            assert (dd, jj) > kth


def test_knn_pads_small_shards():
    X = np.arange(12, dtype=np.float32).reshape(4, 3)
    nbr, dist = oracle.knn(oracle.widen(X), 6, oracle.L2)
    assert (nbr[:, 3:] == -1).all()
    assert np.isinf(dist[:, 3:]).all()
    assert (nbr[:, :3] >= 0).all()


def test_knn_row_subset_equals_full():
    X = synthdata.mixture(200, 8, 3, 0.4, seed=9)
    X64 = oracle.widen(X)
    full, fd = oracle.knn(X64, 9, oracle.L2)
    rows = np.array([5, 0, 199, 77])
    sub, sd = oracle.knn(X64, 9, oracle.L2, rows=rows)
    np.testing.assert_array_equal(sub, full[rows])
    np.testing.assert_array_equal(sd, fd[rows])


def test_widen_dtypes_exact():
    v = np.array([[0.5, -2.0, 65504.0, 6.103515625e-05, 5.960464477539063e-08]], np.float16)
    np.testing.assert_array_equal(oracle.widen(v), v.astype(np.float64))
    b = oracle.to_bf16(np.array([[1.5, -3.25, 1e30]], np.float32))
    np.testing.assert_array_equal(oracle.widen(b, oracle.BF16), oracle.from_bf16(b))
    u = np.array([[0, 255, 17]], np.uint8)
    np.testing.assert_array_equal(oracle.widen(u), u.astype(np.float64))


def test_rerank_with_all_candidates_equals_knn():
    X = synthdata.mixture(150, 10, 3, 0.4, seed=3)
    X64 = oracle.widen(X)
    n = len(X)
    cand = np.array([[j for j in range(n) if j != i][::-1] for i in range(n)], np.int32)
    nbr, dist = oracle.rerank(X64, cand, 12)
    exp, expd = oracle.knn(X64, 12)
    np.testing.assert_array_equal(nbr, exp)
    np.testing.assert_array_equal(dist, expd)


def test_rerank_skips_none_and_pads():
    X = np.arange(15, dtype=np.float32).reshape(5, 3)
    cand = np.array([[1, -1, 2], [-1, -1, -1], [0, 1, 3], [4, 2, -1], [3, -1, -1]], np.int32)
    nbr, dist = oracle.rerank(oracle.widen(X), cand, 2)
    assert nbr.tolist() == [[1, 2], [-1, -1], [1, 3], [2, 4], [3, -1]]
    assert np.isinf(dist[1]).all()


def test_pair_dist_line_and_knn_agree():
    n, d = 20, 2
    X = np.zeros((n, d), np.float32)
    X[:, 1] = np.arange(n)
    X64 = oracle.widen(X)
    rows = np.array([0, 3, 19, 5, -1])
    cols = np.array([19, 3, 0, 9, 2])
    got = oracle.pair_dist(X64, rows, cols)
    assert got[:4].tolist() == [361.0, 0.0, 361.0, 16.0] and np.isinf(got[4])
    assert oracle.pair_dist(X64, [2], [7], oracle.IP).tolist() == [-14.0]
    nbr, dist = oracle.knn(X64, 5)
    np.testing.assert_array_equal(oracle.pair_dist(X64, np.repeat(np.arange(n)[:, None], 5, 1), nbr), dist)


def test_rerank_skips_self_and_repeats():
    X = np.arange(12, dtype=np.float32).reshape(4, 3)
    cand = np.array([[0, 1, 1, 2], [1, 0, 3, -1], [3, 3, 2, 0], [2, 3, 1, 1]], np.int32)
    nbr, _ = oracle.rerank(oracle.widen(X), cand, 3)
    assert nbr.tolist() == [[1, 2, -1], [0, 3, -1], [3, 0, -1], [2, 1, -1]]

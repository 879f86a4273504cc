"""Pins of the oracle's blockwise-adaptive assignment (Sec. V-A, Sec. V-B,
Algorithm 1).

Pinned by: the hand-worked Fig. 2 capacity example (one vector per block
locks v3 out of its nearest cluster; one block with original vectors first
does not), a hand-worked two-block case where the replica threshold keeps
room for a dense cluster's later primaries (tests/golden/blockwise_capacity.json),
the reduction to the single-block rule (one block, no capacity, tau = 1), the
closed forms eps <= 1 => no replicas and eps = inf => the omega nearest
clusters, invariants (capacity respected, no repeated cluster, primary first),
and an independent pure-Python implementation on small integer inputs (where
every FP32 distance is exact).
"""
import json
import os

import numpy as np
import pytest

import oracle
import synthdata

GOLD = os.path.join(os.path.dirname(__file__), "golden")
INF = float("inf")


def _gold():
    with open(os.path.join(GOLD, "blockwise_capacity.json")) as f:
        return json.load(f)


def test_fig2_capacity_lock_out_and_its_fix():
    g = _gold()["fig2"]
    X, Cc = np.array(g["vectors"]), np.array(g["centroids"])
    a, counts = oracle.assign_blockwise(X, Cc, g["omega"], INF, block_rows=1, cap=g["cap"], adaptive=False)
    assert a.tolist() == g["expected_one_vector_per_block"]
    assert a[2, 0] != 2                                 # v3 locked out of c3
    a, counts = oracle.assign_blockwise(X, Cc, g["omega"], INF, block_rows=3, cap=g["cap"])
    assert a.tolist() == g["expected_one_block"]
    assert a[:, 0].tolist() == [0, 1, 2]                # every vector in its nearest cluster
    assert counts.tolist() == [2, 2, 2]


def test_threshold_keeps_room_for_dense_cluster():
    g = _gold()["threshold"]
    X, Cc = np.array(g["vectors"]), np.array(g["centroids"])
    a, _ = oracle.assign_blockwise(X, Cc, g["omega"], INF, block_rows=g["block_rows"], cap=g["cap"])
    assert a.tolist() == g["expected_adaptive"]
    a, _ = oracle.assign_blockwise(X, Cc, g["omega"], INF, block_rows=g["block_rows"], cap=g["cap"],
                                   adaptive=False)
    assert a.tolist() == g["expected_fixed"]


@pytest.mark.parametrize("eps", [1.2, 1.5, INF])
def test_one_block_without_capacity_is_the_single_block_rule(eps):
    X = synthdata.mixture(600, 8, 6, 0.5, seed=3).astype(np.float64)
    S = 6
    Cc, lab = oracle.kmeans(X, S, 5, synthdata.init_rows(600, S, 2))
    ref, rc = oracle.assign_replicas(X, Cc, lab, 3, eps, 1.0)
    got, gc = oracle.assign_blockwise(X, Cc, 3, eps, 1.0)
    diff = np.nonzero((ref != got).any(1))[0]
    # the single-block rule compares unsquared FP64 distances, this one squared
    # FP32 ones: they may differ only where a comparison is a near-tie
    D = np.sqrt(((X[:, None, :] - Cc[None, :, :]) ** 2).sum(-1))
    for i in diff:
        d = np.sort(D[i])
        r = np.array([np.sqrt(((X[lab == c] - Cc[c]) ** 2).sum(-1)).max() for c in range(S)])
        margins = np.concatenate([np.abs(D[i] / (eps * D[i, lab[i]]) - 1) if np.isfinite(eps) else [1.0],
                                  np.abs(D[i] / (eps * r) - 1) if np.isfinite(eps) else [1.0],
                                  np.abs(np.diff(d)) / d[1:]])
        assert margins.min() < 1e-5, i
    assert len(diff) <= 2


@pytest.mark.parametrize("eps", [0.5, 1.0])
def test_eps_at_most_one_gives_no_replicas(eps):
    X = synthdata.mixture(500, 6, 5, 0.6, seed=2).astype(np.float64)
    Cc, _ = oracle.kmeans(X, 5, 4, synthdata.init_rows(500, 5, 3))
    a, counts = oracle.assign_blockwise(X, Cc, 3, eps, 2.0, block_rows=64)
    assert (a[:, 1:] == -1).all()
    assert counts.sum() == 500


def test_eps_inf_without_capacity_is_the_omega_nearest():
    X = synthdata.mixture(400, 5, 6, 0.5, seed=4).astype(np.float64)
    Cc, _ = oracle.kmeans(X, 6, 5, synthdata.init_rows(400, 6, 1))
    a, _ = oracle.assign_blockwise(X, Cc, 3, INF, 3.0, block_rows=50)
    D = ((X[:, None, :].astype(np.float32) - Cc[None, :, :].astype(np.float32)) ** 2).sum(-1)
    order = np.argsort(D, axis=1, kind="stable")
    np.testing.assert_array_equal(a, order[:, :3])


@pytest.mark.parametrize("cap,adaptive", [(90, True), (90, False), (70, True)])
def test_invariants_with_capacity(cap, adaptive):
    n, S, omega = 500, 8, 3
    X = synthdata.mixture(n, 6, 8, 0.6, seed=8).astype(np.float64)
    Cc, _ = oracle.kmeans(X, S, 3, synthdata.init_rows(n, S, 4))
    a, counts = oracle.assign_blockwise(X, Cc, omega, 1.5, 2.0, block_rows=100, cap=cap, adaptive=adaptive)
    assert (a[:, 0] >= 0).all()
    for row in a:
        v = row[row >= 0]
        assert len(set(v.tolist())) == len(v)
        assert (row[len(v):] == -1).all()
    np.testing.assert_array_equal(counts, np.bincount(a[a >= 0], minlength=S))
    # a shard passes its capacity only through a primary placed when every
    # cluster was full (replicas never overflow), and sizes only grow
    if counts.max() > cap:
        assert counts.min() >= cap


def _py_blockwise(X, Cc, omega, eps, tau0, block_rows, cap, adaptive):
    """Algorithm 1 with the blockwise statistics, written out in plain Python
    loops over FP32 scalars (numpy float32), for integer inputs only (every
    squared distance is then an exact integer)."""
    f = np.float32
    n, S = len(X), len(Cc)
    d2 = [[f(sum((float(x) - float(c)) ** 2 for x, c in zip(X[i], Cc[k]))) for k in range(S)] for i in range(n)]
    size, prim, rep, R2 = [0] * S, [0] * S, [0] * S, [f(0)] * S
    out = [[-1] * omega for _ in range(n)]
    eps2 = f(eps) * f(eps)
    t = 0
    for b0 in range(0, n, block_rows):
        t += 1
        rows = range(b0, min(n, b0 + block_rows))
        order = {i: sorted(range(S), key=lambda k: (d2[i][k], k)) for i in rows}
        for i in rows:
            cand = [k for k in order[i] if cap == 0 or size[k] < cap]
            c = cand[0] if cand else order[i][0]
            out[i][0] = c
            size[c] += 1
            prim[c] += 1
            R2[c] = max(R2[c], d2[i][c])
        seen = min(n, b0 + block_rows)
        theta = [10 ** 18 if (cap == 0 or not adaptive) else max(0, cap - (-(-prim[c] * n // seen)))
                 for c in range(S)]
        tau = f(1) + (f(tau0) - f(1)) / f(t)
        et2 = eps2 * (tau * tau)
        for i in rows:
            c = out[i][0]
            got = 1
            for k in order[i]:
                if got >= omega:
                    break
                if k == c or (cap and size[k] >= cap) or rep[k] >= theta[k]:
                    continue
                if eps == INF or (d2[i][k] < eps2 * d2[i][c] and d2[i][k] < et2 * R2[k]):
                    out[i][got] = k
                    got += 1
                    size[k] += 1
                    rep[k] += 1
    return np.array(out), np.array(size)


@pytest.mark.parametrize("seed,block_rows,cap,eps,tau0,adaptive", [
    (0, 7, 0, 1.5, 2.0, True), (1, 5, 9, 1.5, 3.0, True), (2, 4, 8, INF, 1.0, True),
    (3, 6, 10, 2.0, 2.0, False), (4, 40, 12, 1.25, 1.0, True), (5, 3, 7, 1.5, 4.0, True)])
def test_against_plain_python(seed, block_rows, cap, eps, tau0, adaptive):
    rng = np.random.default_rng(seed)
    S = 5
    Cc = rng.integers(0, 40, size=(S, 3)).astype(np.float64)
    X = (Cc[rng.integers(0, S, size=40)] + rng.integers(-9, 10, size=(40, 3))).astype(np.float64)
    a, counts = oracle.assign_blockwise(X, Cc, 3, eps, tau0, block_rows=block_rows, cap=cap, adaptive=adaptive)
    pa, pc = _py_blockwise(X, Cc, 3, eps, tau0, block_rows, cap, adaptive)
    np.testing.assert_array_equal(a, pa)
    np.testing.assert_array_equal(counts, pc)


def test_partition_blockwise_membership_is_ascending():
    X = synthdata.mixture(300, 4, 4, 0.5, seed=6).astype(np.float64)
    C, prim, off, mem = oracle.partition_blockwise(X, 4, 2, 3, synthdata.init_rows(300, 4, 6), eps=1.5,
                                                   tau0=2.0, block_rows=64, cap=120)
    for s in range(4):
        seg = mem[off[s]:off[s + 1]]
        assert (np.diff(seg) > 0).all()
    assert (off[1:] - off[:-1]).max() <= 120

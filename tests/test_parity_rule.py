"""The floating-point parity rule itself, on the CPU.

The rule (tests/parity.py) must accept any list an FP32 computation of the
ranking key can produce -- checked here with numpy FP32 products, whose
summation order differs from the GPU's (the bound holds for any order) -- and
must reject plausible mistakes: a neighbour swapped for a farther row, a wrong
returned distance, an unsorted row, the row itself in its list.  Near-duplicate
unit rows under the inner product are included: there an FP32 dot product
cannot resolve the L2 form 2 - 2x.y to 1e-5, which is why the rule is a
rounding bound and not a fixed relative tolerance.
"""
import numpy as np
import pytest

import oracle
import synthdata
from parity import check_rows, fp32_bound, gamma


def _fp32_knn(X, K, metric):
    """Top-K by an FP32 key computed the way the GPU forms it (row constant
    dropped), ties to the smaller id; distances returned in FP32."""
    X32 = X.astype(np.float32)
    n = len(X32)
    if metric == oracle.L2:
        nrm = np.einsum("ij,ij->i", X32, X32).astype(np.float32)
        key = nrm[None, :] + np.float32(-2.0) * (X32 @ X32.T)
        out_add = nrm
    else:
        key = -(X32 @ X32.T)
        out_add = np.zeros(n, np.float32)
    key[np.arange(n), np.arange(n)] = np.inf
    ids = np.argsort(key, axis=1, kind="stable")[:, :K]      # stable: ties to the smaller id
    kk = np.take_along_axis(key, ids, 1)
    dist = (kk + out_add[:, None]).astype(np.float32)
    return ids.astype(np.int32), dist


def _near_duplicate_unit(n, d, seed):
    rng = np.random.default_rng(seed)
    base = rng.standard_normal((n // 4, d))
    X = np.repeat(base, 4, 0) + 1e-3 * rng.standard_normal((n, d))   # groups of 4 near-duplicates
    return (X / np.linalg.norm(X, axis=1, keepdims=True)).astype(np.float32)


def test_gamma_matches_definition():
    assert gamma(1) == pytest.approx(2.0 ** -24 / (1 - 2.0 ** -24))
    assert gamma(100) > 100 * 2.0 ** -24


@pytest.mark.parametrize("metric", [oracle.L2, oracle.IP])
def test_fp32_lists_pass(metric):
    X = synthdata.mixture(700, 48, 8, 0.3, seed=5)
    if metric == oracle.IP:
        X = synthdata.unit_rows(X)
    X64 = oracle.widen(X)
    onbr, odist = oracle.knn(X64, 24, metric)
    g, gd = _fp32_knn(X, 24, metric)
    assert check_rows(X64, np.arange(len(X)), g, gd, onbr, odist, metric) == []


def test_fp32_lists_pass_on_near_duplicates_under_ip():
    X = _near_duplicate_unit(400, 64, seed=2)
    X64 = oracle.widen(X)
    onbr, odist = oracle.knn(X64, 16, oracle.IP)
    g, gd = _fp32_knn(X, 16, oracle.IP)
    assert check_rows(X64, np.arange(len(X)), g, gd, onbr, odist, oracle.IP) == []
    # a fixed 1e-5 relative tolerance in the L2 form would reject FP32 lists
    # here: the rounding of the dot product is far larger than 1e-5 of 2 - 2x.y
    e = fp32_bound(X64, np.arange(len(X)), onbr[:, :1], oracle.IP)[:, 0]
    l2form = 2.0 + 2.0 * odist[:, 0]
    assert np.max(e / l2form) > 1e-5


def test_oracle_lists_pass():
    X = synthdata.mixture(500, 32, 6, 0.3, seed=9)
    X64 = oracle.widen(X)
    onbr, odist = oracle.knn(X64, 20)
    assert check_rows(X64, np.arange(len(X)), onbr, odist.astype(np.float32), onbr, odist) == []


def _case():
    X = synthdata.mixture(400, 32, 5, 0.3, seed=13)
    X64 = oracle.widen(X)
    onbr, odist = oracle.knn(X64, 16)
    g, gd = _fp32_knn(X, 16, oracle.L2)
    return X, X64, onbr, odist, g.copy(), gd.copy()


def test_rejects_a_farther_neighbour():
    X, X64, onbr, odist, g, gd = _case()
    far, _ = oracle.knn(X64, 40)
    r = 7
    g[r, -1] = far[r, -1]                     # the 40th neighbour in place of the 16th
    gd[r, -1] = oracle.pair_dist(X64, np.array([[r]]), g[r:r + 1, -1:])[0, 0]
    bad = check_rows(X64, np.arange(len(X)), g, gd, onbr, odist)
    assert [b[0] for b in bad] == [r]


def test_rejects_a_wrong_distance():
    X, X64, onbr, odist, g, gd = _case()
    r = 11
    e = fp32_bound(X64, np.array([r]), g[r:r + 1, 3:4])[0, 0]
    gd[r, 3] += 3.0 * e                       # three times the rounding bound of that pair
    gd[r, 3:] = np.maximum.accumulate(gd[r, 3:])
    bad = check_rows(X64, np.arange(len(X)), g, gd, onbr, odist)
    assert [b[0] for b in bad] == [r]


def test_rejects_unsorted_and_self():
    X, X64, onbr, odist, g, gd = _case()
    g[2, [0, 5]] = g[2, [5, 0]]
    gd[2, [0, 5]] = gd[2, [5, 0]]
    g[3, 0] = 3
    bad = dict(check_rows(X64, np.arange(len(X)), g, gd, onbr, odist))
    assert set(bad) == {2, 3}
    assert "self" in bad[3]


def test_rejects_a_swapped_position_without_distances():
    X, X64, onbr, odist, g, gd = _case()
    r = 5
    g[r, [0, 15]] = g[r, [15, 0]]             # nearest and 16th exchanged: position 0 far off
    bad = check_rows(X64, np.arange(len(X)), g, None, onbr, odist)
    assert [b[0] for b in bad] == [r]

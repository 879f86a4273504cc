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
from parity import check_rows, fp32_bound, fp8_group_truncation, gamma


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


def _fp8_model_knn(Xq, K):
    """Top-K L2 lists from keys formed as the FP8 instruction forms them
    (groups of 8 products, each truncated toward zero onto 2^(e-13) of its
    group's largest, group sums added to the FP32 accumulator 64 products at
    a time), over dequantised rows Xq; distances returned in FP32."""
    n, d = Xq.shape
    dp = (d + 63) // 64 * 64
    Z = np.zeros((n, dp))
    Z[:, :d] = Xq
    nrm = np.einsum("ij,ij->i", Xq.astype(np.float32), Xq.astype(np.float32)).astype(np.float32)
    key = np.repeat(nrm[None, :], n, 0).astype(np.float32)         # accumulator start ||y||^2
    for k0 in range(0, dp, 64):
        p = -2.0 * Z[:, None, k0:k0 + 64] * Z[None, :, k0:k0 + 64]  # exact products
        g = p.reshape(n, n, 8, 8)
        gmax = np.abs(g).max(-1, keepdims=True)
        _, e = np.frexp(gmax)
        grid = np.where(gmax > 0, np.ldexp(1.0, e - 1 - 13), 1.0)
        gs = (np.trunc(g / grid) * grid).sum((-1, -2))
        key = (key.astype(np.float64) + gs).astype(np.float32)
    key[np.arange(n), np.arange(n)] = np.inf
    ids = np.argsort(key, axis=1, kind="stable")[:, :K]
    dist = (np.take_along_axis(key, ids, 1) + nrm[:, None]).astype(np.float32)
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


def test_fp8_model_lists_pass_only_with_the_truncation_term():
    # rows whose elements span a wide range: the in-group truncation then
    # exceeds the FP32 rounding bound, and the rule needs its FP8 term
    rng = np.random.default_rng(3)
    X = synthdata.mixture(500, 80, 8, 0.5, seed=3) * np.exp(rng.uniform(-4, 4, (1, 80)))
    oq, os_ = oracle.quant_rows_fp8(X.astype(np.float32))
    Xq = oracle.from_fp8(oq) * os_[:, None].astype(np.float64)
    onbr, odist = oracle.knn(Xq, 16)
    g, gd = _fp8_model_knn(Xq, 16)
    assert check_rows(Xq, np.arange(len(Xq)), g, gd, onbr, odist, fp8=True) == []
    assert check_rows(Xq, np.arange(len(Xq)), g, gd, onbr, odist) != []
    # the FP8 term is still far below the spacing of distinct neighbours
    far, _ = oracle.knn(Xq, 40)
    g2, gd2 = g.copy(), gd.copy()
    g2[7, -1] = far[7, -1]
    gd2[7, -1] = oracle.pair_dist(Xq, np.array([[7]]), g2[7:8, -1:])[0, 0]
    assert [b[0] for b in check_rows(Xq, np.arange(len(Xq)), g2, gd2, onbr, odist, fp8=True)] == [7]


def test_fp8_truncation_term_on_hand_cases():
    # one group of 8 with products 1, 1.5 * 2^-13 and 2^-20: the grid is
    # 2^-13 (the largest product's exponent 0, less 13); each product is
    # charged min(|p|, grid), the key's factor 2 doubles it
    X = np.zeros((2, 16))
    X[0, :3] = [1.0, 1.5 * 2.0 ** -4, 2.0 ** -11]
    X[1, :3] = [1.0, 2.0 ** -9, 2.0 ** -9]
    t = fp8_group_truncation(X, np.array([0]), np.array([[1]]))[0, 0]
    assert t == 2.0 * (2.0 ** -13 + 2.0 ** -13 + 2.0 ** -20)
    # the same products in three groups: each is its group's largest, charged
    # one step of its own grid
    Y = np.zeros((2, 24))
    Y[0, [0, 8, 16]] = X[0, :3]
    Y[1, [0, 8, 16]] = X[1, :3]
    t = fp8_group_truncation(Y, np.array([0]), np.array([[1]]))[0, 0]
    assert t == 2.0 * (2.0 ** -13 + 2.0 ** -26 + 2.0 ** -33)
    # padding (id -1) is charged nothing here; fp32_bound turns it into +inf
    assert fp8_group_truncation(Y, np.array([0]), np.array([[-1]]))[0, 0] >= 0


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

"""Element-level parity of the operand preparation (the A1 step) against the
oracle's number formats, through sg_quantize_rows: BF16 bits (nearest even),
FP8 E4M3 codes with the per-row power-of-two scale, and the norm term; then
the reduced-precision distance kernel on those operands against the exact kNN
of the dequantised rows.

Crafted rows cover the corners a plausible mistake would hit: halfway values
(ties to even), values that round up into the next binade or from the
subnormal range to the smallest normal, saturation at 448, NaN, and rows whose
largest magnitude sits exactly on, or just above, a power-of-two multiple of
448 (where the scale exponent changes)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_10135_amd as sg
import synthdata
from parity import check_rows, fp8_group_truncation, gamma

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _bits32(u):
    return np.array(u, np.uint32).view(np.float32)


def _bf16_rows():
    rng = np.random.default_rng(1)
    R = rng.standard_normal((64, 40)).astype(np.float32) * np.float32(3.0)
    # halfway cases: low 16 bits exactly 0x8000 over even and odd upper halves
    R[0, :8] = _bits32([0x3F808000, 0x3F818000, 0xBF808000, 0xBF818000,
                        0x3F80FFFF, 0x3F807FFF, 0x7F7F8000, 0x00018000])
    R[1, :6] = _bits32([0x7FC00001, 0xFF800000, 0x7F800000, 0x00000001, 0x80000000, 0x7F7FFFFF])
    return R


def test_bf16_bits_against_oracle():
    X = _bf16_rows()
    q, sexp, sq = sg.sg_quantize_rows(torch.from_numpy(X).to(DEV), "bf16", ldo=48)
    torch.cuda.synchronize()
    got = q.cpu().numpy().view(np.uint16)
    np.testing.assert_array_equal(got[:, :40], oracle.to_bf16(X))
    assert (got[:, 40:] == 0).all()
    assert sexp is None


def _fp8_rows():
    rng = np.random.default_rng(2)
    X = (rng.standard_normal((48, 64)) * 5.0).astype(np.float32)
    # amax exactly 448 * 2^e: scale 2^e, the extreme element maps to code 0x7e
    for r, e in enumerate((-3, 0, 2, 7)):
        X[r] = np.clip(X[r], -100, 100) * np.float32(2.0 ** e) / np.float32(4.0)
        X[r, 5] = np.float32(448.0 * 2.0 ** e)
    # amax just above 448 * 2^e: the scale doubles
    for r, e in enumerate((-2, 1, 3), start=4):
        X[r] = np.clip(X[r], -10, 10)
        X[r, 9] = np.nextafter(np.float32(448.0 * 2.0 ** e), np.float32(np.inf))
    # scale 1 (amax 448): halfway values between neighbouring E4M3 codes
    X[8] = 0.0
    X[8, 0] = 448.0
    X[8, 1:9] = [1.0625, 1.1875, 0.53125, 0.59375, 17.0, 19.0, 232.0, 240.0]
    # subnormal spacing 2^-9: 0.5, 1.5, 2.5, 7.5 units round to even; 7.5 -> 8 = smallest normal
    X[8, 9:14] = np.array([0.5, 1.5, 2.5, 7.5, 7.49], np.float32) * np.float32(2.0 ** -9)
    X[8, 14:18] = [-1.0625, -17.0, 447.0, 435.0]
    X[9] = 0.0                                           # all-zero row: scale 2^0
    X[10, 3] = np.float32("nan")                         # NaN: ignored by the scale, code 0x7f
    return X


def test_fp8_codes_and_scales_against_oracle():
    X = _fp8_rows()
    q, sexp, sq = sg.sg_quantize_rows(torch.from_numpy(X).to(DEV), "fp8", ldo=64)
    torch.cuda.synchronize()
    oq, os_ = oracle.quant_rows_fp8(X)
    np.testing.assert_array_equal(q.cpu().numpy(), oq)
    np.testing.assert_array_equal(np.ldexp(np.float32(1.0), sexp.cpu().numpy()), os_)
    # the corner rows landed where intended
    assert [int(e) for e in sexp.cpu().numpy()[:7]] == [-3, 0, 2, 7, -1, 2, 4]
    assert oq[8, 12] == 0x08 and oq[8, 0] == 0x7E


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_norm_term_within_fp32_bound(prec):
    X = synthdata.mixture(300, 96, 6, 0.3, seed=4)
    q, sexp, sq = sg.sg_quantize_rows(torch.from_numpy(X).to(DEV), prec)
    torch.cuda.synchronize()
    if prec == "bf16":
        Xq = oracle.from_bf16(oracle.to_bf16(X))
    else:
        oq, os_ = oracle.quant_rows_fp8(X)
        Xq = oracle.from_fp8(oq) * os_[:, None].astype(np.float64)
    n2 = (Xq * Xq).sum(1)
    assert np.all(np.abs(sq.cpu().numpy() - n2) <= gamma(96) * n2)


@pytest.mark.parametrize("prec", ["fp32", "f16"])
def test_exact_types_on_u8(prec):
    X = synthdata.sift_like_u8(n=200, d=100, seed=3)
    q, _, sq = sg.sg_quantize_rows(torch.from_numpy(X).to(DEV), prec, ldo=112)
    torch.cuda.synchronize()
    got = q.cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(got[:, :100], X.astype(np.float64))
    assert (got[:, 100:] == 0).all()
    np.testing.assert_array_equal(sq.cpu().numpy().astype(np.float64), (X.astype(np.float64) ** 2).sum(1))


def _wide_range_rows(n, d, seed):
    # a mixture whose columns are scaled by e^U(-4, 4): products within a
    # group of 8 elements then span many binades
    rng = np.random.default_rng(seed)
    return (synthdata.mixture(n, d, 10, 0.5, seed=seed) * np.exp(rng.uniform(-4, 4, (1, d)))).astype(np.float32)


@pytest.mark.parametrize("prec,family,d", [("bf16", "mixture", 64), ("fp8", "mixture", 64),
                                           ("fp8", "wide", 80), ("fp8", "deep", 96), ("fp8", "laion", 768)])
def test_reduced_key_knn_equals_exact_knn_of_dequantised_rows(prec, family, d):
    """Without a re-rank, the BF16 / FP8 distance kernel ranks the rows it
    quantised: its lists must be the exact kNN of the dequantised rows under
    the rounding-bound rule.  Products of BF16 or scaled FP8 values are exact;
    BF16 sums round as FP32 does, the FP8 instruction adds its in-group
    truncation (the rule's FP8 term)."""
    if family == "mixture":
        X = synthdata.mixture(2500, d, 20, 0.3, seed=31)
    elif family == "wide":
        X = _wide_range_rows(2500, d, seed=3)
    elif family == "deep":
        X = synthdata.deep_like_unit(3000, d, seed=23)
    else:
        X = synthdata.laion_like_f16(2000, d, seed=5, n_comp=40).astype(np.float32)
    K = 24
    nbr, dist = sg.sg_knn_graph(torch.from_numpy(X).to(DEV), K, "l2", prec)
    torch.cuda.synchronize()
    if prec == "bf16":
        Xq = oracle.from_bf16(oracle.to_bf16(X))
    else:
        oq, os_ = oracle.quant_rows_fp8(X)
        Xq = oracle.from_fp8(oq) * os_[:, None].astype(np.float64)
    onbr, odist = oracle.knn(Xq, K)
    bad = check_rows(Xq, np.arange(len(X)), nbr.cpu().numpy(), dist.cpu().numpy(), onbr, odist,
                     fp8=prec == "fp8")
    assert not bad, bad[:5]


# (row x, row y, returned distance minus the exact one): rows whose FP8 codes
# are exact (scale 2^-8, every value a code), so that the only departure from
# the exact distance is the instruction's in-group truncation of -2 x.y
_FP8_GROUP_CASES = [
    # -3 * 2^-13 shares a group with -2: grid 2^-12, truncated toward zero to -2^-12
    ({0: 1.0, 1: 1.5 * 2.0 ** -4}, {0: 1.0, 1: 2.0 ** -9}, 2.0 ** -13),
    # the same products in different groups of 8: each exact
    ({0: 1.0, 8: 1.5 * 2.0 ** -4}, {0: 1.0, 8: 2.0 ** -9}, 0.0),
    # a positive -2 x_t y_t truncates toward zero as well: the key shrinks
    ({0: 1.0, 1: -1.5 * 2.0 ** -4}, {0: 1.0, 1: 2.0 ** -9}, -(2.0 ** -13)),
    # -2^-19 is below the grid: lost whole
    ({0: 1.0, 7: 2.0 ** -11}, {0: 1.0, 7: 2.0 ** -9}, 2.0 ** -19),
    # the group boundary sits between elements 7 and 8 of the row
    ({0: 1.0, 8: 2.0 ** -11}, {0: 1.0, 8: 2.0 ** -9}, 0.0),
    # a group in the row's second half (element 40 is on the other lane half)
    ({40: 1.0, 47: 1.5 * 2.0 ** -4}, {40: 1.0, 47: 2.0 ** -9}, 2.0 ** -13),
]


@pytest.mark.parametrize("case", range(len(_FP8_GROUP_CASES)))
def test_fp8_instruction_truncates_within_groups_of_eight(case):
    """Pins the FP8 term of the parity rule through the product path: on a
    pair of rows the returned distance departs from the exact one by exactly
    the truncation the stated instruction model predicts, and not at all when
    the products fall in different groups."""
    xs, ys, delta = _FP8_GROUP_CASES[case]
    d = 64
    X = np.zeros((2, d), np.float32)
    for t, v in xs.items():
        X[0, t] = v
    for t, v in ys.items():
        X[1, t] = v
    oq, os_ = oracle.quant_rows_fp8(X)
    Xq = oracle.from_fp8(oq) * os_[:, None].astype(np.float64)
    assert np.array_equal(Xq, X.astype(np.float64)) and list(os_) == [2.0 ** -8, 2.0 ** -8]
    exact = float(((Xq[0] - Xq[1]) ** 2).sum())
    nbr, dist = sg.sg_knn_graph(torch.from_numpy(X).to(DEV), 1, "l2", "fp8")
    torch.cuda.synchronize()
    assert nbr.cpu().numpy().ravel().tolist() == [1, 0]
    got = dist.cpu().numpy().astype(np.float64).ravel()
    assert got.tolist() == [exact + delta, exact + delta], (got - exact, delta)
    # the rule's FP8 term covers the departure
    assert abs(delta) <= fp8_group_truncation(Xq, np.array([0]), np.array([[1]]))[0, 0]

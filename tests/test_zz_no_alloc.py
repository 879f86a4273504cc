"""sg_prune_noalloc, the prune on the library's static scratch (for callers
that cannot allocate), called through the C ABI: its output must equal
sg_prune's (the existing entry point, with a workspace) bit for bit, on two
calls in a row with the second smaller (the scratch keeps the first call's
contents), with and without a row order, and at the widest degree; sizes
beyond the scratch are refused on the host."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import paper_2605_10135_amd as sg
import synthdata

DEV = "cuda:0"


def _near_graph(n, K, seed):
    """n x K distinct ids != row, each within +-2K of the row (mod n)."""
    rng = np.random.default_rng(seed)
    w = 2 * K
    off = np.argsort(rng.random((n, w)), axis=1)[:, :K] + 1
    sign = np.where(rng.random((n, K)) < 0.5, -1, 1)
    return ((np.arange(n)[:, None] + sign * off) % n).astype(np.int32)


def _noalloc(knn, R, order=None):
    L = sg.lib()
    n, K = knn.shape
    out = torch.full((n, R), -7, dtype=torch.int32, device=DEV)
    torch.cuda.synchronize()
    rc = L.sg_prune_noalloc(C.c_void_p(knn.data_ptr()), n, K, R,
                            C.c_void_p(order.data_ptr()) if order is not None else None,
                            C.c_void_p(out.data_ptr()), None)
    assert rc == 0, L.sg_last_error()
    torch.cuda.synchronize()
    return out


@pytest.mark.gpu
def test_noalloc_equals_prune_on_two_calls_second_smaller():
    big = torch.from_numpy(_near_graph(120_000, 64, seed=1)).to(DEV)
    order = torch.from_numpy(np.random.default_rng(2).permutation(120_000).astype(np.int32)).to(DEV)
    got = _noalloc(big, 32, order)
    ref = sg.sg_prune(big, 32, order=order)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    small_h = synthdata.random_graph(3000, 24, seed=3, n_none=4)
    small = torch.from_numpy(small_h).to(DEV)
    got2 = _noalloc(small, 12)
    ref2 = sg.sg_prune(small, 12)
    torch.cuda.synchronize()
    assert torch.equal(got2, ref2)
    np.testing.assert_array_equal(got2.cpu().numpy(), oracle.prune(small_h, 12))


@pytest.mark.gpu
def test_noalloc_widest_degree_and_repeat():
    g = torch.from_numpy(_near_graph(20_000, 256, seed=4)).to(DEV)
    a = _noalloc(g, 128)
    b = _noalloc(g, 128)
    ref = sg.sg_prune(g, 128)
    torch.cuda.synchronize()
    assert torch.equal(a, ref) and torch.equal(b, ref)


def test_noalloc_refuses_sizes_beyond_the_scratch():
    # checked on the host before anything touches a device
    L = sg.lib()
    rc = L.sg_prune_noalloc(C.c_void_p(1), 300_000, 64, 32, None, C.c_void_p(1), None)
    assert rc == -1
    assert b"static scratch" in L.sg_last_error()
    need = C.c_size_t(0)
    assert L.sg_prune_workspace_size(300_000, 64, 32, C.byref(need)) == 0
    assert need.value > 128 << 20

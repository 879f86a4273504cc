"""Plain FP64 CPU oracle for the per-shard kNN-graph build (ScaleGANN).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may use this package; the product path never does.  It wraps
``oracle.c`` (plain C + OpenMP, FP64) with numpy arrays and shares nothing with
the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

NONE = -1
L2, IP = 0, 1
F32, F16, BF16, U8 = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (FP64, no fast-math)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-Wno-unused-function", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build()
            _lib = C.CDLL(_LIB_PATH)
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s rejected its arguments (rc=%d)" % (what, rc))


def _i64(v):
    return C.c_int64(int(v))


def num_threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(_load().orc_num_threads())


# ---------------------------------------------------------------------------
# inputs
# ---------------------------------------------------------------------------

def widen(X, dtype: int | None = None) -> np.ndarray:
    """Stored rows (float32 / float16 / bf16-as-uint16 / uint8) to FP64.

    bf16 arrays must be passed as uint16 with ``dtype=BF16``.
    """
    X = np.ascontiguousarray(X)
    if dtype is None:
        dtype = {np.dtype(np.float32): F32, np.dtype(np.float16): F16,
                 np.dtype(np.uint8): U8}[X.dtype]
    n, d = X.shape
    out = np.empty((n, d), np.float64)
    _check(_load().orc_widen(_p(X), C.c_int(dtype), _i64(n), C.c_int(d), _i64(d), _p(out)),
           "widen")
    return out


# ---------------------------------------------------------------------------
# graph build
# ---------------------------------------------------------------------------

def knn(X64: np.ndarray, K: int, metric: int = L2, rows=None):
    """Exact kNN lists: (nbr int32 [nrows, K], dist float64 [nrows, K])."""
    X64 = np.ascontiguousarray(X64, np.float64)
    n, d = X64.shape
    if rows is None:
        nrows, rp = n, None
    else:
        rows = np.ascontiguousarray(rows, np.int64)
        nrows, rp = rows.shape[0], rows
    nbr = np.empty((nrows, K), np.int32)
    dist = np.empty((nrows, K), np.float64)
    _check(_load().orc_knn(_p(X64), _i64(n), C.c_int(d), C.c_int(metric), C.c_int(K),
                           _p(rp), _i64(nrows), _p(nbr), _p(dist)), "knn")
    return nbr, dist


def pair_dist(X64: np.ndarray, rows, cols, metric: int = L2) -> np.ndarray:
    """delta(rows[p], cols[p]) in FP64; -1 in either gives +inf."""
    X64 = np.ascontiguousarray(X64, np.float64)
    n, d = X64.shape
    pairs = np.ascontiguousarray(np.stack([np.asarray(rows, np.int64).ravel(),
                                           np.asarray(cols, np.int64).ravel()], 1))
    out = np.empty((pairs.shape[0],), np.float64)
    _check(_load().orc_pair_dist(_p(X64), _i64(n), C.c_int(d), C.c_int(metric), _p(pairs),
                                 _i64(pairs.shape[0]), _p(out)), "pair_dist")
    return out.reshape(np.shape(cols))


def detour_prune(knn_ids: np.ndarray, R: int) -> np.ndarray:
    knn_ids = np.ascontiguousarray(knn_ids, np.int32)
    n, K = knn_ids.shape
    P = np.empty((n, R), np.int32)
    _check(_load().orc_detour_prune(_p(knn_ids), _i64(n), C.c_int(K), C.c_int(R), _p(P)),
           "detour_prune")
    return P


def reverse_combine(P: np.ndarray) -> np.ndarray:
    P = np.ascontiguousarray(P, np.int32)
    n, R = P.shape
    F = np.empty((n, R), np.int32)
    _check(_load().orc_reverse_combine(_p(P), _i64(n), C.c_int(R), _p(F)), "reverse_combine")
    return F


def prune(knn_ids: np.ndarray, R: int) -> np.ndarray:
    """Detour-count prune followed by the reverse-edge pass."""
    return reverse_combine(detour_prune(knn_ids, R))


def merge(offsets, member_ids, graphs, R: int, n_global: int, max_degree: int):
    off = np.ascontiguousarray(offsets, np.int64)
    mem = np.ascontiguousarray(member_ids, np.int32)
    g = np.ascontiguousarray(graphs, np.int32).reshape(-1)
    S = off.shape[0] - 1
    out = np.empty((n_global, max_degree), np.int32)
    deg = np.empty((n_global,), np.int32)
    _check(_load().orc_merge(C.c_int(S), _p(off), _p(mem), _p(g), C.c_int(R), _i64(n_global),
                             C.c_int(max_degree), _p(out), _p(deg)), "merge")
    return out, deg


# ---------------------------------------------------------------------------
# partition
# ---------------------------------------------------------------------------

def kmeans(X64: np.ndarray, S: int, iters: int, init_idx):
    X64 = np.ascontiguousarray(X64, np.float64)
    n, d = X64.shape
    init = np.ascontiguousarray(init_idx, np.int64)
    Cc = np.empty((S, d), np.float64)
    lab = np.empty((n,), np.int32)
    _check(_load().orc_kmeans(_p(X64), _i64(n), C.c_int(d), C.c_int(S), C.c_int(iters),
                              _p(init), _p(Cc), _p(lab)), "kmeans")
    return Cc, lab


def assign_replicas(X64, centroids, primary, omega: int, eps: float, tau: float = 1.0):
    X64 = np.ascontiguousarray(X64, np.float64)
    Cc = np.ascontiguousarray(centroids, np.float64)
    prim = np.ascontiguousarray(primary, np.int32)
    n, d = X64.shape
    S = Cc.shape[0]
    assign = np.empty((n, omega), np.int32)
    counts = np.empty((S,), np.int64)
    lib = _load()
    lib.orc_assign_replicas.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_void_p, C.c_int,
                                        C.c_void_p, C.c_int, C.c_double, C.c_double,
                                        C.c_void_p, C.c_void_p]
    _check(lib.orc_assign_replicas(_p(X64), n, d, _p(Cc), S, _p(prim), omega, float(eps),
                                   float(tau), _p(assign), _p(counts)), "assign_replicas")
    return assign, counts


def assign_blockwise(X64, centroids, omega: int, eps: float, tau0: float = 1.0, block_rows: int = 0,
                     cap: int = 0, adaptive: bool = True):
    """Blockwise-adaptive assignment (Sec. V-A/V-B, Algorithm 1): (assign n x
    omega, counts S).  block_rows <= 0 means one block of all rows; cap = 0
    means no size limit."""
    X64 = np.ascontiguousarray(X64, np.float64)
    Cc = np.ascontiguousarray(centroids, np.float64)
    n, d = X64.shape
    S = Cc.shape[0]
    assign = np.empty((max(n, 1), omega), np.int32)
    counts = np.empty((S,), np.int64)
    lib = _load()
    lib.orc_assign_blockwise.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_void_p, C.c_int, C.c_int,
                                         C.c_double, C.c_double, C.c_int64, C.c_int64, C.c_int,
                                         C.c_void_p, C.c_void_p]
    b = int(block_rows) if block_rows > 0 else max(n, 1)
    _check(lib.orc_assign_blockwise(_p(X64), n, d, _p(Cc), S, omega, float(eps), float(tau0), b, int(cap),
                                    int(bool(adaptive)), _p(assign), _p(counts)), "assign_blockwise")
    return assign[:n], counts


def partition_blockwise(X64, S: int, omega: int, iters: int, init_idx, eps: float = float("inf"),
                        tau0: float = 1.0, block_rows: int = 0, cap: int = 0, adaptive: bool = True):
    """k-means, then the blockwise-adaptive assignment and CSR membership:
    (centroids, primary, offsets, members)."""
    Cc, _ = kmeans(X64, S, iters, init_idx)
    assign, _ = assign_blockwise(X64, Cc, omega, eps, tau0, block_rows, cap, adaptive)
    off, mem = membership(assign, S)
    return Cc, assign[:, 0].copy(), off, mem


def membership(assign, S: int):
    a = np.ascontiguousarray(assign, np.int32)
    n, omega = a.shape
    off = np.empty((S + 1,), np.int64)
    total = int((a != NONE).sum())
    mem = np.empty((max(total, 1),), np.int32)
    _check(_load().orc_membership(_p(a), _i64(n), C.c_int(omega), C.c_int(S), _p(off), _p(mem)),
           "membership")
    return off, mem[:total]


def partition(X64, S: int, omega: int, iters: int, init_idx, eps: float = float("inf"),
              tau: float = 1.0):
    """k-means, primary = nearest centroid, selective replicas, CSR membership."""
    Cc, primary = kmeans(X64, S, iters, init_idx)
    assign, _ = assign_replicas(X64, Cc, primary, omega, eps, tau)
    off, mem = membership(assign, S)
    return Cc, primary, off, mem


# ---------------------------------------------------------------------------
# search / rerank
# ---------------------------------------------------------------------------

def medoid(X64) -> int:
    X64 = np.ascontiguousarray(X64, np.float64)
    n, d = X64.shape
    lib = _load()
    lib.orc_medoid.restype = C.c_int64
    return int(lib.orc_medoid(_p(X64), _i64(n), C.c_int(d)))


def search(X64, graph, Q64, topk: int, L: int, metric: int = L2, entry: int = -1):
    X64 = np.ascontiguousarray(X64, np.float64)
    Q64 = np.ascontiguousarray(Q64, np.float64)
    g = np.ascontiguousarray(graph, np.int32)
    n, d = X64.shape
    nq = Q64.shape[0]
    ids = np.empty((nq, topk), np.int32)
    dist = np.empty((nq, topk), np.float64)
    _check(_load().orc_search(_p(X64), _i64(n), C.c_int(d), C.c_int(metric), _p(g),
                              C.c_int(g.shape[1]), _p(Q64), _i64(nq), C.c_int(topk), C.c_int(L),
                              _i64(entry), _p(ids), _p(dist)), "search")
    return ids, dist


def rerank(X64, cand, K: int, metric: int = L2):
    X64 = np.ascontiguousarray(X64, np.float64)
    cand = np.ascontiguousarray(cand, np.int32)
    n, d = X64.shape
    c = cand.shape[1]
    nbr = np.empty((n, K), np.int32)
    dist = np.empty((n, K), np.float64)
    _check(_load().orc_rerank(_p(X64), _i64(n), C.c_int(d), C.c_int(metric), _p(cand),
                              C.c_int(c), C.c_int(K), _p(nbr), _p(dist)), "rerank")
    return nbr, dist


# ---------------------------------------------------------------------------
# number formats
# ---------------------------------------------------------------------------

def to_bf16(x) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float32)
    out = np.empty(x.shape, np.uint16)
    _check(_load().orc_to_bf16(_p(x), _i64(x.size), _p(out)), "to_bf16")
    return out


def from_bf16(b) -> np.ndarray:
    b = np.ascontiguousarray(b, np.uint16)
    out = np.empty(b.shape, np.float64)
    _check(_load().orc_from_bf16(_p(b), _i64(b.size), _p(out)), "from_bf16")
    return out


def to_fp8(x) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float32)
    out = np.empty(x.shape, np.uint8)
    _check(_load().orc_to_fp8e4m3(_p(x), _i64(x.size), _p(out)), "to_fp8")
    return out


def from_fp8(b) -> np.ndarray:
    b = np.ascontiguousarray(b, np.uint8)
    out = np.empty(b.shape, np.float64)
    _check(_load().orc_from_fp8e4m3(_p(b), _i64(b.size), _p(out)), "from_fp8")
    return out


def quant_rows_fp8(X):
    X = np.ascontiguousarray(X, np.float32)
    n, d = X.shape
    q = np.empty((n, d), np.uint8)
    s = np.empty((n,), np.float32)
    _check(_load().orc_quant_rows_fp8(_p(X), _i64(n), C.c_int(d), _p(q), _p(s)), "quant_rows_fp8")
    return q, s


# ---------------------------------------------------------------------------
# learned proposer
# ---------------------------------------------------------------------------

def _f64(a):
    return np.ascontiguousarray(a, np.float64)


def mlp_forward(X, W1, b1, W2, b2, mu, sigma: float):
    X, W1, b1, W2, b2, mu = map(_f64, (X, W1, b1, W2, b2, mu))
    n, D = X.shape
    H, E = W1.shape[0], W2.shape[0]
    F = np.empty((n, E), np.float64)
    lib = _load()
    lib.orc_mlp_forward.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_int] + \
        [C.c_void_p] * 5 + [C.c_double, C.c_void_p]
    _check(lib.orc_mlp_forward(_p(X), n, D, H, E, _p(W1), _p(b1), _p(W2), _p(b2), _p(mu),
                               float(sigma), _p(F)), "mlp_forward")
    return F


def mlp_loss_grad(Xa, Xp, W1, b1, W2, b2, mu, sigma: float, T: float):
    Xa, Xp, W1, b1, W2, b2, mu = map(_f64, (Xa, Xp, W1, b1, W2, b2, mu))
    B, D = Xa.shape
    H, E = W1.shape[0], W2.shape[0]
    loss = C.c_double(0.0)
    gW1 = np.empty_like(W1)
    gb1 = np.empty_like(b1)
    gW2 = np.empty_like(W2)
    gb2 = np.empty_like(b2)
    lib = _load()
    lib.orc_mlp_loss_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_int,
                                      C.c_int] + [C.c_void_p] * 5 + \
        [C.c_double, C.c_double, C.c_void_p] + [C.c_void_p] * 4
    _check(lib.orc_mlp_loss_grad(_p(Xa), _p(Xp), B, D, H, E, _p(W1), _p(b1), _p(W2), _p(b2),
                                 _p(mu), float(sigma), float(T), C.byref(loss), _p(gW1),
                                 _p(gb1), _p(gW2), _p(gb2)), "mlp_loss_grad")
    return loss.value, gW1, gb1, gW2, gb2


def adam(w, g, m, v, lr: float, beta1: float, beta2: float, eps: float, step: int):
    """One Adam step; returns new (w, m, v) as FP64 copies."""
    w, g, m, v = (np.array(a, np.float64, copy=True) for a in (w, g, m, v))
    lib = _load()
    lib.orc_adam.argtypes = [C.c_void_p] * 4 + [C.c_int64, C.c_double, C.c_double, C.c_double,
                                                C.c_double, C.c_int64]
    _check(lib.orc_adam(_p(w), _p(g), _p(m), _p(v), w.size, lr, beta1, beta2, eps, step),
           "adam")
    return w, m, v

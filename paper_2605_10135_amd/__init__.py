"""MI355X (gfx950) shard-graph build for divide-and-merge graph ANN indexing.

Thin Python binding over the C ABI of ``libsg.so`` (declared in include/sg.h).
Every function here only marshals arguments: torch tensors provide device
memory and the current HIP stream, and every step runs in the library's HIP
kernels.  There is no CPU fallback: if the library is not built, importing the
binding functions raises.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsg.so")

SG_NONE = -1
METRICS = {"l2": 0, "ip": 1}
PRECS = {"fp32": 0, "f16": 1, "bf16": 2, "fp8": 3, "i8": 4}
_DTYPES = {torch.float32: 0, torch.float16: 1, torch.bfloat16: 2, torch.uint8: 3}

_lib = None
_lock = threading.Lock()


class SgError(RuntimeError):
    def __init__(self, call, status, detail):
        super().__init__("%s failed: %s (%s)" % (call, status, detail))
        self.status = status


def lib():
    """Load libsg.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libsg.so not found at %s: build it with "
                                   "paper_2605_10135_amd.build.build()" % LIB_PATH)
            L = C.CDLL(LIB_PATH)
            _declare(L)
            _lib = L
    return _lib


vp, i32, i64, f32, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_size_t
psz = C.POINTER(C.c_size_t)

_SIGS = {
    "sg_status_str": (C.c_char_p, [i32]),
    "sg_last_error": (C.c_char_p, []),
    "sg_version": (C.c_char_p, []),
    "sg_partition_workspace_size": (i32, [i64, i32, i32, i32, psz]),
    "sg_partition": (i32, [vp, i32, i64, i32, i64, i32, i32, i32, f32, f32, vp, vp, vp, vp, vp,
                           i64, vp, sz, vp]),
    "sg_partition_blockwise_workspace_size": (i32, [i64, i32, i32, i32, i64, psz]),
    "sg_partition_blockwise": (i32, [vp, i32, i64, i32, i64, i32, i32, i32, f32, f32, i64, i64, i32, vp, vp,
                                     vp, vp, vp, i64, vp, sz, vp]),
    "sg_knn_graph_workspace_size": (i32, [i64, i32, i32, i32, i32, psz]),
    "sg_knn_graph": (i32, [vp, i32, i64, i32, i64, i32, i32, i32, i32, vp, vp, vp, vp, sz, vp]),
    "sg_knn_rows_workspace_size": (i32, [i64, i32, i64, i32, i32, i32, psz]),
    "sg_knn_rows": (i32, [vp, i32, i64, i32, i64, i32, vp, i64, i32, i32, i32, vp, vp, vp, sz, vp]),
    "sg_prune_workspace_size": (i32, [i64, i32, i32, psz]),
    "sg_prune": (i32, [vp, i64, i32, i32, vp, vp, vp, sz, vp]),
    "sg_prune_noalloc": (i32, [vp, i64, i32, i32, vp, vp, vp]),
    "sg_merge_workspace_size": (i32, [i32, vp, i64, psz]),
    "sg_merge": (i32, [i32, vp, vp, vp, i32, i64, i32, vp, vp, vp, sz, vp]),
    "sg_search_workspace_size": (i32, [i64, i32, i64, psz]),
    "sg_rerank": (i32, [vp, i32, i64, i32, i64, i32, vp, i32, i32, vp, vp, vp]),
    "sg_quantize_rows": (i32, [vp, i32, i64, i32, i64, i32, vp, i64, vp, vp, vp]),
    "sg_knn_variant_count": (i32, [i32, i32, i32, C.POINTER(C.c_int32)]),
    "sg_knn_autotune": (i32, [vp, i32, i64, i32, i64, i32, i32, i32, i32, vp, sz, vp, vp, vp, i32]),
    "sg_knn_force_variant": (i32, [i32]),
    "sg_knn_graph_batched_workspace_size": (i32, [vp, i32, i32, i32, i32, i32, i32, psz]),
    "sg_knn_graph_batched": (i32, [vp, i32, i32, i64, vp, i32, i32, i32, i32, i32, i32, vp, vp, vp, sz, vp,
                                   C.POINTER(C.c_void_p)]),
    "sg_batch_plan_destroy": (None, [vp]),
    "sg_knn_graph_batched_autotune": (i32, [vp, i32, i32, i64, vp, i32, i32, i32, i32, i32, i32, vp, vp, vp, sz,
                                            vp, C.POINTER(C.c_int32), vp, i32]),
    "sg_knn_graph_learned_workspace_size": (i32, [i64, i32, i32, psz]),
    "sg_knn_graph_learned": (i32, [vp, i32, i32, i64, i32, vp, i64, i32, i64, i32, i32, vp, vp, vp, sz, vp]),
    "sg_mlp_workspace_size": (i32, [i32, i32, i32, i32, psz]),
    "sg_mlp_project_workspace_size": (i32, [i32, i32, i32, psz]),
    "sg_mlp_stats": (i32, [vp, i64, i32, i64, vp, i64, vp, vp, vp, sz, vp]),
    "sg_mlp_loss_grad": (i32, [vp, i64, i32, i64, vp, vp, i32, i32, i32, vp, vp, vp, vp, vp, vp, f32, vp,
                               vp, vp, vp, vp, vp, sz, vp]),
    "sg_mlp_train": (i32, [vp, i64, i32, i64, vp, vp, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp,
                           f32, f32, f32, f32, f32, vp, i32, vp, sz, vp]),
    "sg_mlp_project": (i32, [vp, i64, i32, i64, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]),
    "sg_cost_model": (i32, [C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                            C.POINTER(C.c_double)]),
    "sg_sched_fit_linear": (i32, [vp, vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "sg_sched_simulate": (i32, [vp, vp, i32, vp, i32, i32, C.c_double, vp, vp, vp, vp, vp]),
    "sg_profile_begin": (i32, []),
    "sg_profile_end": (i32, [C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "sg_search": (i32, [vp, i32, i64, i32, i64, i32, vp, i32, vp, i64, i64, i32, i32, i64, vp, vp,
                        vp, sz, vp]),
}


def exported_symbols():
    """Names of the C ABI entry points this binding expects."""
    return sorted(_SIGS)


def _declare(L):
    for name, (res, args) in _SIGS.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args


def _check(call, rc):
    if rc != 0:
        L = lib()
        raise SgError(call, L.sg_status_str(rc).decode(), L.sg_last_error().decode())


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_tensor(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    return t


def _rows(X, name="X"):
    _dev_tensor(X, name)
    if X.dim() != 2:
        raise ValueError("%s must be 2-D" % name)
    if X.stride(1) != 1:
        raise ValueError("%s rows must be contiguous" % name)
    if X.dtype not in _DTYPES:
        raise TypeError("%s dtype %s not supported" % (name, X.dtype))
    return _DTYPES[X.dtype], X.shape[0], X.shape[1], X.stride(0)


class _Workspace:
    """Grow-only device workspace per (device, tag)."""

    def __init__(self):
        self.bufs = {}

    def get(self, nbytes, device, tag="default"):
        key = (str(device), tag)
        b = self.bufs.get(key)
        if b is None or b.numel() < nbytes:
            b = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
            self.bufs[key] = b
        return b


_ws = _Workspace()


def _size(fn, *args):
    out = C.c_size_t(0)
    _check(fn.__name__, fn(*args, C.byref(out)))
    return out.value


# ---------------------------------------------------------------------------
# calls
# ---------------------------------------------------------------------------

def sg_knn_graph(X, k, metric="l2", prec="fp32", rerank=0, dist=True, stream=None, out=None, order_out=None):
    """kNN graph of one shard: (nbr int32 [n,k], dist float32 [n,k] or None).
    order_out (optional int32 [n] tensor) receives the row order the build used,
    to pass to sg_prune."""
    L = lib()
    dt, n, d, ld = _rows(X)
    m, p = METRICS[metric], PRECS[prec]
    nbytes = _size(L.sg_knn_graph_workspace_size, n, d, k, p, rerank)
    ws = _ws.get(nbytes, X.device, "knn")
    if out is not None:
        nbr, dd = out
    else:
        nbr = torch.empty((n, k), dtype=torch.int32, device=X.device)
        dd = torch.empty((n, k), dtype=torch.float32, device=X.device) if dist else None
    if order_out is not None and (order_out.dtype != torch.int32 or order_out.numel() < n):
        raise ValueError("order_out must be an int32 tensor of n entries")
    _check("sg_knn_graph", L.sg_knn_graph(_ptr(X), dt, n, d, ld, m, k, p, rerank, _ptr(nbr), _ptr(dd),
                                          _ptr(order_out), _ptr(ws), ws.numel(), _stream(stream)))
    return nbr, dd


_OPERAND_DTYPES = {0: torch.float32, 1: torch.float16, 2: torch.int16, 3: torch.uint8, 4: torch.int8}


def sg_quantize_rows(X, prec="fp32", ldo=None, stream=None):
    """Operand rows of `prec` as the distance kernel prepares them:
    (rows [n, ldo] -- float32, float16, BF16 bits as int16, FP8 E4M3 codes as
    uint8 or U8 values - 128 as int8 --, scale exponents int32 [n] for FP8 else
    None, squared norms of the operand rows float32 [n])."""
    L = lib()
    dt, n, d, ld = _rows(X)
    p = PRECS[prec]
    ldo = d if ldo is None else int(ldo)
    out = torch.empty((n, ldo), dtype=_OPERAND_DTYPES[p], device=X.device)
    sexp = torch.empty(n, dtype=torch.int32, device=X.device) if prec == "fp8" else None
    sq = torch.empty(n, dtype=torch.float32, device=X.device)
    _check("sg_quantize_rows", L.sg_quantize_rows(_ptr(X), dt, n, d, ld, p, _ptr(out), ldo, _ptr(sexp), _ptr(sq),
                                                  _stream(stream)))
    return out, sexp, sq


def sg_knn_variant_count(d, k, prec="fp32"):
    """Number of distance-kernel variants for (prec, d, k)."""
    c = C.c_int32(0)
    _check("sg_knn_variant_count", lib().sg_knn_variant_count(PRECS[prec], d, k, C.byref(c)))
    return c.value


def sg_knn_autotune(X, k, metric="l2", prec="fp32", rerank=0, stream=None):
    """Time every distance-kernel variant on X and record the fastest for this
    shape: (chosen index, [milliseconds per variant])."""
    L = lib()
    dt, n, d, ld = _rows(X)
    m, p = METRICS[metric], PRECS[prec]
    ws = _ws.get(_size(L.sg_knn_graph_workspace_size, n, d, k, p, rerank), X.device, "knn")
    nv = sg_knn_variant_count(d, k, prec)
    times = (C.c_float * max(nv, 1))()
    chosen = C.c_int32(-1)
    _check("sg_knn_autotune", L.sg_knn_autotune(_ptr(X), dt, n, d, ld, m, k, p, rerank, _ptr(ws), ws.numel(),
                                                _stream(stream), C.byref(chosen), times, nv))
    return chosen.value, [float(times[i]) for i in range(nv)]


def sg_knn_force_variant(variant):
    """Make this thread's later kNN calls use variant `variant` (-1: the recorded choice)."""
    _check("sg_knn_force_variant", lib().sg_knn_force_variant(int(variant)))


class BatchPlan:
    """A captured batched build (HIP graph) for one fixed set of arguments;
    pass it to sg_knn_graph_batched again to replay.  Freed on close()/GC."""

    def __init__(self):
        self.ptr = C.c_void_p(None)

    def close(self):
        if self.ptr.value:
            lib().sg_batch_plan_destroy(self.ptr)
            self.ptr = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sg_knn_graph_batched(X, offsets, k, R, metric="l2", prec="fp32", knn=True, out=None, stream=None,
                         plan=None, rerank=0):
    """Pruned graphs (and kNN lists) of the shards X[offsets[s]:offsets[s+1]]:
    (graphs int32 [n, R], knn int32 [n, k] or None), ids local to each shard."""
    L = lib()
    dt, n, d, ld = _rows(X)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    S = off.size - 1
    offp = off.ctypes.data_as(C.c_void_p)
    m, p = METRICS[metric], PRECS[prec]
    nbytes = _size(L.sg_knn_graph_batched_workspace_size, offp, S, d, k, R, p, rerank)
    ws = _ws.get(nbytes, X.device, "batched")
    if out is not None:
        graphs, kn = out
    else:
        graphs = torch.empty((int(off[-1]), R), dtype=torch.int32, device=X.device)
        kn = torch.empty((int(off[-1]), k), dtype=torch.int32, device=X.device) if knn else None
    pp = C.byref(plan.ptr) if plan is not None else None
    _check("sg_knn_graph_batched", L.sg_knn_graph_batched(_ptr(X), dt, d, ld, offp, S, m, k, R, p, rerank,
                                                          _ptr(graphs),
                                                          _ptr(kn), _ptr(ws), ws.numel(), _stream(stream), pp))
    return graphs, kn


def sg_knn_graph_batched_autotune(X, offsets, k, R, metric="l2", prec="fp32", rerank=0, stream=None):
    """Time the batched pass per launch shape and record the fastest for
    batched calls of this shape: (chosen index, per-shape milliseconds)."""
    L = lib()
    dt, n, d, ld = _rows(X)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    S = off.size - 1
    offp = off.ctypes.data_as(C.c_void_p)
    m, p = METRICS[metric], PRECS[prec]
    nbytes = _size(L.sg_knn_graph_batched_workspace_size, offp, S, d, k, R, p, rerank)
    ws = _ws.get(nbytes, X.device, "batched")
    graphs = torch.empty((int(off[-1]), R), dtype=torch.int32, device=X.device)
    kn = torch.empty((int(off[-1]), k), dtype=torch.int32, device=X.device)
    nv = sg_knn_variant_count(d, rerank if rerank > k else k, prec)
    times = (C.c_float * max(nv, 1))()
    chosen = C.c_int32(-1)
    _check("sg_knn_graph_batched_autotune",
           L.sg_knn_graph_batched_autotune(_ptr(X), dt, d, ld, offp, S, m, k, R, p, rerank, _ptr(graphs), _ptr(kn),
                                           _ptr(ws), ws.numel(), _stream(stream), C.byref(chosen),
                                           C.cast(times, C.c_void_p), nv))
    return chosen.value, list(times)[:nv]


def sg_knn_rows(X, rows, k, metric="l2", prec="fp32", rerank=0, stream=None):
    """kNN of the listed rows of X against all rows: (nbr int32 [nq,k], dist float32 [nq,k])."""
    L = lib()
    dt, n, d, ld = _rows(X)
    r = torch.as_tensor(rows, dtype=torch.int64).to(X.device).contiguous()
    nq = r.numel()
    m, p = METRICS[metric], PRECS[prec]
    ws = _ws.get(_size(L.sg_knn_rows_workspace_size, n, d, nq, k, p, rerank), X.device, "knn_rows")
    nbr = torch.empty((nq, k), dtype=torch.int32, device=X.device)
    dd = torch.empty((nq, k), dtype=torch.float32, device=X.device)
    _check("sg_knn_rows", L.sg_knn_rows(_ptr(X), dt, n, d, ld, m, _ptr(r), nq, k, p, rerank, _ptr(nbr),
                                        _ptr(dd), _ptr(ws), ws.numel(), _stream(stream)))
    return nbr, dd


def sg_prune(knn, R, stream=None, out=None, order=None):
    """Detour-count prune + reverse-edge pass: int32 [n, R].  order: optional
    int32 [n] row permutation to process in (e.g. from sg_knn_graph)."""
    L = lib()
    _dev_tensor(knn, "knn")
    if knn.dtype != torch.int32 or not knn.is_contiguous():
        raise TypeError("knn must be a contiguous int32 tensor")
    n, K = knn.shape
    ws = _ws.get(_size(L.sg_prune_workspace_size, n, K, R), knn.device, "prune")
    o = out if out is not None else torch.empty((n, R), dtype=torch.int32, device=knn.device)
    if order is not None:
        _dev_tensor(order, "order")
        if order.dtype != torch.int32 or order.numel() != n:
            raise ValueError("order must be an int32 tensor of n entries")
    _check("sg_prune", L.sg_prune(_ptr(knn), n, K, R, _ptr(order), _ptr(o), _ptr(ws), ws.numel(),
                                  _stream(stream)))
    return o


def sg_prune_noalloc(knn, R, out, stream=None, order=None):
    """sg_prune on the library's static scratch (no workspace, no allocation
    in the call): the caller passes the int32 [n, R] output."""
    L = lib()
    _dev_tensor(knn, "knn")
    _dev_tensor(out, "out")
    if knn.dtype != torch.int32 or not knn.is_contiguous():
        raise TypeError("knn must be a contiguous int32 tensor")
    n, K = knn.shape
    if out.dtype != torch.int32 or not out.is_contiguous() or tuple(out.shape) != (n, R):
        raise ValueError("out must be a contiguous int32 tensor of shape (n, R)")
    if order is not None:
        _dev_tensor(order, "order")
        if order.dtype != torch.int32 or order.numel() != n:
            raise ValueError("order must be an int32 tensor of n entries")
    _check("sg_prune_noalloc", L.sg_prune_noalloc(_ptr(knn), n, K, R, _ptr(order), _ptr(out), _stream(stream)))
    return out


def sg_merge(shard_offsets, member_ids, graphs, R, n_global, max_degree, stream=None):
    """Edge-union merge: (out int32 [n_global, max_degree], degree int32 [n_global])."""
    L = lib()
    _dev_tensor(member_ids, "member_ids")
    _dev_tensor(graphs, "graphs")
    off = torch.as_tensor(shard_offsets, dtype=torch.int64).cpu().contiguous()
    S = off.numel() - 1
    offp = C.c_void_p(off.data_ptr())
    ws = _ws.get(_size(L.sg_merge_workspace_size, S, offp, n_global), member_ids.device, "merge")
    out = torch.empty((n_global, max_degree), dtype=torch.int32, device=member_ids.device)
    deg = torch.empty((n_global,), dtype=torch.int32, device=member_ids.device)
    _check("sg_merge", L.sg_merge(S, offp, _ptr(member_ids.contiguous()), _ptr(graphs.contiguous()), R,
                                  n_global, max_degree, _ptr(out), _ptr(deg), _ptr(ws), ws.numel(),
                                  _stream(stream)))
    return out, deg


def sg_partition(X, S, omega, iters, init_idx, epsilon=float("inf"), tau=1.0, stream=None):
    """k-means + selective replication: (centroids f64 [S,d], primary int32 [n],
    shard_offsets int64 [S+1] (host), member_ids int32 [total])."""
    L = lib()
    dt, n, d, ld = _rows(X)
    init = torch.as_tensor(init_idx, dtype=torch.int64).cpu().contiguous()
    ws = _ws.get(_size(L.sg_partition_workspace_size, n, d, S, omega), X.device, "partition")
    cent = torch.empty((S, d), dtype=torch.float64, device=X.device)
    prim = torch.empty((n,), dtype=torch.int32, device=X.device)
    off = torch.empty((S + 1,), dtype=torch.int64)
    cap = n * omega
    mem = torch.empty((cap,), dtype=torch.int32, device=X.device)
    _check("sg_partition", L.sg_partition(_ptr(X), dt, n, d, ld, S, omega, iters, float(epsilon),
                                          float(tau), C.c_void_p(init.data_ptr()), _ptr(cent),
                                          _ptr(prim), C.c_void_p(off.data_ptr()), _ptr(mem), cap,
                                          _ptr(ws), ws.numel(), _stream(stream)))
    return cent, prim, off, mem[: int(off[-1])]


def sg_partition_blockwise(X, S, omega, iters, init_idx, epsilon=float("inf"), tau0=1.0, block_rows=None,
                           shard_cap=0, adaptive=True, stream=None):
    """k-means + blockwise-adaptive assignment with selective replication:
    (centroids f64 [S,d], primary int32 [n], shard_offsets int64 [S+1] (host),
    member_ids int32 [total]).  block_rows None: one block of all rows."""
    L = lib()
    dt, n, d, ld = _rows(X)
    b = n if block_rows is None else int(block_rows)
    init = torch.as_tensor(init_idx, dtype=torch.int64).cpu().contiguous()
    ws = _ws.get(_size(L.sg_partition_blockwise_workspace_size, n, d, S, omega, b), X.device, "partition")
    cent = torch.empty((S, d), dtype=torch.float64, device=X.device)
    prim = torch.empty((n,), dtype=torch.int32, device=X.device)
    off = torch.empty((S + 1,), dtype=torch.int64)
    cap = n * omega
    mem = torch.empty((cap,), dtype=torch.int32, device=X.device)
    _check("sg_partition_blockwise",
           L.sg_partition_blockwise(_ptr(X), dt, n, d, ld, S, omega, iters, float(epsilon), float(tau0), b,
                                    int(shard_cap), int(bool(adaptive)), C.c_void_p(init.data_ptr()), _ptr(cent),
                                    _ptr(prim), C.c_void_p(off.data_ptr()), _ptr(mem), cap, _ptr(ws), ws.numel(),
                                    _stream(stream)))
    return cent, prim, off, mem[: int(off[-1])]


def sg_search(X, graph, Q, topk, L_beam, metric="l2", entry=-1, stream=None):
    """Greedy beam search: (ids int32 [nq, topk], dist float32 [nq, topk])."""
    L = lib()
    dt, n, d, ld = _rows(X)
    dq, nq, dq_, ldq = _rows(Q, "Q")
    if dq != dt or dq_ != d:
        raise ValueError("Q must match X in dtype and width")
    _dev_tensor(graph, "graph")
    graph = graph.contiguous()
    ws = _ws.get(_size(L.sg_search_workspace_size, n, d, nq), X.device, "search")
    ids = torch.empty((nq, topk), dtype=torch.int32, device=X.device)
    dist = torch.empty((nq, topk), dtype=torch.float32, device=X.device)
    _check("sg_search", L.sg_search(_ptr(X), dt, n, d, ld, METRICS[metric], _ptr(graph), graph.shape[1],
                                    _ptr(Q), nq, ldq, topk, L_beam, entry, _ptr(ids), _ptr(dist),
                                    _ptr(ws), ws.numel(), _stream(stream)))
    return ids, dist


def sg_profile_begin():
    """Start recording HIP events around each distance-kernel launch."""
    _check("sg_profile_begin", lib().sg_profile_begin())


def sg_profile_end():
    """(summed distance-kernel milliseconds, launches) since sg_profile_begin."""
    ms, n = C.c_double(0.0), C.c_int64(0)
    _check("sg_profile_end", lib().sg_profile_end(C.byref(ms), C.byref(n)))
    return ms.value, n.value


def sg_rerank(X, cand, k, metric="l2", stream=None):
    """Exact FP32 re-rank of candidate lists cand [n, c]: (nbr [n,k], dist [n,k])."""
    L = lib()
    dt, n, d, ld = _rows(X)
    _dev_tensor(cand, "cand")
    cand = cand.to(torch.int32).contiguous()
    c = cand.shape[1]
    nbr = torch.empty((n, k), dtype=torch.int32, device=X.device)
    dd = torch.empty((n, k), dtype=torch.float32, device=X.device)
    _check("sg_rerank", L.sg_rerank(_ptr(X), dt, n, d, ld, METRICS[metric], _ptr(cand), c, k, _ptr(nbr),
                                    _ptr(dd), _stream(stream)))
    return nbr, dd


def sg_knn_graph_learned(X, P, c, k, metric="l2", dist=True, stream=None, out=None):
    """kNN graph of X from the top-c FP8 proposals on projections P, re-ranked on X:
    (nbr int32 [n, k], dist float32 [n, k] or None)."""
    L = lib()
    dt, n, d, ld = _rows(X)
    _dev_tensor(P, "P")
    if P.dtype != torch.float32 or P.shape[0] != n or P.stride(1) != 1:
        raise ValueError("P must be an FP32 [n, e] tensor with unit column stride")
    e, ldp = P.shape[1], P.stride(0)
    ws = _ws.get(_size(L.sg_knn_graph_learned_workspace_size, n, e, c), X.device, "learned")
    if out is not None:
        nbr, dd = out
    else:
        nbr = torch.empty((n, k), dtype=torch.int32, device=X.device)
        dd = torch.empty((n, k), dtype=torch.float32, device=X.device) if dist else None
    _check("sg_knn_graph_learned", L.sg_knn_graph_learned(_ptr(X), dt, d, ld, METRICS[metric], _ptr(P), n, e, ldp,
                                                          c, k, _ptr(nbr), _ptr(dd), _ptr(ws), ws.numel(),
                                                          _stream(stream)))
    return nbr, dd


class MLP:
    """Device tensors of the learned proposer (FP32 masters + Adam moments)."""

    def __init__(self, W1, b1, W2, b2, mu, sigma):
        self.W1, self.b1, self.W2, self.b2 = (t.float().contiguous() for t in (W1, b1, W2, b2))
        self.mu = mu.float().contiguous()
        self.sigma = sigma.float().reshape(1).contiguous()
        self.H, self.D = self.W1.shape
        self.E = self.W2.shape[0]
        n = self.W1.numel() + self.b1.numel() + self.W2.numel() + self.b2.numel()
        self.m = torch.zeros(n, dtype=torch.float32, device=self.W1.device)
        self.v = torch.zeros(n, dtype=torch.float32, device=self.W1.device)


def sg_mlp_stats(X, rows, stream=None):
    """(mu [D], sigma [1]) of the listed rows of X (FP32)."""
    L = lib()
    _dev_tensor(X, "X")
    n, D = X.shape
    r = torch.as_tensor(rows, dtype=torch.int64).to(X.device).contiguous()
    mu = torch.empty(D, dtype=torch.float32, device=X.device)
    sigma = torch.empty(1, dtype=torch.float32, device=X.device)
    ws = _ws.get(4096, X.device, "mlp_stats")
    _check("sg_mlp_stats", L.sg_mlp_stats(_ptr(X), n, D, X.stride(0), _ptr(r), r.numel(), _ptr(mu), _ptr(sigma),
                                          _ptr(ws), ws.numel(), _stream(stream)))
    return mu, sigma


def sg_mlp_loss_grad(X, net, anchors, positives, T, stream=None):
    """(loss scalar tensor, gW1, gb1, gW2, gb2) for one batch."""
    L = lib()
    n, D = X.shape
    a = torch.as_tensor(anchors, dtype=torch.int64).to(X.device).contiguous()
    p = torch.as_tensor(positives, dtype=torch.int64).to(X.device).contiguous()
    B = a.numel()
    ws = _ws.get(_size(L.sg_mlp_workspace_size, B, D, net.H, net.E), X.device, "mlp")
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    g = [torch.empty_like(t) for t in (net.W1, net.b1, net.W2, net.b2)]
    _check("sg_mlp_loss_grad", L.sg_mlp_loss_grad(
        _ptr(X), n, D, X.stride(0), _ptr(a), _ptr(p), B, net.H, net.E, _ptr(net.W1), _ptr(net.b1),
        _ptr(net.W2), _ptr(net.b2), _ptr(net.mu), _ptr(net.sigma), float(T), _ptr(loss), _ptr(g[0]),
        _ptr(g[1]), _ptr(g[2]), _ptr(g[3]), _ptr(ws), ws.numel(), _stream(stream)))
    return (loss, *g)


def sg_mlp_train(X, net, anchors, positives, B, steps, T=0.05, lr=1e-3, betas=(0.9, 0.999), eps=1e-8,
                 use_graph=True, stream=None):
    """Run `steps` Adam steps in place on net; returns the per-step losses."""
    L = lib()
    n, D = X.shape
    a = torch.as_tensor(anchors, dtype=torch.int64).to(X.device).contiguous()
    p = torch.as_tensor(positives, dtype=torch.int64).to(X.device).contiguous()
    if a.numel() < B * steps or p.numel() < B * steps:
        raise ValueError("need B*steps anchors and positives")
    ws = _ws.get(_size(L.sg_mlp_workspace_size, B, D, net.H, net.E), X.device, "mlp")
    losses = torch.empty(steps, dtype=torch.float32, device=X.device)
    _check("sg_mlp_train", L.sg_mlp_train(
        _ptr(X), n, D, X.stride(0), _ptr(a), _ptr(p), B, steps, net.H, net.E, _ptr(net.W1), _ptr(net.b1),
        _ptr(net.W2), _ptr(net.b2), _ptr(net.m), _ptr(net.v), _ptr(net.mu), _ptr(net.sigma), float(T),
        float(lr), float(betas[0]), float(betas[1]), float(eps), _ptr(losses), 1 if use_graph else 0,
        _ptr(ws), ws.numel(), _stream(stream)))
    return losses


def sg_mlp_project(X, net, stream=None):
    """Unit-norm projections F [n, E] of every row of X."""
    L = lib()
    n, D = X.shape
    ws = _ws.get(_size(L.sg_mlp_project_workspace_size, D, net.H, net.E), X.device, "mlp_proj")
    F = torch.empty((n, net.E), dtype=torch.float32, device=X.device)
    _check("sg_mlp_project", L.sg_mlp_project(
        _ptr(X), n, D, X.stride(0), net.H, net.E, _ptr(net.W1), _ptr(net.b1), _ptr(net.W2), _ptr(net.b2),
        _ptr(net.mu), _ptr(net.sigma), _ptr(F), _ptr(ws), ws.numel(), _stream(stream)))
    return F


# ---------------------------------------------------------------------------
# scheduling shard builds on cloud GPU instances (host-only calls)
# ---------------------------------------------------------------------------
class SgInstance(C.Structure):
    _fields_ = [("ready", C.c_double), ("end", C.c_double), ("notice", C.c_double)]


def sg_cost_model(overall_time, gpu_active_time, transfer_time, cpu_price, gpu_price):
    """Cost of a build: (overall + transfer) x CPU price + (GPU active + transfer) x GPU price."""
    out = C.c_double(0.0)
    _check("sg_cost_model", lib().sg_cost_model(overall_time, gpu_active_time, transfer_time, cpu_price,
                                                gpu_price, C.byref(out)))
    return out.value


def sg_sched_fit_linear(sizes, times):
    """(a, b) of the least-squares line time = a + b * size."""
    x = np.ascontiguousarray(sizes, np.float64)
    y = np.ascontiguousarray(times, np.float64)
    a, b = C.c_double(0.0), C.c_double(0.0)
    _check("sg_sched_fit_linear", lib().sg_sched_fit_linear(x.ctypes.data, y.ctypes.data, len(x), C.byref(a),
                                                            C.byref(b)))
    return a.value, b.value


def sg_sched_simulate(est, actual, instances, time_based=True, transfer=0.0):
    """Simulate the task scheduler.  instances: sequence of (ready, end,
    notice).  Returns a dict: task_instance, task_start, task_end, attempts
    (numpy arrays), makespan, gpu_active, preemptions, completed."""
    est = np.ascontiguousarray(est, np.float64)
    actual = np.ascontiguousarray(actual, np.float64)
    T, G = len(est), len(instances)
    arr = (SgInstance * max(G, 1))(*[SgInstance(*map(float, t)) for t in instances])
    ti = np.empty(T, np.int32)
    t0 = np.empty(T, np.float64)
    t1 = np.empty(T, np.float64)
    att = np.empty(T, np.int32)
    summ = np.empty(4, np.float64)
    _check("sg_sched_simulate", lib().sg_sched_simulate(est.ctypes.data, actual.ctypes.data, T, C.cast(arr, C.c_void_p),
                                                        G, int(bool(time_based)), float(transfer), ti.ctypes.data,
                                                        t0.ctypes.data, t1.ctypes.data, att.ctypes.data,
                                                        summ.ctypes.data))
    return dict(task_instance=ti, task_start=t0, task_end=t1, attempts=att, makespan=float(summ[0]),
                gpu_active=float(summ[1]), preemptions=int(summ[2]), completed=int(summ[3]))

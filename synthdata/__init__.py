"""Seeded synthetic inputs for the per-shard kNN-graph build.

This module only draws data: Gaussian-mixture vectors with the shapes and
distributions of the paper's workloads (Table III shapes: 128-d uint8 like
Sift, 96-d float like Deep, 768-d like Laion), k-means seed rows, random
graphs for the integer passes, and the uneven shard windows of the batched
workload.  It holds none of the method's arithmetic, and both the GPU path's
tests and the CPU oracle consume the arrays it returns.

Recipe (all numpy PCG64): component of each row uniform over the mixture;
x = mu_c + sigma * N(0, I); rows generated in fixed chunks of CHUNK rows so
that memory stays bounded and the stream does not depend on machine size.
"""
from __future__ import annotations

import math

import numpy as np

CHUNK = 1 << 16


def _rng(seed: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([seed, stream]))


def mixture(n: int, d: int, n_comp: int, sigma: float, seed: int, *, centres: str = "normal",
            centre_lo: float = 0.0, centre_hi: float = 1.0, stream: int = 0,
            centres_seed_stream: int = 1000) -> np.ndarray:
    """n x d float32 rows from an n_comp-component Gaussian mixture.

    centres: "normal" -> N(0, I); "uniform" -> U[centre_lo, centre_hi]^d.
    The centres come from their own stream so that a second draw from the same
    mixture (held-out queries, ``stream`` != 0) shares them.
    """
    crng = _rng(seed, centres_seed_stream)
    if centres == "normal":
        mu = crng.standard_normal((n_comp, d)).astype(np.float32)
    elif centres == "uniform":
        mu = crng.uniform(centre_lo, centre_hi, (n_comp, d)).astype(np.float32)
    else:
        raise ValueError(centres)
    rng = _rng(seed, stream)
    out = np.empty((n, d), np.float32)
    for a in range(0, n, CHUNK):
        b = min(n, a + CHUNK)
        comp = rng.integers(0, n_comp, b - a)
        noise = rng.standard_normal((b - a, d), dtype=np.float32)
        out[a:b] = mu[comp] + np.float32(sigma) * noise
    return out


def unit_rows(X: np.ndarray) -> np.ndarray:
    """Scale each row to unit L2 norm (input preparation for the IP workloads)."""
    nrm = np.sqrt((X.astype(np.float64) ** 2).sum(1, keepdims=True))
    nrm[nrm == 0] = 1.0
    return (X / nrm).astype(np.float32)


def init_rows(n: int, S: int, seed: int) -> np.ndarray:
    """k-means seed rows: the first S of a seeded permutation of 0..n-1."""
    return _rng(seed, 7).permutation(n)[:S].astype(np.int64)


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

def small_f32(seed: int = 1000, n: int = 8192, d: int = 96) -> np.ndarray:
    """8192 x 96 FP32, 32-component mixture, centres N(0, 1), std 0.3."""
    return mixture(n, d, 32, 0.3, seed)


def sift_like_u8(n: int = 1_000_000, d: int = 128, seed: int = 1001, stream: int = 0,
                 n_comp: int = 1000) -> np.ndarray:
    """uint8 rows: clip(rint(mixture of 1000 Gaussians, centres U[0,200], std 12), 0, 255).

    np.rint rounds half to even.  stream=1 draws the held-out queries.
    """
    X = mixture(n, d, n_comp, 12.0, seed, centres="uniform", centre_lo=0.0, centre_hi=200.0,
                stream=stream)
    return np.clip(np.rint(X), 0, 255).astype(np.uint8)


def deep_like_unit(n: int = 4_000_000, d: int = 96, seed: int = 1002, n_comp: int = 2000,
                   sigma: float = 0.15, stream: int = 0) -> np.ndarray:
    """Unit-norm FP32 rows from a 2000-component mixture (std 0.15)."""
    out = np.empty((n, d), np.float32)
    for a in range(0, n, 1 << 20):
        b = min(n, a + (1 << 20))
        out[a:b] = unit_rows(mixture(b - a, d, n_comp, sigma, seed, stream=stream * 4096 + a))
    return out


def laion_like_f16(n: int, d: int = 768, seed: int = 1003, n_comp: int = 4000,
                   sigma: float = 0.15, stream: int = 0) -> np.ndarray:
    """Unit-norm rows rounded to FP16 (round to nearest even), 4000 components."""
    out = np.empty((n, d), np.float16)
    for a in range(0, n, 1 << 18):
        b = min(n, a + (1 << 18))
        out[a:b] = unit_rows(mixture(b - a, d, n_comp, sigma, seed,
                                     stream=stream * 4096 + a)).astype(np.float16)
    return out


def l1_nonneg(n: int, d: int = 960, seed: int = 1004, n_comp: int = 500, sigma: float = 0.2,
              stream: int = 0) -> np.ndarray:
    """abs(mixture of 500 Gaussians, std 0.2) scaled to unit L1 norm per row."""
    out = np.empty((n, d), np.float32)
    for a in range(0, n, 1 << 18):
        b = min(n, a + (1 << 18))
        X = np.abs(mixture(b - a, d, n_comp, sigma, seed, stream=stream * 4096 + a))
        s = X.astype(np.float64).sum(1, keepdims=True)
        s[s == 0] = 1.0
        out[a:b] = (X / s).astype(np.float32)
    return out


def batched_shard_sizes(n_shards: int = 64, seed: int = 1003, mu: float = math.log(1e5),
                        sigma: float = 0.8, lo: int = 20_000, hi: int = 500_000) -> np.ndarray:
    """Shard sizes lognormal(mu, sigma), rounded down, clipped to [lo, hi]."""
    s = _rng(seed, 11).lognormal(mu, sigma, n_shards)
    return np.clip(np.floor(s), lo, hi).astype(np.int64)


def overlapping_windows(sizes: np.ndarray, overlap: float = 0.25):
    """Shard t = window of sizes[t] consecutive ids starting at
    o_t = sum_{u<t} floor((1-overlap) * n_u) (mod N), N = sum_u floor((1-overlap) * n_u).

    Returns (N, offsets[S+1], member_ids ascending per shard)."""
    step = np.floor((1.0 - overlap) * sizes).astype(np.int64)
    N = int(step.sum())
    starts = np.concatenate([[0], np.cumsum(step)[:-1]])
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    mem = np.empty(int(offs[-1]), np.int32)
    for t, (o, m) in enumerate(zip(starts, sizes)):
        ids = (o + np.arange(m, dtype=np.int64)) % N
        mem[offs[t]:offs[t + 1]] = np.sort(ids).astype(np.int32)
    return N, offs, mem


# ---------------------------------------------------------------------------
# small random structures for the integer passes
# ---------------------------------------------------------------------------

def random_graph(n: int, K: int, seed: int, n_none: int = 0) -> np.ndarray:
    """n x K lists of distinct ids != row, drawn uniformly; the last n_none
    entries of some rows are set to -1 to exercise padding."""
    rng = _rng(seed, 3)
    g = np.empty((n, K), np.int32)
    for i in range(n):
        pool = rng.choice(n - 1, size=K, replace=False)
        pool = np.where(pool >= i, pool + 1, pool)
        g[i] = pool
    if n_none:
        rows = rng.choice(n, size=max(1, n // 8), replace=False)
        g[rows, K - n_none:] = -1
    return g


def local_graph(n: int, K: int, seed: int, window: int = 0) -> np.ndarray:
    """Lists biased to nearby ids (heavy mutual overlap, like a real kNN graph):
    ids drawn from a window around the row, distinct, != row."""
    rng = _rng(seed, 5)
    w = max(window, 2 * K + 2)
    g = np.empty((n, K), np.int32)
    for i in range(n):
        lo = max(0, min(i - w // 2, n - w))
        cand = np.arange(lo, min(n, lo + w))
        cand = cand[cand != i]
        g[i] = rng.choice(cand, size=K, replace=False)
    return g

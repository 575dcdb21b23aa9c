"""Seeded synthetic graph inputs shared by the oracle tests and the device path.

This module only produces inputs: edge lists, dense adjacency matrices with a
non-edge sentinel and a zero diagonal, and request streams.  It contains no
shortest-path arithmetic.

Every random draw comes from ``numpy.random.default_rng(SeedSequence([1902,
config_id, item_id]))`` so each workload is reproducible bit for bit.

Workload families (the paper's own inputs are Erdos-Renyi graphs, Sec. 5.1;
the n=16384 and n=65536 runs and the serving mix use a k-nearest-neighbour
graph over a noisy Swiss roll instead):

* ``er_edges``          G(n, p) over unordered pairs, integer weights
* ``swiss_roll_knn``    exact k-NN (k=10) over Swiss-roll points, union
                        symmetrised, fp32 Euclidean weights
* ``batched_sizes``     log-uniform sizes for the many-small-graphs batch
* ``serving_requests``  Poisson arrivals with a size mix
"""
from __future__ import annotations

import math

import numpy as np

INF_I32 = 1 << 30

# Workload identifiers used in the seed sequences.
CFG_PLAIN_SMALL = 1      # ER n=512, p=0.05, int32 U{1..100}
CFG_SWISS_16K = 2        # Swiss-roll kNN, n=16384, fp32
CFG_SWISS_64K = 3        # Swiss-roll kNN, n=65536, fp32
CFG_BATCHED = 4          # 4096 ER graphs, n log-uniform in [32, 512], p=8/n
CFG_SERVING = 5          # Poisson request stream, Swiss-roll kNN graphs
CFG_SWISS_256K = 6       # Swiss-roll kNN, n=262144, fp32 (256 GiB matrix)
CFG_TEST = 100           # ad-hoc test inputs


def rng_for(config_id: int, item_id: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([1902, int(config_id), int(item_id)]))


# --------------------------------------------------------------------------
# Edge lists: (u, v, w) with u < v, one entry per undirected edge.
# --------------------------------------------------------------------------

def er_edges(n: int, p: float, wlo: int, whi: int, rng: np.random.Generator):
    """Erdos-Renyi G(n, p): each unordered pair is an edge independently with
    probability p; integer weight uniform on {wlo..whi}."""
    if n < 2:
        z = np.zeros(0, np.int64)
        return z, z, np.zeros(0, np.int32)
    iu, ju = np.triu_indices(n, k=1)
    coin = rng.random(iu.size)
    w = rng.integers(wlo, whi + 1, size=iu.size, dtype=np.int64)
    keep = coin < p
    return iu[keep].astype(np.int64), ju[keep].astype(np.int64), w[keep].astype(np.int32)


def swiss_roll_points(n: int, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """Swiss roll: t = 1.5*pi*(1 + 2u), point (t cos t, 21 v, t sin t) + N(0, sigma^2 I)."""
    u = rng.random(n)
    v = rng.random(n)
    t = 1.5 * math.pi * (1.0 + 2.0 * u)
    pts = np.stack([t * np.cos(t), 21.0 * v, t * np.sin(t)], axis=1)
    pts += rng.normal(0.0, sigma, size=(n, 3))
    return pts


def knn_union_edges(points: np.ndarray, k: int):
    """Exact k-nearest-neighbour graph (self excluded), symmetrised by union.

    An unordered pair {i, j} is an edge if j is among the k nearest of i or i
    among the k nearest of j.  The weight is the fp64 Euclidean distance of the
    pair, rounded once to fp32, so both directions carry the same bits.
    """
    from scipy.spatial import cKDTree

    n = points.shape[0]
    if n < 2:
        z = np.zeros(0, np.int64)
        return z, z, np.zeros(0, np.float32)
    kk = min(k + 1, n)
    tree = cKDTree(points)
    _, idx = tree.query(points, k=kk)
    idx = np.asarray(idx, np.int64).reshape(n, kk)
    src = np.repeat(np.arange(n, dtype=np.int64), kk)
    dst = idx.ravel()
    keep = src != dst
    src, dst = src[keep], dst[keep]
    # at most k neighbours per source after removing self
    order = np.lexsort((np.arange(src.size), src))
    src, dst = src[order], dst[order]
    first = np.searchsorted(src, np.arange(n))
    rank = np.arange(src.size) - first[src]
    keep = rank < k
    src, dst = src[keep], dst[keep]
    u = np.minimum(src, dst)
    v = np.maximum(src, dst)
    key = np.unique(u * n + v)
    u = key // n
    v = key % n
    d = points[u] - points[v]
    w = np.sqrt(np.sum(d * d, axis=1)).astype(np.float32)
    return u, v, w


def swiss_roll_knn(n: int, config_id: int, item_id: int = 0, k: int = 10, sigma: float = 0.05):
    rng = rng_for(config_id, item_id)
    return knn_union_edges(swiss_roll_points(n, sigma, rng), k)


# --------------------------------------------------------------------------
# Dense adjacency matrices and CSR lists
# --------------------------------------------------------------------------

def with_hub_edges(n: int, u, v, w, K: int, rng: np.random.Generator):
    """The edges (u, v, w) plus a star from vertex 0 to vertices 1..K-1 and an
    edge from every vertex j >= K to vertex j % K, weights U[0.5, 1.5) fp32,
    dropping those that duplicate an existing edge.  After the first K
    pivots of Floyd-Warshall every pair is then joined by a path of a few
    hops, so every entry of the matrix holds a finite length."""
    j = np.arange(K, n, dtype=np.int64)
    hu = np.concatenate([np.zeros(K - 1, dtype=np.int64), j])
    hv = np.concatenate([np.arange(1, K, dtype=np.int64), j % K])
    hw = rng.uniform(0.5, 1.5, size=hu.size).astype(np.float32)
    u, v = np.asarray(u, np.int64), np.asarray(v, np.int64)
    key = np.minimum(u, v) * n + np.maximum(u, v)
    hkey = np.minimum(hu, hv) * n + np.maximum(hu, hv)
    keep = ~np.isin(hkey, key)
    return (np.concatenate([u, hu[keep]]), np.concatenate([v, hv[keep]]),
            np.concatenate([np.asarray(w, np.float32), hw[keep]]))


def dense_from_edges(n: int, u, v, w, dtype, ld: int | None = None) -> np.ndarray:
    """Dense n x n (row-major, leading dimension ``ld``) adjacency matrix.

    Non-edges hold the sentinel (2**30 for int32, +inf for float32), the
    diagonal holds 0, and each edge is written in both directions.  Returns the
    full n x ld buffer's n x n view.
    """
    ld = n if ld is None else ld
    dtype = np.dtype(dtype)
    fill = INF_I32 if dtype == np.int32 else np.inf
    buf = np.full((n, ld), fill, dtype=dtype)
    A = buf[:, :n]
    A[u, v] = w
    A[v, u] = w
    if n:
        np.fill_diagonal(A, 0)
    return A


def csr_from_edges(n: int, u, v, w):
    """Adjacency lists with both directions of every edge: (indptr, indices, weights)."""
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    ww = np.concatenate([np.asarray(w), np.asarray(w)])
    order = np.argsort(src, kind="stable")
    src, dst, ww = src[order], dst[order], ww[order]
    indptr = np.zeros(n + 1, np.int64)
    np.add.at(indptr, src + 1, 1)
    return np.cumsum(indptr).astype(np.int64), dst, ww


def device_dense_from_edges(n: int, u, v, w, dtype, device, ld: int | None = None):
    """Same matrix as ``dense_from_edges`` built directly in device memory (torch).

    Returns the n x n view of an n x ld buffer.
    """
    import torch

    ld = n if ld is None else ld
    tdt = {np.dtype(np.int32): torch.int32, np.dtype(np.float32): torch.float32}[np.dtype(dtype)]
    fill = INF_I32 if tdt == torch.int32 else float("inf")
    buf = torch.full((n, ld), fill, dtype=tdt, device=device)
    A = buf[:, :n]
    if len(u):
        tu = torch.as_tensor(np.asarray(u, np.int64), device=device)
        tv = torch.as_tensor(np.asarray(v, np.int64), device=device)
        tw = torch.as_tensor(np.asarray(w).astype(np.dtype(dtype)), device=device)
        A[tu, tv] = tw
        A[tv, tu] = tw
    idx = torch.arange(n, device=device)
    A[idx, idx] = 0
    return A


# --------------------------------------------------------------------------
# Workload presets
# --------------------------------------------------------------------------

def plain_small(item: int = 0, n: int = 512, p: float = 0.05):
    """ER n=512, p=0.05, int32 weights U{1..100}: dense int32 matrix."""
    u, v, w = er_edges(n, p, 1, 100, rng_for(CFG_PLAIN_SMALL, item))
    return dense_from_edges(n, u, v, w, np.int32), (u, v, w)


def batched_sizes(count: int, rng: np.random.Generator, lo: int = 32, hi: int = 512) -> np.ndarray:
    """n_i = round(exp(U[ln lo, ln hi]))."""
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)


def batched_graphs(count: int = 4096, item: int = 0, lo: int = 32, hi: int = 512,
                   wlo: int = 1, whi: int = 1000):
    """Many independent ER graphs, n log-uniform in [lo, hi], p = 8/n, int32 U{wlo..whi}.

    Returns a list of dense int32 matrices.
    """
    rng = rng_for(CFG_BATCHED, item)
    ns = batched_sizes(count, rng, lo, hi)
    out = []
    for g, n in enumerate(ns):
        u, v, w = er_edges(int(n), min(1.0, 8.0 / n), wlo, whi, rng_for(CFG_BATCHED, 1_000_000 + g))
        out.append(dense_from_edges(int(n), u, v, w, np.int32))
    return out


SERVING_SIZES = (256, 1024, 4096, 8192)
SERVING_PROBS = (0.4, 0.3, 0.2, 0.1)


def serving_requests(count: int, qps: float, item: int = 0, sizes=SERVING_SIZES,
                     probs=SERVING_PROBS):
    """Poisson arrival times (seconds from 0) and request sizes."""
    rng = rng_for(CFG_SERVING, item)
    gaps = rng.exponential(1.0 / qps, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    ns = rng.choice(np.asarray(sizes, np.int64), size=count, p=np.asarray(probs))
    return arrivals, ns

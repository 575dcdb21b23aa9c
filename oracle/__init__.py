"""Host oracle for all-pairs shortest-path lengths (arXiv:1902.04446, Sec. 3).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product library must not,
and shares no code with it.  All arithmetic lives in ``apsp_oracle.c``; this
module only marshals numpy arrays into it.

Conventions (the paper fixes neither element type nor sentinel):

* int32 weights: entries in [0, 2**30], ``INF_I32 = 2**30`` marks a non-edge.
  Lengths come back as int64 (no overflow possible), saturated at 2**30.
* fp32 weights: entries in [0, +inf], +inf marks a non-edge.  Lengths come
  back as float64.
* The diagonal is the empty path: 0.

Functions:

``fw``             classic Floyd-Warshall, Sec. 3 (Table 1 FloydWarshall)
``fw_steps``       the same loop stopped after pivots k0..k1-1 (the state a
                   blocked solver must reach after each round)
``fw_prefix_rows`` rows of the state after pivots 0..K-1 from adjacency lists
                   (paths with intermediates in the first K vertices), for
                   sizes where no n x n matrix fits on the host
``dijkstra``       Dijkstra from the given sources (independent algorithm)
``brute``          minimum over all simple paths, n <= 10 (the definition)
``blocked``        three-phase blocked method, Sec. 4.4/4.5, Alg. 3/4, in the
                   element type the device computes in (uint32 or fp32)
``minplus_acc``    Table 1 MinPlus: C = min(C, A (x) B)
``squaring``       repeated min-plus squaring, Sec. 4.2, Alg. 1
``bellman_*``      Bellman optimality certificate over chosen rows
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

INF_I32 = 1 << 30

_LIBS: dict[int, ctypes.CDLL] = {}

_i64 = ctypes.c_int64
_p = ctypes.c_void_p


def _lib(mutant: int = 0) -> ctypes.CDLL:
    lib = _LIBS.get(mutant)
    if lib is not None:
        return lib
    path = _build.build(mutant)
    lib = ctypes.CDLL(path)
    sig = {
        "orc_mutant": ([], ctypes.c_int),
        "orc_max_threads": ([], ctypes.c_int),
        "orc_fw_steps_i64": ([_p, _i64, _i64, _i64, ctypes.c_int], None),
        "orc_fw_steps_f64": ([_p, _i64, _i64, _i64, ctypes.c_int], None),
        "orc_prepare_i32": ([_p, _i64, _i64, _p], None),
        "orc_prepare_f32": ([_p, _i64, _i64, _p], None),
        "orc_apsp_i32": ([_p, _i64, _i64, _p, ctypes.c_int], None),
        "orc_apsp_f32": ([_p, _i64, _i64, _p, ctypes.c_int], None),
        "orc_dijkstra_csr_f64": ([_p, _p, _p, _i64, _p, _i64, _p, ctypes.c_int], None),
        "orc_dijkstra_csr_i64": ([_p, _p, _p, _i64, _p, _i64, _p, ctypes.c_int], None),
        "orc_brute_f64": ([_p, _i64, _p], ctypes.c_int),
        "orc_minplus_acc_f32": ([_p, _i64, _p, _i64, _p, _i64, _i64, _i64, _i64], None),
        "orc_minplus_acc_u32": ([_p, _i64, _p, _i64, _p, _i64, _i64, _i64, _i64], None),
        "orc_blocked_u32": ([_p, _i64, _i64, _i64, _i64], None),
        "orc_squaring_u32": ([_p, _i64, _i64], None),
        "orc_squaring_f32": ([_p, _i64, _i64], None),
        "orc_blocked_f32": ([_p, _i64, _i64, _i64, _i64], None),
        "orc_bellman_residual_f32": ([_p, _i64, _i64, _p, _p, _p, _p, _i64, ctypes.c_int],
                                     ctypes.c_double),
        "orc_bellman_violations_i32": ([_p, _i64, _i64, _p, _p, _p, _p, _i64, ctypes.c_int],
                                       ctypes.c_int64),
        "orc_fw_prefix_rows_f64": ([_p, _p, _p, _i64, _i64, _p, _i64, _p, ctypes.c_int], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _LIBS[mutant] = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _as2d(W: np.ndarray, dtype) -> np.ndarray:
    W = np.asarray(W)
    if W.ndim != 2 or W.shape[0] != W.shape[1]:
        raise ValueError("expected a square matrix")
    if W.dtype != dtype:
        raise TypeError(f"expected {np.dtype(dtype)}, got {W.dtype}")
    if W.strides[1] != W.itemsize:
        W = np.ascontiguousarray(W)
    return W


def max_threads() -> int:
    return int(_lib().orc_max_threads())


def fw(W: np.ndarray, threads: int = 1, mutant: int = 0) -> np.ndarray:
    """All-pairs shortest lengths by classic Floyd-Warshall.

    int32 in -> int64 out (saturated at 2**30); float32 in -> float64 out.
    """
    lib = _lib(mutant)
    W = np.asarray(W)
    n = W.shape[0]
    if W.dtype == np.int32:
        W = _as2d(W, np.int32)
        D = np.empty((n, n), np.int64)
        lib.orc_apsp_i32(_ptr(W), n, W.strides[0] // 4, _ptr(D), threads)
        return D
    if W.dtype == np.float32:
        W = _as2d(W, np.float32)
        D = np.empty((n, n), np.float64)
        lib.orc_apsp_f32(_ptr(W), n, W.strides[0] // 4, _ptr(D), threads)
        return D
    raise TypeError("fw takes int32 or float32 weights")


def prepare(W: np.ndarray) -> np.ndarray:
    """Normalised starting matrix (int64 / float64): diagonal 0, int >= 2**30 -> 2**30."""
    lib = _lib()
    n = W.shape[0]
    if W.dtype == np.int32:
        W = _as2d(W, np.int32)
        D = np.empty((n, n), np.int64)
        lib.orc_prepare_i32(_ptr(W), n, W.strides[0] // 4, _ptr(D))
        return D
    W = _as2d(W, np.float32)
    D = np.empty((n, n), np.float64)
    lib.orc_prepare_f32(_ptr(W), n, W.strides[0] // 4, _ptr(D))
    return D


def fw_steps(D: np.ndarray, k0: int, k1: int, threads: int = 1, mutant: int = 0) -> np.ndarray:
    """Run Floyd-Warshall pivots k0..k1-1 in place on a prepared int64/float64 matrix."""
    lib = _lib(mutant)
    n = D.shape[0]
    if D.dtype == np.int64:
        D = _as2d(D, np.int64)
        lib.orc_fw_steps_i64(_ptr(D), n, k0, k1, threads)
    elif D.dtype == np.float64:
        D = _as2d(D, np.float64)
        lib.orc_fw_steps_f64(_ptr(D), n, k0, k1, threads)
    else:
        raise TypeError("fw_steps takes int64 or float64")
    return D


def csr_from_dense(W: np.ndarray):
    """Adjacency lists (both directions as stored) of the finite off-diagonal entries."""
    W = np.asarray(W)
    n = W.shape[0]
    if W.dtype == np.int32:
        mask = W < INF_I32
    else:
        mask = np.isfinite(W)
    np.fill_diagonal(mask, False)
    rows, cols = np.nonzero(mask)
    indptr = np.zeros(n + 1, np.int64)
    np.add.at(indptr, rows + 1, 1)
    indptr = np.cumsum(indptr).astype(np.int64)
    return indptr, cols.astype(np.int64), W[rows, cols]


def dijkstra(csr, n: int, sources, threads: int = 1, integer: bool = False) -> np.ndarray:
    """Shortest lengths from each source (rows), via Dijkstra over a CSR graph.

    ``csr`` = (indptr, indices, weights).  ``integer`` returns int64 saturated at
    2**30; otherwise float64 with +inf for unreachable.
    """
    lib = _lib()
    indptr = np.ascontiguousarray(csr[0], np.int64)
    indices = np.ascontiguousarray(csr[1], np.int64)
    src = np.ascontiguousarray(np.asarray(sources, np.int64).ravel())
    if integer:
        w = np.ascontiguousarray(csr[2], np.int64)
        out = np.empty((src.size, n), np.int64)
        lib.orc_dijkstra_csr_i64(_ptr(indptr), _ptr(indices), _ptr(w), n, _ptr(src), src.size,
                                 _ptr(out), threads)
    else:
        w = np.ascontiguousarray(csr[2], np.float64)
        out = np.empty((src.size, n), np.float64)
        lib.orc_dijkstra_csr_f64(_ptr(indptr), _ptr(indices), _ptr(w), n, _ptr(src), src.size,
                                 _ptr(out), threads)
    return out


def fw_prefix_rows(csr, n: int, K: int, rows, threads: int = 1) -> np.ndarray:
    """Rows of the Floyd-Warshall state after pivots 0..K-1, from adjacency lists.

    ``csr`` = (indptr, indices, weights); the result (len(rows) x n, float64,
    +inf = no path) equals those rows of ``fw_steps(prepare(W), 0, K)`` for
    the matrix W the lists describe, without forming any n x n matrix.
    """
    lib = _lib()
    indptr = np.ascontiguousarray(csr[0], np.int64)
    indices = np.ascontiguousarray(csr[1], np.int64)
    w = np.ascontiguousarray(csr[2], np.float64)
    src = np.ascontiguousarray(np.asarray(rows, np.int64).ravel())
    out = np.empty((src.size, n), np.float64)
    lib.orc_fw_prefix_rows_f64(_ptr(indptr), _ptr(indices), _ptr(w), n, K, _ptr(src), src.size,
                               _ptr(out), threads)
    return out


def brute(W: np.ndarray) -> np.ndarray:
    """Minimum over all simple paths (float64; +inf = unreachable).  n <= 10.

    int32 input: entries >= 2**30 are non-edges.
    """
    W = np.asarray(W)
    n = W.shape[0]
    if W.dtype == np.int32:
        Wd = np.where(W >= INF_I32, np.inf, W.astype(np.float64))
    else:
        Wd = W.astype(np.float64)
    Wd = np.ascontiguousarray(Wd)
    out = np.empty((n, n), np.float64)
    if _lib().orc_brute_f64(_ptr(Wd), n, _ptr(out)) != 0:
        raise ValueError("brute force is limited to n <= 10")
    return out


def blocked(W: np.ndarray, b: int, r0: int = 0, r1: int | None = None) -> np.ndarray:
    """Blocked three-phase solve in the device element type.

    int32 in -> int32 out (computed as uint32); float32 in -> float32 out.
    Starts from the normalised input (diagonal 0, int clamp at 2**30) when
    ``r0 == 0``; otherwise ``W`` must be a state returned by an earlier call.
    """
    lib = _lib()
    W = np.asarray(W)
    n = W.shape[0]
    q = -(-n // b) if n else 0
    if r1 is None:
        r1 = q
    if W.dtype == np.int32:
        D = np.ascontiguousarray(W).astype(np.int64)
        if r0 == 0:
            D = prepare(np.ascontiguousarray(W))
        D = D.astype(np.uint32)
        lib.orc_blocked_u32(_ptr(D), n, b, r0, r1)
        return D.astype(np.int32)
    if W.dtype == np.float32:
        D = np.ascontiguousarray(W).copy()
        if r0 == 0:
            np.fill_diagonal(D, 0.0)
        lib.orc_blocked_f32(_ptr(D), n, b, r0, r1)
        return D
    raise TypeError("blocked takes int32 or float32")


def squaring_steps(n: int) -> int:
    """Squarings that cover every path of up to n - 1 edges: ceil(log2(n - 1))."""
    s = 0
    while n > 2 and (1 << s) < n - 1:
        s += 1
    return s


def squaring(W: np.ndarray, steps: int | None = None) -> np.ndarray:
    """Repeated min-plus squaring (Sec. 4.2, Alg. 1) in the device element type.

    int32 in -> int32 out (computed as uint32); float32 in -> float32 out.
    """
    lib = _lib()
    W = np.asarray(W)
    n = W.shape[0]
    steps = squaring_steps(n) if steps is None else steps
    if W.dtype == np.int32:
        X = prepare(np.ascontiguousarray(W)).astype(np.uint32)
        lib.orc_squaring_u32(_ptr(X), n, steps)
        return X.astype(np.int32)
    if W.dtype == np.float32:
        X = np.ascontiguousarray(W).copy()
        if n:
            np.fill_diagonal(X, 0.0)
        lib.orc_squaring_f32(_ptr(X), n, steps)
        return X
    raise TypeError("squaring takes int32 or float32")


def minplus_acc(C: np.ndarray, A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Table 1 MinPlus on whole matrices: returns min(C, A (x) B) (same dtype)."""
    lib = _lib()
    m, kk = A.shape
    kk2, nn = B.shape
    assert kk == kk2 and C.shape == (m, nn)
    out = np.ascontiguousarray(C).copy()
    if C.dtype == np.float32:
        A = np.ascontiguousarray(A, np.float32)
        B = np.ascontiguousarray(B, np.float32)
        lib.orc_minplus_acc_f32(_ptr(A), kk, _ptr(B), nn, _ptr(out), nn, m, nn, kk)
    else:
        A = np.ascontiguousarray(A).astype(np.uint32)
        B = np.ascontiguousarray(B).astype(np.uint32)
        out = out.astype(np.uint32)
        lib.orc_minplus_acc_u32(_ptr(A), kk, _ptr(B), nn, _ptr(out), nn, m, nn, kk)
        out = out.astype(C.dtype)
    return out


def bellman_residual_f32(D: np.ndarray, csr, rows, threads: int = 1) -> float:
    """Largest relative Bellman residual of an fp32 distance matrix over ``rows``."""
    D = np.asarray(D)
    assert D.dtype == np.float32 and D.strides[1] == 4
    n = D.shape[0]
    indptr = np.ascontiguousarray(csr[0], np.int64)
    indices = np.ascontiguousarray(csr[1], np.int64)
    w = np.ascontiguousarray(csr[2], np.float64)
    rows = np.ascontiguousarray(np.asarray(rows, np.int64).ravel())
    return float(_lib().orc_bellman_residual_f32(_ptr(D), D.strides[0] // 4, n, _ptr(indptr),
                                                 _ptr(indices), _ptr(w), _ptr(rows), rows.size,
                                                 threads))


def bellman_violations_i32(D: np.ndarray, csr, rows, threads: int = 1) -> int:
    """Number of entries over ``rows`` violating the exact Bellman certificate (int32)."""
    D = np.asarray(D)
    assert D.dtype == np.int32 and D.strides[1] == 4
    n = D.shape[0]
    indptr = np.ascontiguousarray(csr[0], np.int64)
    indices = np.ascontiguousarray(csr[1], np.int64)
    w = np.ascontiguousarray(csr[2], np.int64)
    rows = np.ascontiguousarray(np.asarray(rows, np.int64).ravel())
    return int(_lib().orc_bellman_violations_i32(_ptr(D), D.strides[0] // 4, n, _ptr(indptr),
                                                 _ptr(indices), _ptr(w), _ptr(rows), rows.size,
                                                 threads))

"""Python binding of the MI355X APSP library (``libapsp.so``, C ABI in include/apsp.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  PyTorch supplies device memory and the current HIP stream.  There
is no CPU fallback: if the library is not built, importing this module fails.

    import torch, paper_1902_04446_amd as apsp
    D = ...  # (n, n) int32 or float32 tensor on a ROCm device, row stride = ld
    apsp.solve(D)              # in place, enqueued on torch's current stream
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "APSP_I32", "APSP_F32", "INF_I32", "ApspError", "lib_path", "library",
    "solve", "solve_profiled", "solve_rounds", "solve_batched", "validate", "round_width",
    "batched_round_width", "num_rounds", "version",
]

APSP_I32 = 0
APSP_F32 = 1
INF_I32 = 1 << 30
BATCHED_MAX_N = 4096

_HERE = os.path.dirname(os.path.abspath(__file__))


def lib_path() -> str:
    return os.path.join(_HERE, "libapsp.so")


class ApspError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {_LIB.apsp_status_string(status).decode()} (status {status})")


def _load() -> ctypes.CDLL:
    path = lib_path()
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python paper_1902_04446_amd/build.py` "
            "(there is no fallback implementation)")
    lib = ctypes.CDLL(path)
    i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
    sigs = {
        "apsp_solve": ([vp, i64, i64, i32, vp], i32),
        "apsp_solve_rounds": ([vp, i64, i64, i32, i64, i64, vp], i32),
        "apsp_solve_profiled": ([vp, i64, i64, i32, vp, ctypes.POINTER(ctypes.c_double)], i32),
        "apsp_round_width": ([i64, i32], i32),
        "apsp_batched_round_width": ([i64, i32], i32),
        "apsp_solve_batched": ([vp, vp, i32, vp], i32),
        "apsp_solve_batched_ex": ([vp, vp, vp, i32, i32, vp], i32),
        "apsp_validate": ([vp, i64, i64, i32, vp], i32),
        "apsp_status_string": ([i32], ctypes.c_char_p),
        "apsp_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_LIB = _load()


def library() -> ctypes.CDLL:
    return _LIB


def version() -> str:
    return _LIB.apsp_version().decode()


def _dtype_code(t) -> int:
    import torch

    if t.dtype == torch.int32:
        return APSP_I32
    if t.dtype == torch.float32:
        return APSP_F32
    raise TypeError(f"APSP matrices are int32 or float32, got {t.dtype}")


def _matrix_args(t):
    """(pointer, n, ld, dtype) of a square device matrix view with unit column stride."""
    if not t.is_cuda:
        raise ValueError("the APSP library works on device (ROCm) tensors only")
    if t.dim() != 2 or t.shape[0] != t.shape[1]:
        raise ValueError(f"expected a square 2-D matrix, got shape {tuple(t.shape)}")
    n = int(t.shape[0])
    if n > 1 and t.stride(1) != 1:
        raise ValueError("matrix columns must be contiguous (stride(1) == 1)")
    ld = int(t.stride(0)) if n > 1 else max(1, int(t.stride(0)))
    return t.data_ptr(), n, max(ld, n, 1), _dtype_code(t)


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check(status: int, what: str):
    if status != 0:
        raise ApspError(status, what)


def round_width(n: int = 0, dtype: int = APSP_F32) -> int:
    return int(_LIB.apsp_round_width(n, dtype))


def batched_round_width(n: int = 0, dtype: int = APSP_I32) -> int:
    return int(_LIB.apsp_batched_round_width(n, dtype))


def num_rounds(n: int, dtype: int = APSP_F32) -> int:
    b = round_width(n, dtype)
    return -(-n // b) if n else 0


def solve(t, stream=None):
    """Solve the APSP problem of matrix ``t`` in place (asynchronous on ``stream``)."""
    ptr, n, ld, dt = _matrix_args(t)
    with _device_of(t):
        _check(_LIB.apsp_solve(ctypes.c_void_p(ptr), n, ld, dt, _stream(stream)), "apsp_solve")
    return t


def solve_profiled(t, stream=None) -> dict:
    """Solve in place, timing each phase with HIP events on the stream; synchronous.

    Returns milliseconds {"prologue", "phase1", "phase2", "phase3", "total",
    "phase3_rest", "phase3_rest_launches", "phase3_other"}; see apsp_solve_profiled.
    """
    ptr, n, ld, dt = _matrix_args(t)
    out = (ctypes.c_double * 8)()
    with _device_of(t):
        _check(_LIB.apsp_solve_profiled(ctypes.c_void_p(ptr), n, ld, dt, _stream(stream), out),
               "apsp_solve_profiled")
    keys = ("prologue", "phase1", "phase2", "phase3", "total", "phase3_rest",
            "phase3_rest_launches", "phase3_other")
    return dict(zip(keys, list(out)))


def solve_rounds(t, r0: int, r1: int, stream=None):
    """Run rounds r0..r1-1 of the blocked method in place (r0 == 0 normalises the input)."""
    ptr, n, ld, dt = _matrix_args(t)
    with _device_of(t):
        _check(_LIB.apsp_solve_rounds(ctypes.c_void_p(ptr), n, ld, dt, r0, r1, _stream(stream)),
               "apsp_solve_rounds")
    return t


def solve_batched(mats, stream=None):
    """Solve a list of independent square matrices (all int32, or all float32) in one launch."""
    import torch

    mats = list(mats)
    if not mats:
        return mats
    codes = {_dtype_code(m) for m in mats}
    if len(codes) != 1:
        raise TypeError("a batch must have a single dtype")
    dt = codes.pop()
    count = len(mats)
    ptrs = (ctypes.c_void_p * count)()
    ns = (ctypes.c_int32 * count)()
    lds = (ctypes.c_int64 * count)()
    dev = mats[0].device
    for g, m in enumerate(mats):
        if m.device != dev:
            raise ValueError("all matrices of a batch must be on one device")
        p, n, ld, _ = _matrix_args(m)
        ptrs[g] = p
        ns[g] = n
        lds[g] = ld
    with torch.cuda.device(dev):
        _check(_LIB.apsp_solve_batched_ex(ptrs, ns, lds, count, dt, _stream(stream)),
               "apsp_solve_batched_ex")
    return mats


def validate(t, stream=None) -> bool:
    """True when every entry is a valid weight (>= 0, not NaN).  Synchronous."""
    ptr, n, ld, dt = _matrix_args(t)
    with _device_of(t):
        st = _LIB.apsp_validate(ctypes.c_void_p(ptr), n, ld, dt, _stream(stream))
    if st == 5:
        return False
    _check(st, "apsp_validate")
    return True


def _device_of(t):
    import torch

    return torch.cuda.device(t.device)

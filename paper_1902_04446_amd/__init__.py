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
    "solve", "solve_profiled", "solve_rounds", "solve_batched", "solve_batched_noalloc",
    "BatchArgs", "BatchPlan", "validate",
    "minplus", "solve_squaring", "squarings", "solve_symmetric",
    "round_width", "batched_round_width", "num_rounds", "version",
    "TUNE_BUCKETS", "batched_tuning", "set_batched_tuning", "batched_autotune",
    "batched_autotune_batch", "set_round_pair_threshold", "set_width64_max_n",
    "set_aligned_copy_min_n",
    "stream_state_bytes", "stream_state_count", "release_stream_state",
]

APSP_I32 = 0
APSP_F32 = 1
INF_I32 = 1 << 30
BATCHED_MAX_N = 4096
TUNE_BUCKETS = 9

_HERE = os.path.dirname(os.path.abspath(__file__))


def lib_path() -> str:
    return os.path.join(_HERE, "libapsp.so")


class ApspError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        detail = _LIB.apsp_last_error().decode() if status in (3, 4) else ""
        super().__init__(f"{what}: {_LIB.apsp_status_string(status).decode()} (status {status})"
                         + (f" [{detail}]" if detail else ""))


def _load() -> ctypes.CDLL:
    # libapsp.so needs the HIP runtime (SONAME libamdhip64.so.7).  PyTorch
    # ships its own copy of it: load torch first so the library binds to that
    # one instance.  Loading ours first would put two HIP runtimes in the
    # process, and the second would see no device.
    import torch  # noqa: F401

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
        "apsp_set_round_pair_threshold": ([i32], i32),
        "apsp_set_width64_max_n": ([i64], i64),
        "apsp_set_aligned_copy_min_n": ([i64], i64),
        "apsp_stream_state_bytes": ([i64, i32], i64),
        "apsp_stream_state_count": ([], i64),
        "apsp_release_stream_state": ([vp], i32),
        "apsp_solve_batched": ([vp, vp, i32, vp], i32),
        "apsp_solve_batched_ex": ([vp, vp, vp, i32, i32, vp], i32),
        "apsp_solve_batched_noalloc": ([vp, vp, vp, i32, i32, vp], i32),
        "apsp_validate": ([vp, i64, i64, i32, vp], i32),
        "apsp_batched_plan_create": ([vp, vp, vp, i32, i32, vp, ctypes.POINTER(vp)], i32),
        "apsp_batched_plan_run": ([vp, vp], i32),
        "apsp_batched_plan_info": ([vp, ctypes.POINTER(i64)], i32),
        "apsp_batched_plan_destroy": ([vp], i32),
        "apsp_batched_plan_create_tiled": ([vp, vp, vp, i32, i32, i32, vp, ctypes.POINTER(vp)],
                                           i32),
        "apsp_batched_tuning_get": ([ctypes.POINTER(i32), i32], i32),
        "apsp_batched_tuning_set": ([ctypes.POINTER(i32), i32], i32),
        "apsp_batched_autotune": ([i32, i64, vp, ctypes.POINTER(i32),
                                   ctypes.POINTER(ctypes.c_double)], i32),
        "apsp_batched_autotune_batch": ([vp, vp, vp, i32, i32, vp, ctypes.POINTER(i32),
                                         ctypes.POINTER(ctypes.c_double)], i32),
        "apsp_status_string": ([i32], ctypes.c_char_p),
        "apsp_version": ([], ctypes.c_char_p),
        "apsp_minplus": ([vp, i64, vp, i64, vp, i64, i64, i64, i64, i32, i32, vp], i32),
        "apsp_solve_squaring": ([vp, i64, i64, i32, vp, i64, vp], i32),
        "apsp_squarings": ([i64], i32),
        "apsp_solve_symmetric": ([vp, i64, i64, i32, vp], i32),
        "apsp_last_error": ([], ctypes.c_char_p),
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


def _row_stride(shape, stride, what="matrix") -> int:
    """Leading dimension of a 2-D view with unit column stride: ``stride[0]``,
    which must be at least the row length so that rows do not overlap (a
    broadcast or overlapping ``as_strided`` view would make the library write
    one element through several indices).  Single-row views have no row
    stride to check; they report max(stride[0], cols, 1)."""
    rows, cols = int(shape[0]), int(shape[1])
    if cols > 1 and stride[1] != 1:
        raise ValueError(f"{what} columns must be contiguous (stride(1) == 1)")
    if rows > 1:
        if stride[0] < max(cols, 1):
            raise ValueError(f"{what} rows overlap: stride(0) = {stride[0]} < {cols} columns "
                             "(broadcast or overlapping view)")
        return int(stride[0])
    return max(int(stride[0]), cols, 1)


def _matrix_args(t):
    """(pointer, n, ld, dtype) of a square device matrix view with unit column stride."""
    if t.dim() != 2 or t.shape[0] != t.shape[1]:
        raise ValueError(f"expected a square 2-D matrix, got shape {tuple(t.shape)}")
    n = int(t.shape[0])
    ld = _row_stride(t.shape, t.stride())
    dt = _dtype_code(t)
    if not t.is_cuda:
        raise ValueError("the APSP library works on device (ROCm) tensors only")
    return t.data_ptr(), n, ld, dt


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check(status: int, what: str):
    if status != 0:
        raise ApspError(status, what)


def set_round_pair_threshold(rounds: int) -> int:
    """Rounds from which solves run phase 3 in round pairs (process-wide;
    default 72); returns the previous value.  The results are the same."""
    prev = int(_LIB.apsp_set_round_pair_threshold(int(rounds)))
    if prev < 0:
        raise ValueError("the threshold is a number of rounds >= 2")
    return prev


def set_width64_max_n(n: int) -> int:
    """Largest n solved in rounds of width 64 (process-wide; default 5120;
    0 disables them); returns the previous value.  fp32 results follow the
    blocked method at the width round_width(n) reports."""
    prev = int(_LIB.apsp_set_width64_max_n(int(n)))
    if prev < 0:
        raise ValueError("the limit is a vertex count in [0, 8192]")
    return prev


def set_aligned_copy_min_n(n: int) -> int:
    """Smallest n from which a solve whose layout would be slow (rows not
    16-byte aligned, or n not a multiple of 128 with rounds of 128) runs on
    a working copy (process-wide; default 512; a value above every n turns
    the copy off); returns the previous value.  The result is the same either
    way."""
    prev = int(_LIB.apsp_set_aligned_copy_min_n(int(n)))
    if prev < 0:
        raise ValueError("the threshold is a vertex count >= 0")
    return prev


def stream_state_bytes(n: int, dtype: int = APSP_F32) -> int:
    """Device bytes of the per-stream state a full solve of an n-vertex
    matrix creates on a stream without state (0 if it creates none)."""
    v = int(_LIB.apsp_stream_state_bytes(int(n), int(dtype)))
    if v < 0:
        raise ValueError("bad dtype or vertex count")
    return v


def stream_state_count() -> int:
    """How many (device, stream) solver states the process holds."""
    return int(_LIB.apsp_stream_state_count())


def release_stream_state(stream=None, device=None):
    """Release the solver state kept for ``stream`` (default: the current
    stream) on ``device``: waits for that stream's work, then frees its helper
    streams and memory.  Call it before dropping a stream solves ran on."""
    import torch

    dev = torch.device(device) if device is not None else (
        stream.device if stream is not None else torch.device("cuda", torch.cuda.current_device()))
    with torch.cuda.device(dev):
        _check(_LIB.apsp_release_stream_state(_stream(stream)), "apsp_release_stream_state")


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


def solve_symmetric(t, stream=None):
    """Solve an undirected graph's matrix in place from its upper triangle (Sec. 4 storage)."""
    ptr, n, ld, dt = _matrix_args(t)
    with _device_of(t):
        _check(_LIB.apsp_solve_symmetric(ctypes.c_void_p(ptr), n, ld, dt, _stream(stream)),
               "apsp_solve_symmetric")
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


def _batch_arrays(mats):
    """Host arrays (ptrs, ns, lds) and dtype code of a list of square device matrices."""
    import torch

    count = len(mats)
    ptrs = (ctypes.c_void_p * count)()
    ns = (ctypes.c_int32 * count)()
    lds = (ctypes.c_int64 * count)()
    if count == 0:
        return ptrs, ns, lds, APSP_I32, None
    dt = _dtype_code(mats[0])
    dev = mats[0].device
    tdt = mats[0].dtype
    for g, m in enumerate(mats):
        if m.dtype != tdt:
            raise TypeError("a batch must have a single dtype")
        shp = m.shape
        if len(shp) != 2 or shp[0] != shp[1]:
            raise ValueError(f"expected square 2-D matrices, got shape {tuple(shp)}")
        lds[g] = _row_stride(shp, m.stride(), f"matrix {g}")
    if not mats[0].is_cuda:
        raise ValueError("the APSP library works on device (ROCm) tensors only")
    for g, m in enumerate(mats):
        if m.device != dev:
            raise ValueError("all matrices of a batch must be on one device")
        ptrs[g] = m.data_ptr()
        ns[g] = int(m.shape[0])
    del torch
    return ptrs, ns, lds, dt, dev


class BatchArgs:
    """The host arrays (pointers, sizes, leading dimensions) of a batch of
    device matrices, marshalled once.  solve_batched / solve_batched_noalloc
    accept it in place of the list, so a caller that solves the same buffers
    repeatedly pays the per-tensor Python work once (about 1 us per matrix).
    It refers to the matrices' memory: keep ``mats`` alive while it is used."""

    def __init__(self, mats):
        self.mats = list(mats)
        self.ptrs, self.ns, self.lds, self.dtype, self.device = _batch_arrays(self.mats)

    def __len__(self):
        return len(self.mats)


def _batch_call(fn, name, mats, stream):
    import torch

    args = mats if isinstance(mats, BatchArgs) else BatchArgs(mats)
    if len(args) == 0:
        return args.mats
    with torch.cuda.device(args.device):
        _check(fn(args.ptrs, args.ns, args.lds, len(args), args.dtype, _stream(stream)), name)
    return args.mats


def solve_batched(mats, stream=None):
    """Solve a list of independent square matrices (all int32, or all float32)
    together (or a BatchArgs of them)."""
    return _batch_call(_LIB.apsp_solve_batched_ex, "apsp_solve_batched_ex", mats, stream)


def solve_batched_noalloc(mats, stream=None):
    """solve_batched without any device allocation: the tables go to the
    library's fixed per-GPU workspace (apsp_solve_batched_noalloc; calls that
    overlap on one GPU race on it)."""
    return _batch_call(_LIB.apsp_solve_batched_noalloc, "apsp_solve_batched_noalloc", mats,
                       stream)


class BatchPlan:
    """A reusable batched solve of fixed matrices (apsp_batched_plan_*).

    The descriptor and work tables live in device memory; ``run()`` only
    enqueues kernels, so it is cheap to repeat and can be graph-captured.
    The plan refers to the matrices' memory: keep ``mats`` alive while it is used.
    """

    def __init__(self, mats, stream=None, tile: int = 0):
        """``tile`` 64 or 128 forces that round width for every graph; 0 takes
        each graph's width from the device's batched tuning table."""
        import torch

        self.mats = list(mats)
        self._plan = ctypes.c_void_p(None)
        ptrs, ns, lds, dt, dev = _batch_arrays(self.mats)
        self.device = dev
        with torch.cuda.device(dev) if dev is not None else _nullcontext():
            _check(_LIB.apsp_batched_plan_create_tiled(ptrs, ns, lds, len(self.mats), dt, tile,
                                                       _stream(stream), ctypes.byref(self._plan)),
                   "apsp_batched_plan_create_tiled")

    def run(self, stream=None):
        import torch

        with torch.cuda.device(self.device) if self.device is not None else _nullcontext():
            _check(_LIB.apsp_batched_plan_run(self._plan, _stream(stream)),
                   "apsp_batched_plan_run")
        return self.mats

    def info(self) -> dict:
        out = (ctypes.c_int64 * 3)()
        _check(_LIB.apsp_batched_plan_info(self._plan, out), "apsp_batched_plan_info")
        return {"launches": int(out[0]), "items": int(out[1]), "tile_updates": int(out[2])}

    def close(self):
        if self._plan:
            _LIB.apsp_batched_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batched_tuning() -> list:
    """The current device's batched round widths per size bucket (bucket b < 8:
    n in (64b, 64b + 64]; bucket 8: n > 512)."""
    out = (ctypes.c_int32 * TUNE_BUCKETS)()
    _check(_LIB.apsp_batched_tuning_get(out, TUNE_BUCKETS), "apsp_batched_tuning_get")
    return list(out)


def set_batched_tuning(widths) -> None:
    """Replace the current device's batched round widths (9 entries, 64 or 128)."""
    widths = list(widths)
    arr = (ctypes.c_int32 * len(widths))(*widths)
    _check(_LIB.apsp_batched_tuning_set(arr, len(widths)), "apsp_batched_tuning_set")


def batched_autotune(dtype: int = APSP_I32, batch_elems: int = 1 << 24, stream=None) -> dict:
    """Time both batched round widths per size bucket on the current device and
    keep the faster; returns {"widths": [...], "ms": [(ms_128, ms_64), ...]}."""
    table = (ctypes.c_int32 * TUNE_BUCKETS)()
    ms = (ctypes.c_double * (2 * TUNE_BUCKETS))()
    _check(_LIB.apsp_batched_autotune(dtype, batch_elems, _stream(stream), table, ms),
           "apsp_batched_autotune")
    return {"widths": list(table),
            "ms": [(float(ms[2 * b]), float(ms[2 * b + 1])) for b in range(TUNE_BUCKETS)]}


def batched_autotune_batch(mats, stream=None) -> dict:
    """Tune the current device's batched round widths for this batch (solved
    on copies; ``mats`` is only read); returns {"widths": [...],
    "ms_all_128": t0, "ms_tuned": t1}."""
    import torch

    mats = list(mats)
    ptrs, ns, lds, dt, dev = _batch_arrays(mats)
    table = (ctypes.c_int32 * TUNE_BUCKETS)()
    ms = (ctypes.c_double * 2)()
    with torch.cuda.device(dev) if dev is not None else _nullcontext():
        _check(_LIB.apsp_batched_autotune_batch(ptrs, ns, lds, len(mats), dt, _stream(stream),
                                                table, ms), "apsp_batched_autotune_batch")
    return {"widths": list(table), "ms_all_128": float(ms[0]), "ms_tuned": float(ms[1])}


class _nullcontext:
    def __enter__(self):
        return None

    def __exit__(self, *exc):
        return False


def minplus(C, A, B, accumulate: bool = False, stream=None):
    """C = A (x) B (min-plus product), or C = min(C, A (x) B) with accumulate.  In place on C."""
    lds = {}
    for name, t in (("C", C), ("A", A), ("B", B)):
        if t.dim() != 2:
            raise ValueError(f"{name} must be a 2-D matrix")
        lds[name] = _row_stride(t.shape, t.stride(), name)
    if not (C.dtype == A.dtype == B.dtype):
        raise TypeError("C, A and B must have one dtype")
    m, k = A.shape
    k2, n = B.shape
    if k != k2 or tuple(C.shape) != (m, n):
        raise ValueError(f"shape mismatch: C {tuple(C.shape)}, A {tuple(A.shape)}, B {tuple(B.shape)}")
    dt = _dtype_code(C)
    for name, t in (("C", C), ("A", A), ("B", B)):
        if not t.is_cuda:
            raise ValueError(f"{name} must be a device (ROCm) matrix")
    with _device_of(C):
        _check(_LIB.apsp_minplus(ctypes.c_void_p(C.data_ptr()), lds["C"],
                                 ctypes.c_void_p(A.data_ptr()), lds["A"],
                                 ctypes.c_void_p(B.data_ptr()), lds["B"], m, n, k, dt,
                                 1 if accumulate else 0, _stream(stream)), "apsp_minplus")
    return C


def squarings(n: int) -> int:
    return int(_LIB.apsp_squarings(n))


def solve_squaring(t, work, stream=None):
    """APSP by repeated min-plus squaring (Sec. 4.2); ``work`` is an n x n scratch matrix."""
    ptr, n, ld, dt = _matrix_args(t)
    wptr, wn, wld, wdt = _matrix_args(work)
    if wn != n or wdt != dt:
        raise ValueError("work must be an n x n matrix of the same dtype")
    with _device_of(t):
        _check(_LIB.apsp_solve_squaring(ctypes.c_void_p(ptr), n, ld, dt, ctypes.c_void_p(wptr), wld,
                                        _stream(stream)), "apsp_solve_squaring")
    return t


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

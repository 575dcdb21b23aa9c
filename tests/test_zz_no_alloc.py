"""The allocation-free batched entry point (apsp_solve_batched_noalloc) against
apsp_solve_batched_ex on the same inputs, through the C ABI: two calls in a
row on the same stream, the second with a smaller batch, both dtypes; int32
results also against the oracle.  Runs last (its workspace is shared by every
call on the GPU)."""
import ctypes

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def apsp():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1902_04446_amd as mod

    fn = mod.library().apsp_solve_batched_noalloc
    vp = ctypes.c_void_p
    fn.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_int32, vp]
    fn.restype = ctypes.c_int32
    return mod


def _graphs(dtype, count, item):
    """Batch graphs (ER, n log-uniform in [32, 512]) as int32, or the same
    graphs with fp32 weights."""
    Ws = gg.batched_graphs(count, item=item)
    if dtype == np.float32:
        Ws = [np.where(W >= oracle.INF_I32, np.inf, W.astype(np.float32) * 0.25).astype(np.float32)
              for W in Ws]
    return Ws


def _solve_both(apsp, Ws):
    import torch

    dev = torch.device("cuda:0")
    a = [torch.from_numpy(W).to(dev) for W in Ws]
    b = [x.clone() for x in a]
    s = torch.cuda.current_stream()
    ptrs, ns, lds, dt, _ = apsp._batch_arrays(a)
    st = apsp.library().apsp_solve_batched_noalloc(ptrs, ns, lds, len(a), dt,
                                                   ctypes.c_void_p(s.cuda_stream))
    assert st == 0, apsp.library().apsp_last_error()
    ptrs, ns, lds, dt, _ = apsp._batch_arrays(b)
    assert apsp.library().apsp_solve_batched_ex(ptrs, ns, lds, len(b), dt,
                                                ctypes.c_void_p(s.cuda_stream)) == 0
    return a, b


@pytest.mark.parametrize("dtype", [np.int32, np.float32])
def test_noalloc_equals_batched_twice_smaller_second(apsp, dtype):
    import torch

    first = _graphs(dtype, 512, item=21)
    second = _graphs(dtype, 40, item=22)
    a1, b1 = _solve_both(apsp, first)
    a2, b2 = _solve_both(apsp, second)
    torch.cuda.synchronize()
    for Ws, a, b in ((first, a1, b1), (second, a2, b2)):
        for W, x, y in zip(Ws, a, b):
            assert torch.equal(x, y), W.shape
        if dtype == np.int32:
            for g in range(0, len(Ws), max(1, len(Ws) // 12)):
                assert np.array_equal(a[g].cpu().numpy().astype(np.int64), oracle.fw(Ws[g]))


def test_noalloc_refuses_a_batch_beyond_its_workspace(apsp):
    """Tables larger than the workspace: APSP_ERR_UNSUPPORTED, nothing enqueued,
    the matrices untouched; a following call still works."""
    import torch

    dev = torch.device("cuda:0")
    # 40 graphs of 4096 vertices at width 128: 40 (1 + 32 (32^2 - 1)) items,
    # 10.5 MB of tables
    big = [torch.full((4096, 4096), 1.0, device=dev) for _ in range(40)]
    ptrs, ns, lds, dt, _ = apsp._batch_arrays(big)
    lib = apsp.library()
    st = lib.apsp_solve_batched_noalloc(ptrs, ns, lds, len(big), dt, None)
    assert st == 2, st
    assert b"allocation-free workspace" in lib.apsp_last_error()
    torch.cuda.synchronize()
    assert all(bool((m == 1.0).all()) for m in big)
    del big
    Ws = _graphs(np.int32, 16, item=23)
    a, b = _solve_both(apsp, Ws)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)

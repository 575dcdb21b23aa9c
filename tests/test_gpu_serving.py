"""The continuous-batching server on the GPU: every result is the same alone
and in the mix (bit for bit: a solve split into round slices runs the same
phases on the same data), admission keeps resident matrices within the
budget, and small results still match the host oracle."""
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

    return mod


def _requests(sizes, seed0):
    from paper_1902_04446_amd.serving import Request

    reqs = []
    for i, n in enumerate(sizes):
        u, v, w = gg.swiss_roll_knn(n, gg.CFG_TEST, seed0 + i)
        reqs.append(Request(rid=i, n=n, arrival=0.0, payload=(u, v, w)))
    return reqs


def _alone(apsp, req, dev):
    import torch

    u, v, w = req.payload
    D = gg.device_dense_from_edges(req.n, u, v, w, np.float32, dev)
    apsp.solve(D)
    torch.cuda.synchronize()
    return D


@pytest.mark.parametrize("slice_rounds", [1, 3])
def test_mix_equals_alone(apsp, slice_rounds):
    import torch

    from paper_1902_04446_amd.serving import ApspServer, GpuBackend

    dev = torch.device("cuda:0")
    sizes = [256, 1024, 300, 700, 129, 2048, 256, 1024, 1]
    reqs = _requests(sizes, 800 + slice_rounds)
    backend = GpuBackend(dev, slots=3, keep_results=True)
    srv = ApspServer(backend, hbm_budget=1 << 30, slots=3, slice_rounds=slice_rounds)
    stats = srv.run(reqs, realtime=False)
    torch.cuda.synchronize()
    assert stats["done"] == len(sizes)
    for r in reqs:
        assert r.status == "done"
        assert torch.equal(r.result, _alone(apsp, r, dev)), r.n
    for r in reqs:
        if r.n <= 300:
            u, v, w = r.payload
            W = gg.dense_from_edges(r.n, u, v, w, np.float32)
            assert np.array_equal(r.result.cpu().numpy(), oracle.blocked(W, apsp.round_width(W.shape[0])))


@pytest.mark.parametrize("slice_rounds", [3, 4])
def test_mix_equals_alone_round_pairs(apsp, slice_rounds):
    """The same kind of mix with round pairs from 2 rounds on: each slice of
    3 or 4 rounds runs as pairs (a 3-round slice ends with a round alone),
    q from 2 to 16, on 3 slot streams at once, each stream with its own panel
    copies.  Every result equals the single-round solve of the request alone."""
    import torch

    from paper_1902_04446_amd.serving import ApspServer, GpuBackend

    dev = torch.device("cuda:0")
    sizes = [1024, 129, 300, 2048, 700, 256, 1100, 513, 1024]
    reqs = _requests(sizes, 850 + slice_rounds)
    backend = GpuBackend(dev, slots=3, keep_results=True)
    srv = ApspServer(backend, hbm_budget=1 << 30, slots=3, slice_rounds=slice_rounds)
    prev_w = apsp.set_width64_max_n(0)  # round pairs run at width 128
    try:
        prev = apsp.set_round_pair_threshold(2)
        try:
            stats = srv.run(reqs, realtime=False)
            torch.cuda.synchronize()
        finally:
            apsp.set_round_pair_threshold(prev)
        assert stats["done"] == len(sizes)
        for r in reqs:  # alone: single rounds, at the same width
            assert r.status == "done"
            assert torch.equal(r.result, _alone(apsp, r, dev)), r.n
    finally:
        apsp.set_width64_max_n(prev_w)


def test_admission_under_small_budget(apsp):
    import torch

    from paper_1902_04446_amd.serving import ApspServer, GpuBackend

    dev = torch.device("cuda:0")
    sizes = [1024, 1024, 1024, 512, 512, 4096]
    reqs = _requests(sizes, 900)
    backend = GpuBackend(dev, slots=4, keep_results=True)
    budget = 2 * backend.bytes_needed(1024) + 1
    srv = ApspServer(backend, hbm_budget=budget, slots=4, slice_rounds=2)
    peak = {"used": 0}
    orig_step = srv.step

    def step(now=None):
        out = orig_step(now)
        peak["used"] = max(peak["used"], srv.used)
        return out

    srv.step = step
    stats = srv.run(reqs, realtime=False)
    torch.cuda.synchronize()
    assert peak["used"] <= budget
    assert reqs[-1].status == "rejected"          # 4096^2 fp32 does not fit at all
    assert stats["done"] == len(sizes) - 1
    for r in reqs[:-1]:
        assert torch.equal(r.result, _alone(apsp, r, dev))

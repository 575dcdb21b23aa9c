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


@pytest.mark.parametrize("policy", ["srpt", "fifo"])
def test_forced_failures_resume_from_checkpoints(apsp, policy):
    """Slices forced to fail from the host (the backend reports the slice
    failed and overwrites the matrix): each such request resumes from its last
    good checkpoint and still ends with the bits of the solve alone."""
    import torch

    from paper_1902_04446_amd.serving import ApspServer, GpuBackend

    dev = torch.device("cuda:0")
    sizes = [1024, 2048, 300, 1100, 256]
    reqs = _requests(sizes, 950)
    # rounds of 64: 16, 32, 5, 18, 4; the failing slices hold these rounds
    fail_at = {0: 9, 1: 21, 3: 4}
    backend = GpuBackend(dev, slots=3, keep_results=True, fail_at=fail_at)
    srv = ApspServer(backend, hbm_budget=1 << 30, slots=3, slice_rounds=3, inflight=2,
                     checkpoint_rounds=6, policy=policy, max_running=2)
    stats = srv.run(reqs, realtime=False)
    torch.cuda.synchronize()
    assert stats["done"] == len(sizes) and srv.used == 0
    assert not backend.fail_at  # every forced failure happened
    for r in reqs:
        assert r.retries == (1 if r.rid in fail_at else 0), r.rid
        assert torch.equal(r.result, _alone(apsp, r, dev)), r.n


def test_stream_state_released_with_the_stream(apsp):
    """A server that creates and drops streams does not accumulate solver
    state: releasing a stream's state frees it (and a later solve on the
    stream recreates it), and the state of a round-pair solve is the size
    apsp_stream_state_bytes reports."""
    import torch

    dev = torch.device("cuda:0")
    n = 300
    u, v, w = gg.swiss_roll_knn(n, gg.CFG_TEST, 990)
    W = gg.dense_from_edges(n, u, v, w, np.int32)
    ref = oracle.fw(W)
    for i in range(5):
        # torch hands out streams from a pool: this one may carry state from
        # earlier solves, so release it first
        s = torch.cuda.Stream(dev)
        apsp.release_stream_state(s)
        base = apsp.stream_state_count()
        D = torch.from_numpy(W).to(dev)
        apsp.solve(D, stream=s)          # int32: keeps the scan word per stream
        assert apsp.stream_state_count() == base + 1
        apsp.release_stream_state(s)
        assert apsp.stream_state_count() == base
        assert np.array_equal(D.cpu().numpy().astype(np.int64), ref)
    s = torch.cuda.Stream(dev)
    apsp.release_stream_state(s)
    before = apsp.stream_state_count()
    apsp.release_stream_state(s)  # no state left: a no-op
    assert apsp.stream_state_count() == before
    # round pairs at width 128 from 3 rounds: the copies come with the state
    prev_w = apsp.set_width64_max_n(0)
    prev_p = apsp.set_round_pair_threshold(3)
    try:
        n = 2048
        u, v, w = gg.swiss_roll_knn(n, gg.CFG_TEST, 991)
        D = gg.device_dense_from_edges(n, u, v, w, np.float32, dev)
        want = apsp.stream_state_bytes(n, apsp.APSP_F32)
        assert want == 256 + 8 * 128 * 2048 * 4
        s = torch.cuda.Stream(dev)
        apsp.release_stream_state(s)
        base = apsp.stream_state_count()
        torch.cuda.synchronize()
        apsp.solve(D, stream=s)
        torch.cuda.synchronize()
        free_before, _ = torch.cuda.mem_get_info(dev)
        apsp.release_stream_state(s)
        free_after, _ = torch.cuda.mem_get_info(dev)
        assert free_after - free_before >= 8 * 128 * 2048 * 4
        assert apsp.stream_state_count() == base
        E = gg.device_dense_from_edges(n, u, v, w, np.float32, dev)
        apsp.solve(E, stream=s)          # recreated on demand, same bits
        torch.cuda.synchronize()
        assert torch.equal(D, E)
        apsp.release_stream_state(s)
    finally:
        apsp.set_round_pair_threshold(prev_p)
        apsp.set_width64_max_n(prev_w)
    assert apsp.stream_state_count() == base

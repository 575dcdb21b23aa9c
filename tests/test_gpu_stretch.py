"""The largest single-GPU problem: n = 262144 (a 256 GiB fp32 matrix in HBM).

A full solve takes minutes, so the test runs the first rounds of the blocked
method in the launch configuration the benchmark times (apsp_solve_rounds,
round width 128) and checks sampled rows of the state they leave against the
host oracle: after rounds 0..R-1 the matrix is the Floyd-Warshall state after
pivots 0..128R-1, whose rows the oracle builds from the adjacency lists.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N = 262144
ROUNDS = 3
REL_TOL = 1e-5


@pytest.mark.parametrize("hubs", [False, True])
def test_stretch_262144_first_rounds(hubs):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    need = N * N * 4
    free, _ = torch.cuda.mem_get_info()
    if free < need + (4 << 30):
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory, {free / 2**30:.0f} free")
    import paper_1902_04446_amd as apsp

    u, v, w = gg.swiss_roll_knn(N, gg.CFG_SWISS_256K, 0)
    if hubs:
        u, v, w = gg.with_hub_edges(N, u, v, w, ROUNDS * apsp.round_width(N),
                                    gg.rng_for(gg.CFG_TEST, 7))
    D = gg.device_dense_from_edges(N, u, v, w, np.float32, "cuda:0")
    apsp.solve_rounds(D, 0, ROUNDS)
    torch.cuda.synchronize()
    K = ROUNDS * apsp.round_width(N)
    rows = np.array([0, 77, K - 1, K, 100003, N - 1], np.int64)
    got = D[torch.as_tensor(rows, device=D.device)].cpu().numpy().astype(np.float64)
    del D
    torch.cuda.empty_cache()
    ref = oracle.fw_prefix_rows(gg.csr_from_edges(N, u, v, w), N, K, rows, threads=8)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(got)), "reachability differs"
    rel = np.abs(got[fin] - ref[fin]) / np.maximum(ref[fin], 1e-300)
    assert (got[fin][ref[fin] == 0] == 0).all()
    print(f"n={N}, {ROUNDS} rounds, hubs={hubs}: {fin.sum()} finite sampled entries, "
          f"max rel err {rel.max():.3e}")
    if hubs:
        assert fin.mean() > 0.99
    assert rel.max() <= REL_TOL

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


def _with_hubs(u, v, w, K, seed):
    """The kNN edges plus a star from vertex 0 to vertices 1..K-1 and an edge
    from every other vertex j to vertex j % K, so that after the first K
    pivots most entries are finite (a kNN graph alone leaves nearly all of
    them "no edge") through paths of a few hops."""
    rng = gg.rng_for(gg.CFG_TEST, seed)
    j = np.arange(K, N, dtype=np.int64)
    hu = np.concatenate([np.zeros(K - 1, dtype=np.int64), j])
    hv = np.concatenate([np.arange(1, K, dtype=np.int64), j % K])
    hw = rng.uniform(0.5, 1.5, size=hu.size).astype(np.float32)
    u, v = np.asarray(u, np.int64), np.asarray(v, np.int64)
    key = np.minimum(u, v) * N + np.maximum(u, v)
    hkey = np.minimum(hu, hv) * N + np.maximum(hu, hv)
    keep = ~np.isin(hkey, key)  # no parallel edges
    return (np.concatenate([u, hu[keep]]), np.concatenate([v, hv[keep]]),
            np.concatenate([np.asarray(w, np.float32), hw[keep]]))


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
        u, v, w = _with_hubs(u, v, w, ROUNDS * apsp.round_width(N), 7)
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

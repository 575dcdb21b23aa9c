"""Pins for the host oracle (CPU only).

The paper prints no worked example or distance values, so the oracle is
pinned by what the mathematics fixes: brute force over simple paths (the
definition itself), Dijkstra (an independent algorithm), closed forms,
invariants, the Bellman certificate, metamorphic relations, and an external
library (scipy's csgraph, run, not copied).  ``test_mutants_are_caught``
builds oracle variants with one planted mistake each and checks that these
pins reject every one of them.
"""
import math

import numpy as np
import pytest

import graphgen as gg
import oracle

INF = oracle.INF_I32


def _rand_int_graph(n, p, wlo, whi, seed):
    rng = gg.rng_for(gg.CFG_TEST, seed)
    u, v, w = gg.er_edges(n, p, wlo, whi, rng)
    return gg.dense_from_edges(n, u, v, w, np.int32), (u, v, w)


def _rand_dyadic_f32(n, p, seed):
    # weights k/8: every path sum is exact in fp32 and fp64
    rng = gg.rng_for(gg.CFG_TEST, 5000 + seed)
    u, v, w = gg.er_edges(n, p, 0, 64, rng)
    return gg.dense_from_edges(n, u, v, (w / 8.0).astype(np.float32), np.float32), (u, v, w)


def _brute_as_int(B):
    return np.where(np.isinf(B), INF, B).astype(np.int64)


# ---------------------------------------------------------------- definition

@pytest.mark.parametrize("seed", range(40))
def test_brute_force_int(seed):
    n = 1 + seed % 8
    p = [0.2, 0.4, 0.7, 1.0][seed % 4]
    W, (u, v, w) = _rand_int_graph(n, p, 0 if seed % 3 == 0 else 1, 9, seed)
    ref = _brute_as_int(oracle.brute(W))
    assert np.array_equal(oracle.fw(W), ref)
    csr = gg.csr_from_edges(n, u, v, w)
    assert np.array_equal(oracle.dijkstra(csr, n, np.arange(n), integer=True), ref)
    for b in (1, 2, 3, n):
        assert np.array_equal(oracle.blocked(W, b).astype(np.int64), ref)


@pytest.mark.parametrize("seed", range(20))
def test_brute_force_f32_dyadic(seed):
    n = 2 + seed % 7
    W, _ = _rand_dyadic_f32(n, 0.5, seed)
    ref = oracle.brute(W)
    assert np.array_equal(oracle.fw(W), ref)
    for b in (1, 3, n):
        assert np.array_equal(oracle.blocked(W, b).astype(np.float64), ref)


def test_brute_force_directed():
    # The method also applies when symmetry is dropped (directed graphs).
    rng = gg.rng_for(gg.CFG_TEST, 77)
    for trial in range(20):
        n = 2 + trial % 7
        W = rng.integers(1, 20, size=(n, n)).astype(np.int32)
        W[rng.random((n, n)) < 0.5] = INF
        ref = _brute_as_int(oracle.brute(W))
        assert np.array_equal(oracle.fw(W), ref)
        assert np.array_equal(oracle.blocked(W, 3).astype(np.int64), ref)


# ------------------------------------------------------------- closed forms

def _path(n, w, dtype):
    i = np.arange(n - 1)
    return gg.dense_from_edges(n, i, i + 1, np.full(n - 1, w, dtype), dtype)


def _cycle(n, w, dtype):
    i = np.arange(n)
    return gg.dense_from_edges(n, i, (i + 1) % n, np.full(n, w, dtype), dtype)


def _grid(r, c, dtype):
    idx = np.arange(r * c).reshape(r, c)
    u = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    v = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    return gg.dense_from_edges(r * c, u, v, np.ones(u.size, dtype), dtype)


@pytest.mark.parametrize("dtype", [np.int32, np.float32])
@pytest.mark.parametrize("n", [1, 2, 5, 64, 97])
def test_closed_forms(dtype, n):
    w = 3 if dtype == np.int32 else 0.5
    i = np.arange(n)
    dist = np.abs(i[:, None] - i[None, :])
    got = oracle.fw(_path(n, w, dtype)) if n > 1 else oracle.fw(np.zeros((1, 1), dtype))
    assert np.array_equal(got, dist * w)
    if n >= 3:
        cyc = np.minimum(dist, n - dist) * w
        assert np.array_equal(oracle.fw(_cycle(n, w, dtype)), cyc)
        assert np.array_equal(oracle.blocked(_cycle(n, w, dtype), 16).astype(np.float64), cyc)
        # star centred at 0: 1 to the centre, 2 between leaves
        star = gg.dense_from_edges(n, np.zeros(n - 1, np.int64), np.arange(1, n),
                                   np.ones(n - 1, dtype), dtype)
        exp = np.full((n, n), 2)
        exp[0, :] = 1
        exp[:, 0] = 1
        np.fill_diagonal(exp, 0)
        assert np.array_equal(oracle.fw(star), exp)
        # complete graph with unit weights
        iu, ju = np.triu_indices(n, 1)
        comp = gg.dense_from_edges(n, iu, ju, np.ones(iu.size, dtype), dtype)
        assert np.array_equal(oracle.fw(comp), 1 - np.eye(n))
    # empty graph: unreachable everywhere off the diagonal
    empty = gg.dense_from_edges(n, [], [], np.zeros(0, dtype), dtype)
    unreach = INF if dtype == np.int32 else np.inf
    exp = np.full((n, n), unreach, dtype=np.float64)
    np.fill_diagonal(exp, 0)
    assert np.array_equal(oracle.fw(empty).astype(np.float64), exp)


def test_grid_manhattan():
    r, c = 9, 13
    G = _grid(r, c, np.int32)
    y, x = np.divmod(np.arange(r * c), c)
    man = np.abs(y[:, None] - y[None, :]) + np.abs(x[:, None] - x[None, :])
    assert np.array_equal(oracle.fw(G), man)
    assert np.array_equal(oracle.blocked(G, 10).astype(np.int64), man)


def test_disjoint_union_is_unreachable_across():
    A = _path(30, 2, np.int32)
    B = _cycle(20, 5, np.int32)
    n = 50
    W = np.full((n, n), INF, np.int32)
    W[:30, :30] = A
    W[30:, 30:] = B
    D = oracle.fw(W)
    assert (D[:30, 30:] == INF).all() and (D[30:, :30] == INF).all()
    assert np.array_equal(D[:30, :30], oracle.fw(A))
    assert np.array_equal(D[30:, 30:], oracle.fw(B))


def test_saturation_at_inf():
    # A path whose true length exceeds 2^30 is reported as 2^30 (unreachable).
    w = (1 << 29) + 7
    W = _path(4, w, np.int32)
    D = oracle.fw(W)
    assert D[0, 1] == w and D[0, 2] == INF and D[0, 3] == INF
    assert np.array_equal(oracle.blocked(W, 2).astype(np.int64), D)
    # entries above 2^30 on input mean "no edge"
    W2 = W.copy()
    W2[0, 1] = W2[1, 0] = np.int32(2**31 - 1)
    assert oracle.fw(W2)[0, 1] == INF


# --------------------------------------------------- independent algorithms

@pytest.mark.parametrize("seed", range(3))
def test_dijkstra_vs_fw_int(seed):
    n = 300 + 37 * seed
    W, (u, v, w) = _rand_int_graph(n, 0.02, 1, 100, 100 + seed)
    D = oracle.fw(W, threads=4)
    csr = gg.csr_from_edges(n, u, v, w)
    assert np.array_equal(oracle.dijkstra(csr, n, np.arange(n), threads=4, integer=True), D)


def test_dijkstra_vs_fw_swiss_f32():
    n = 500
    u, v, w = gg.swiss_roll_knn(n, gg.CFG_TEST, 3)
    W = gg.dense_from_edges(n, u, v, w, np.float32)
    D = oracle.fw(W, threads=4)
    csr = gg.csr_from_edges(n, u, v, w)
    Dj = oracle.dijkstra(csr, n, np.arange(n), threads=4)
    fin = np.isfinite(D)
    assert np.array_equal(fin, np.isfinite(Dj))
    rel = np.abs(D[fin] - Dj[fin]) / np.maximum(D[fin], 1e-300)
    assert rel.max() <= 1e-12


def test_scipy_csgraph_agrees():
    from scipy.sparse.csgraph import shortest_path

    n = 257
    W, _ = _rand_int_graph(n, 0.03, 1, 50, 9)
    dense = np.where(W >= INF, 0, W).astype(np.float64)  # csgraph: 0 = no edge
    S = shortest_path(dense, method="D", directed=False)
    assert np.array_equal(np.where(np.isinf(S), INF, S).astype(np.int64), oracle.fw(W))


# ------------------------------------------------------------------- blocked

@pytest.mark.parametrize("n,b", [(1, 1), (2, 1), (7, 3), (64, 8), (97, 16), (130, 64),
                                 (129, 128), (128, 128), (50, 200), (200, 33)])
def test_blocked_equals_fw_int(n, b):
    W, _ = _rand_int_graph(n, 0.06, 1, 100, 1000 + n + b)
    assert np.array_equal(oracle.blocked(W, b).astype(np.int64), oracle.fw(W))


@pytest.mark.parametrize("n,b", [(97, 16), (130, 64), (200, 33)])
def test_blocked_f32_within_tolerance_of_fp64(n, b):
    u, v, w = gg.swiss_roll_knn(n, gg.CFG_TEST, n)
    W = gg.dense_from_edges(n, u, v, w, np.float32)
    D = oracle.fw(W)
    B = oracle.blocked(W, b).astype(np.float64)
    fin = np.isfinite(D)
    assert np.array_equal(fin, np.isfinite(B))
    assert (np.abs(B[fin] - D[fin]) <= 1e-5 * D[fin]).all()
    assert (np.diag(B) == 0).all()


@pytest.mark.parametrize("n,b", [(100, 16), (130, 32), (64, 64)])
def test_blocked_round_state_matches_fw_prefix(n, b):
    # After round r the blocked state equals Floyd-Warshall stopped after
    # pivots 0..min((r+1)b, n)-1 (the invariant of the three-phase method).
    W, _ = _rand_int_graph(n, 0.05, 1, 100, 2000 + n)
    q = -(-n // b)
    state = oracle.blocked(W, b, 0, 0)
    fw_state = oracle.prepare(W)
    for r in range(q):
        state = oracle.blocked(state, b, r, r + 1)
        oracle.fw_steps(fw_state, r * b, min((r + 1) * b, n))
        assert np.array_equal(state.astype(np.int64), np.minimum(fw_state, INF))


@pytest.mark.parametrize("n,K", [(1, 0), (1, 1), (60, 0), (60, 1), (120, 17), (150, 64),
                                 (97, 97), (200, 300)])
def test_fw_prefix_rows_match_stopped_loop(n, K):
    # Rows of the state after pivots 0..K-1, built from adjacency lists by
    # splitting paths at their first and last intermediate vertex, equal the
    # classic loop stopped after K pivots (different algorithm, same state).
    W, (u, v, w) = _rand_int_graph(n, 0.05, 1, 100, 3000 + n + K)
    fw_state = np.minimum(oracle.fw_steps(oracle.prepare(W), 0, min(K, n)), INF)
    csr = gg.csr_from_edges(n, u, v, w)
    rows = np.arange(n)
    P = oracle.fw_prefix_rows(csr, n, K, rows, threads=4)
    assert np.array_equal(np.where(np.isinf(P), INF, P).astype(np.int64), fw_state)


def test_fw_prefix_rows_directed_and_full():
    # directed adjacency lists; K = n is the full solve (Dijkstra)
    n = 140
    rng = gg.rng_for(gg.CFG_TEST, 3100)
    W = rng.integers(1, 60, size=(n, n)).astype(np.int32)
    W[rng.random((n, n)) > 0.04] = INF
    csr = oracle.csr_from_dense(W)
    for K in (0, 5, 70):
        P = oracle.fw_prefix_rows(csr, n, K, np.arange(n))
        ref = np.minimum(oracle.fw_steps(oracle.prepare(W), 0, K), INF)
        assert np.array_equal(np.where(np.isinf(P), INF, P).astype(np.int64), ref), K
    P = oracle.fw_prefix_rows(csr, n, n, [0, 7, 139])
    D = oracle.dijkstra(csr, n, [0, 7, 139], integer=True)
    assert np.array_equal(np.where(np.isinf(P), INF, P).astype(np.int64), D)


def test_minplus_matches_definition():
    rng = gg.rng_for(gg.CFG_TEST, 42)
    A = rng.random((13, 7)).astype(np.float32)
    B = rng.random((7, 11)).astype(np.float32)
    C = rng.random((13, 11)).astype(np.float32)
    A[0, :] = np.inf
    ref = np.minimum(C, np.min(A[:, :, None] + B[None, :, :], axis=1))
    assert np.array_equal(oracle.minplus_acc(C, A, B), ref)
    Ai = rng.integers(0, INF + 1, (9, 5)).astype(np.int32)
    Bi = rng.integers(0, INF + 1, (5, 6)).astype(np.int32)
    Ci = rng.integers(0, INF + 1, (9, 6)).astype(np.int32)
    refi = np.minimum(Ci, np.min(Ai[:, :, None].astype(np.int64) + Bi[None], axis=1))
    assert np.array_equal(oracle.minplus_acc(Ci, Ai, Bi).astype(np.int64), refi)


@pytest.mark.parametrize("n", [1, 2, 3, 9, 64, 130])
def test_squaring_int_equals_fw(n):
    W, _ = _rand_int_graph(n, min(1.0, 3.0 / n), 1, 100, 4000 + n)
    assert np.array_equal(oracle.squaring(W).astype(np.int64), oracle.fw(W))


def test_squaring_step_count_is_minimal_on_a_path():
    # a path of n vertices needs paths of n-1 edges: ceil(log2(n-1)) squarings
    # reach the far end, one fewer does not
    for n in (3, 4, 5, 9, 17, 33, 70):
        W = _path(n, 1, np.int32)
        s = oracle.squaring_steps(n)
        assert (1 << s) >= n - 1 and (s == 0 or (1 << (s - 1)) < n - 1)
        assert oracle.squaring(W, s)[0, n - 1] == n - 1
        if s:
            assert oracle.squaring(W, s - 1)[0, n - 1] == INF


def test_squaring_f32_within_tolerance():
    n = 150
    u, v, w = gg.swiss_roll_knn(n, gg.CFG_TEST, 4100)
    W = gg.dense_from_edges(n, u, v, w, np.float32)
    D = oracle.fw(W)
    S = oracle.squaring(W).astype(np.float64)
    fin = np.isfinite(D)
    assert np.array_equal(fin, np.isfinite(S))
    assert (np.abs(S[fin] - D[fin]) <= 1e-5 * D[fin]).all()


# ------------------------------------------------------- invariants / Bellman

def _check_invariants(W, D):
    n = W.shape[0]
    Wp = oracle.prepare(W).astype(np.float64)
    Df = D.astype(np.float64)
    assert (np.diag(Df) == 0).all()
    assert np.array_equal(Df, Df.T)
    assert (Df <= Wp).all()
    # triangle inequality D_ij <= D_ik + D_kj over all triples (n small)
    for k in range(n):
        assert (Df <= Df[:, k:k + 1] + Df[k:k + 1, :]).all()


def test_invariants_hold():
    W, _ = _rand_int_graph(150, 0.03, 1, 100, 31)
    _check_invariants(W, oracle.fw(W))
    u, v, w = gg.swiss_roll_knn(150, gg.CFG_TEST, 31)
    Wf = gg.dense_from_edges(150, u, v, w, np.float32)
    _check_invariants(Wf, oracle.fw(Wf))


def test_bellman_certificate():
    n = 220
    W, (u, v, w) = _rand_int_graph(n, 0.03, 1, 100, 51)
    csr = gg.csr_from_edges(n, u, v, w)
    D = oracle.fw(W).astype(np.int32)
    assert oracle.bellman_violations_i32(D, csr, np.arange(n)) == 0
    bad = D.copy()
    i, j = np.argwhere((bad > 0) & (bad < INF))[5]
    bad[i, j] -= 1
    assert oracle.bellman_violations_i32(bad, csr, np.arange(n)) > 0
    uf, vf, wf = gg.swiss_roll_knn(n, gg.CFG_TEST, 52)
    Wf = gg.dense_from_edges(n, uf, vf, wf, np.float32)
    csrf = gg.csr_from_edges(n, uf, vf, wf)
    Df = oracle.fw(Wf).astype(np.float32)
    assert oracle.bellman_residual_f32(Df, csrf, np.arange(n)) <= 1e-6
    badf = Df.copy()
    badf[3, 7] *= np.float32(1.01)
    assert oracle.bellman_residual_f32(badf, csrf, np.arange(n)) > 1e-3


# ------------------------------------------------------------- metamorphic

def test_permutation_equivariance():
    n = 120
    W, _ = _rand_int_graph(n, 0.05, 1, 100, 61)
    perm = gg.rng_for(gg.CFG_TEST, 62).permutation(n)
    D = oracle.fw(W)
    Dp = oracle.fw(np.ascontiguousarray(W[np.ix_(perm, perm)]))
    assert np.array_equal(Dp, D[np.ix_(perm, perm)])
    assert np.array_equal(oracle.blocked(np.ascontiguousarray(W[np.ix_(perm, perm)]), 32)
                          .astype(np.int64), D[np.ix_(perm, perm)])


def test_scaling_by_power_of_two_is_exact():
    n = 150
    u, v, w = gg.swiss_roll_knn(n, gg.CFG_TEST, 63)
    W = gg.dense_from_edges(n, u, v, w, np.float32)
    B = oracle.blocked(W, 32)
    B8 = oracle.blocked(W * np.float32(8.0), 32)
    assert np.array_equal(B8, B * np.float32(8.0))


def test_idempotence_and_monotonicity():
    n = 130
    W, (u, v, w) = _rand_int_graph(n, 0.04, 1, 100, 64)
    D = oracle.fw(W)
    assert np.array_equal(oracle.fw(D.astype(np.int32)), D)
    W2 = W.copy()
    W2[0, n - 1] = W2[n - 1, 0] = 1
    D2 = oracle.fw(W2)
    assert (D2 <= D).all() and D2[0, n - 1] == 1


def test_paper_workload_reference_digest():
    """Digest of the ER n=512 workload and its oracle solution (regression anchor).

    Stored by tests/golden/make_golden.py, which calls only graphgen and oracle.
    """
    import hashlib
    import json
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "plain_small_digest.json")
    with open(path) as f:
        gold = json.load(f)
    W, _ = gg.plain_small(0)
    assert hashlib.sha256(np.ascontiguousarray(W).tobytes()).hexdigest() == gold["input_sha256"]
    D = oracle.fw(W, threads=4).astype(np.int32)
    assert hashlib.sha256(D.tobytes()).hexdigest() == gold["output_sha256"]
    assert int(D.astype(np.int64).sum()) == gold["sum"]
    assert int(D.max()) == gold["max"]


def test_metric_definition_matches_paper():
    """The throughput metric is n^3 / t (Sec. 5.4); the paper's own figures follow."""
    import json
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "paper_metric.json")
    with open(path) as f:
        gold = json.load(f)
    from bench import cell_updates_per_s

    t1 = gold["T1"]
    # printed to three decimals (truncated): 256^3 / 0.022 s = 0.7626e9
    assert math.floor(cell_updates_per_s(t1["n"], t1["seconds"]) / 1e6) / 1e3 == t1["gops"]
    cb = gold["blocked_cb_p1024"]
    per_core = cell_updates_per_s(cb["n"], cb["seconds"]) / cb["cores"] / 1e9
    # the paper truncates: 0.5996 / 0.762 = 78.7%, printed as 78%
    assert math.floor(100 * per_core / t1["gops"]) == cb["percent_of_T1_per_core"]


# ----------------------------------------------------------------- mutants

def _pins_pass(mutant):
    """A compact subset of the pins above, run against an oracle build."""
    rng = gg.rng_for(gg.CFG_TEST, 301)
    for seed in range(12):
        n = 3 + seed % 6
        W, _ = _rand_int_graph(n, 0.5, 1, 9, 300 + seed)
        if not np.array_equal(oracle.fw(W, mutant=mutant), _brute_as_int(oracle.brute(W))):
            return False
        Wf, _ = _rand_dyadic_f32(n, 0.5, 300 + seed)
        if not np.array_equal(oracle.fw(Wf, mutant=mutant), oracle.brute(Wf)):
            return False
        # directed weights and a non-zero input diagonal (which must be ignored)
        Wd = rng.integers(1, 20, size=(n, n)).astype(np.int32)
        Wd[rng.random((n, n)) < 0.4] = INF
        if not np.array_equal(oracle.fw(Wd, mutant=mutant), _brute_as_int(oracle.brute(Wd))):
            return False
    return True


def test_unmutated_oracle_passes_compact_pins():
    assert _pins_pass(0)


@pytest.mark.parametrize("mutant", [1, 2, 3, 4, 5])
def test_mutants_are_caught(mutant):
    assert not _pins_pass(mutant), f"planted mistake {mutant} was not detected"

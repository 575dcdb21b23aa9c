"""Parity of the HIP path (through the C ABI) with the host oracle, on an MI355X.

int32 results must equal the oracle bit for bit.  fp32 results must equal the
oracle's blocked fp32 model at the same round width bit for bit (every
candidate is one IEEE add and the minimum is exact, so tile shapes and k order
cannot change bits), and lie within 1e-5 relative of the fp64 oracle.  At the
full workload sizes the oracle checks sampled rows (Dijkstra from sampled
sources) and the Bellman certificate on them.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

INF = oracle.INF_I32
REL_TOL = 1e-5


@pytest.fixture(scope="module")
def apsp():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1902_04446_amd as mod

    return mod


@pytest.fixture(scope="module")
def dev(apsp):
    import torch

    return torch.device("cuda:0")


def _to_dev(W, dev, ld=None, offset=0):
    """Copy a host matrix into a device buffer with leading dimension ld,
    starting ``offset`` elements into the allocation; returns (view, buffer)."""
    import torch

    n = W.shape[0]
    ld = n if ld is None else ld
    tdt = torch.int32 if W.dtype == np.int32 else torch.float32
    fill = -7 if tdt == torch.int32 else -3.5  # sentinel for the untouched padding
    buf = torch.full((offset + max(n, 1) * max(ld, 1),), fill, dtype=tdt, device=dev)
    view = buf[offset:offset + n * ld].view(n, ld)[:, :n] if n else buf[:0].view(0, 0)
    if n:
        view.copy_(torch.from_numpy(np.ascontiguousarray(W)).to(dev))
    return view, buf


def _solve(apsp, W, dev, **kw):
    import torch

    view, _ = _to_dev(W, dev, **kw)
    apsp.solve(view)
    torch.cuda.synchronize()
    return view.cpu().numpy()


def _assert_f32_close(got, ref64):
    fin = np.isfinite(ref64)
    assert np.array_equal(fin, np.isfinite(got)), "reachability differs"
    rel = np.abs(got[fin].astype(np.float64) - ref64[fin]) / np.maximum(ref64[fin], 1e-300)
    exact_zero = ref64[fin] == 0
    assert (got[fin][exact_zero] == 0).all()
    assert rel.max(initial=0.0) <= REL_TOL, f"max rel err {rel.max():.3e}"
    return float(rel.max(initial=0.0))


def _er(n, p, seed, wlo=1, whi=100):
    u, v, w = gg.er_edges(n, p, wlo, whi, gg.rng_for(gg.CFG_TEST, seed))
    return gg.dense_from_edges(n, u, v, w, np.int32), (u, v, w)


def _swiss(n, seed):
    u, v, w = gg.swiss_roll_knn(n, gg.CFG_TEST, seed)
    return gg.dense_from_edges(n, u, v, w, np.float32), (u, v, w)


# ------------------------------------------------------------ small config

@pytest.mark.parametrize("item", range(5))
def test_er512_int32_bit_exact(apsp, dev, item):
    W, _ = gg.plain_small(item)
    got = _solve(apsp, W, dev)
    assert np.array_equal(got.astype(np.int64), oracle.fw(W, threads=8))


@pytest.mark.parametrize("n", [1, 2, 3, 64, 127, 128, 129, 255, 256, 257, 384, 500])
def test_shapes_int32(apsp, dev, n):
    W, _ = _er(n, min(1.0, 3.0 / max(n, 1)), 100 + n)
    got = _solve(apsp, W, dev)
    assert np.array_equal(got.astype(np.int64), oracle.fw(W, threads=8))


@pytest.mark.parametrize("n", [1, 2, 129, 256, 300, 513])
def test_shapes_fp32(apsp, dev, n):
    W, _ = _swiss(n, 200 + n) if n > 11 else (np.zeros((n, n), np.float32), None)
    got = _solve(apsp, W, dev)
    assert np.array_equal(got, oracle.blocked(W, apsp.round_width(n, apsp.APSP_F32)))
    _assert_f32_close(got, oracle.fw(W, threads=8))


@pytest.mark.parametrize("ld_extra,offset", [(1, 0), (4, 0), (212, 0), (0, 1), (3, 3)])
def test_leading_dimension_and_alignment(apsp, dev, ld_extra, offset):
    import torch

    n = 300
    Wi, _ = _er(n, 0.02, 7)
    Wf, _ = _swiss(n, 8)
    for W in (Wi, Wf):
        view, buf = _to_dev(W, dev, ld=n + ld_extra, offset=offset)
        before = buf.clone()
        apsp.solve(view)
        torch.cuda.synchronize()
        got = view.cpu().numpy()
        if W.dtype == np.int32:
            assert np.array_equal(got.astype(np.int64), oracle.fw(W, threads=8))
        else:
            assert np.array_equal(got, oracle.blocked(W, apsp.round_width(n)))
        # nothing outside the n x n view was written
        mask = torch.ones_like(buf, dtype=torch.bool)
        mask[offset:offset + n * (n + ld_extra)].view(n, n + ld_extra)[:, :n] = False
        assert torch.equal(buf[mask], before[mask])


# ------------------------------------------------------------ closed forms

def test_closed_forms_on_device(apsp, dev):
    n = 1000
    i = np.arange(n)
    path = gg.dense_from_edges(n, i[:-1], i[1:], np.full(n - 1, 3, np.int32), np.int32)
    assert np.array_equal(_solve(apsp, path, dev).astype(np.int64),
                          3 * np.abs(i[:, None] - i[None, :]))
    n = 777
    i = np.arange(n)
    cyc = gg.dense_from_edges(n, i, (i + 1) % n, np.full(n, 0.5, np.float32), np.float32)
    d = np.abs(i[:, None] - i[None, :])
    assert np.array_equal(_solve(apsp, cyc, dev), (np.minimum(d, n - d) * 0.5).astype(np.float32))
    r, c = 30, 41
    idx = np.arange(r * c).reshape(r, c)
    u = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    v = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    grid = gg.dense_from_edges(r * c, u, v, np.ones(u.size, np.int32), np.int32)
    y, x = np.divmod(np.arange(r * c), c)
    man = np.abs(y[:, None] - y[None, :]) + np.abs(x[:, None] - x[None, :])
    assert np.array_equal(_solve(apsp, grid, dev).astype(np.int64), man)
    # disjoint components stay unreachable; empty graph
    empty = gg.dense_from_edges(200, [], [], np.zeros(0, np.int32), np.int32)
    exp = np.full((200, 200), INF)
    np.fill_diagonal(exp, 0)
    assert np.array_equal(_solve(apsp, empty, dev).astype(np.int64), exp)


def test_directed_int32(apsp, dev):
    rng = gg.rng_for(gg.CFG_TEST, 4242)
    n = 333
    W = rng.integers(1, 1000, size=(n, n)).astype(np.int32)
    W[rng.random((n, n)) > 0.015] = INF
    assert np.array_equal(_solve(apsp, W, dev).astype(np.int64), oracle.fw(W, threads=8))


def test_saturation_and_large_sentinels(apsp, dev):
    w = (1 << 29) + 7
    n = 200
    i = np.arange(n)
    W = gg.dense_from_edges(n, i[:-1], i[1:], np.full(n - 1, w, np.int32), np.int32)
    W[5, 100] = np.int32(2**31 - 1)  # above the sentinel: "no edge"
    assert np.array_equal(_solve(apsp, W, dev).astype(np.int64), oracle.fw(W))


# ------------------------------------------------- rounds, resume, profiling

def test_round_state_matches_fw_prefix(apsp, dev):
    import torch

    n = 400
    W, _ = _er(n, 0.01, 31)
    b = apsp.round_width(n, apsp.APSP_I32)
    for r in (1, 2, 3):
        view, _ = _to_dev(W, dev)
        apsp.solve_rounds(view, 0, r)
        torch.cuda.synchronize()
        ref = oracle.prepare(W)
        oracle.fw_steps(ref, 0, min(r * b, n))
        assert np.array_equal(view.cpu().numpy().astype(np.int64), np.minimum(ref, INF))


def test_resume_equals_full_solve(apsp, dev):
    import torch

    n = 700
    W, _ = _swiss(n, 32)
    full = _solve(apsp, W, dev)
    view, _ = _to_dev(W, dev)
    q = apsp.num_rounds(n)
    apsp.solve_rounds(view, 0, 2)
    torch.cuda.synchronize()
    snapshot = view.cpu().numpy()
    # checkpoint -> fresh buffer -> resume
    view2, _ = _to_dev(snapshot, dev)
    apsp.solve_rounds(view2, 2, q)
    torch.cuda.synchronize()
    assert np.array_equal(view2.cpu().numpy(), full)


@pytest.mark.parametrize("w64", [True, False])
def test_profiled_equals_plain_and_is_deterministic(apsp, dev, w64):
    """Profiled and plain solves agree bit for bit and repeat exactly: in 11
    rounds of 64 (each round's whole phase 3 on the caller's stream) and in
    6 rounds of 128 (the rest of phase 3 beside the next round's phases)."""
    import torch

    n = 700
    W, _ = _swiss(n, 33)
    prev = apsp.set_width64_max_n(5120 if w64 else 0)
    try:
        a = _solve(apsp, W, dev)
        view, _ = _to_dev(W, dev)
        t = apsp.solve_profiled(view)
        assert np.array_equal(view.cpu().numpy(), a)
        assert all(t[k] >= 0 for k in t) and t["total"] > 0 and t["phase3"] > 0
        q = apsp.num_rounds(n)
        assert q == (11 if w64 else 6)
        assert t["phase3_rest_launches"] == (0 if w64 else q - 1)
        b = _solve(apsp, W, dev)
        assert a.tobytes() == b.tobytes()
        torch.cuda.synchronize()
    finally:
        apsp.set_width64_max_n(prev)


def test_validate(apsp, dev):
    import torch

    W, _ = _er(100, 0.05, 34)
    view, _ = _to_dev(W, dev)
    assert apsp.validate(view)
    view[3, 4] = -1
    assert not apsp.validate(view)
    Wf, _ = _swiss(100, 35)
    vf, _ = _to_dev(Wf, dev)
    assert apsp.validate(vf)
    vf[1, 2] = float("nan")
    assert not apsp.validate(vf)
    vf[1, 2] = -0.0
    assert apsp.validate(vf)
    vf[7, 7] = -2.0
    assert not apsp.validate(vf)
    torch.cuda.synchronize()


# ------------------------------------------------------------- full sizes

def _full_size_swiss(apsp, dev, n, cfg, nsrc, bellman_rows=0):
    import torch

    u, v, w = gg.swiss_roll_knn(n, cfg, 0)
    D = gg.device_dense_from_edges(n, u, v, w, np.float32, dev)
    apsp.solve(D)  # the configuration the benchmark times
    torch.cuda.synchronize()
    csr = gg.csr_from_edges(n, u, v, w)
    rng = gg.rng_for(gg.CFG_TEST, n)
    src = np.concatenate([[0, n - 1], rng.choice(np.arange(1, n - 1), size=nsrc, replace=False)])
    tsrc = torch.as_tensor(src, device=dev)
    rows = D[tsrc].cpu().numpy()
    cols = D[:, tsrc].cpu().numpy().T
    ref = oracle.dijkstra(csr, n, src, threads=16)
    worst = _assert_f32_close(rows, ref)
    assert (rows[np.arange(src.size), src] == 0).all()
    # undirected input: column i holds the same lengths as row i
    _assert_f32_close(cols, ref)
    bell = None
    if bellman_rows:
        host = D.cpu().numpy()
        brows = np.concatenate([src, rng.choice(n, size=bellman_rows, replace=False)])
        bell = oracle.bellman_residual_f32(host, csr, brows, threads=16)
        assert bell <= REL_TOL, f"Bellman residual {bell:.3e}"
    return worst, bell


def test_full_size_swiss_16384(apsp, dev):
    worst, bell = _full_size_swiss(apsp, dev, 16384, gg.CFG_SWISS_16K, 48, bellman_rows=2000)
    print(f"n=16384 fp32: max rel err vs fp64 Dijkstra on sampled rows {worst:.3e}; "
          f"Bellman residual {bell:.3e}")


def test_full_size_swiss_ragged_16461(apsp, dev):
    """n = 16461 = 128 * 128 + 77 fp32: 64 round pairs, then the partial last
    round alone."""
    worst, _ = _full_size_swiss(apsp, dev, 16461, gg.CFG_TEST, 16)
    print(f"n=16461 fp32: max rel err vs fp64 Dijkstra on sampled rows {worst:.3e}")


@pytest.mark.slow
def test_full_size_swiss_65536(apsp, dev):
    worst, _ = _full_size_swiss(apsp, dev, 65536, gg.CFG_SWISS_64K, 16)
    print(f"n=65536 fp32: max rel err vs fp64 Dijkstra on sampled rows {worst:.3e}")


@pytest.mark.parametrize("n,whi,diag", [
    (65, 131071, 0),        # 2*64*131071 = 2^24 - 128: fp32 pipe
    (65, 131072, 0),        # 2^24: uint32
    (300, 1 << 21, 0),      # far above the bound
    (200, 1000, 1 << 29),   # huge diagonal entries are not weights
    (150, 1 << 29, 0),      # sums reach 2^30: saturation
    (1000, 1000, 0),        # lookahead, fp32 pipe
    (2100, 3, 0),           # 17 rounds
])
def test_int32_fp32_pipe_bound_single(apsp, dev, n, whi, diag):
    """apsp_solve takes the fp32 pipe for int32 only when exact: results equal
    the oracle bit for bit on both sides of 2 (n-1) wmax < 2^24."""
    rng = gg.rng_for(gg.CFG_TEST, 1400 + n + whi)
    W = rng.integers(max(1, whi // 2), whi + 1, size=(n, n), dtype=np.int64)
    W[rng.random((n, n)) > min(1.0, 6.0 / n)] = INF
    np.fill_diagonal(W, diag)
    W = W.astype(np.int32)
    assert np.array_equal(_solve(apsp, W, dev).astype(np.int64), oracle.fw(W, threads=4))


def test_int32_slices_switch_pipes(apsp, dev):
    """A solve split in round slices rescans each slice's starting matrix: the
    input qualifies for the fp32 pipe, later states (larger lengths) may not;
    the result is exact either way."""
    import torch

    n = 700
    rng = gg.rng_for(gg.CFG_TEST, 1500)
    W = rng.integers(1, 1 << 13, size=(n, n), dtype=np.int64)
    W[rng.random((n, n)) > 4.0 / n] = INF
    W = W.astype(np.int32)
    assert 2 * (n - 1) * int(W[W < INF].max()) < (1 << 24)
    view, _ = _to_dev(W, dev)
    q = apsp.num_rounds(n)
    for r0 in range(q):
        apsp.solve_rounds(view, r0, r0 + 1)
        torch.cuda.synchronize()
        part = view.cpu().numpy()
        if r0 + 1 < q:
            ref = np.minimum(oracle.fw_steps(oracle.prepare(W), 0, (r0 + 1) * apsp.round_width(n),
                                              threads=4),
                             INF)
            assert np.array_equal(part.astype(np.int64), ref), r0
    fin = part[part < INF]
    print(f"final largest length {fin.max()}, bound {2 * (n - 1) * int(fin.max())} vs 2^24")
    assert np.array_equal(part.astype(np.int64), oracle.fw(W, threads=4))


@pytest.mark.parametrize("pairs", [False, True])
@pytest.mark.parametrize("whi", [100, 1 << 20])
def test_banded_ragged_int32_rows(apsp, dev, whi, pairs):
    """n = 8300: 65 rounds, so phase 3 runs as two bands of block rows, in
    single rounds or (threshold lowered) in round pairs ending with a round
    alone, and the last block is partial (8300 = 64 * 128 + 108).  U{1..100}
    takes the fp32 pipe, U{1..2^20} uint32.  Sampled rows and columns (the
    last vertex among them) equal the oracle's Dijkstra exactly, and the
    exact Bellman certificate holds on a larger sample of rows."""
    prev = apsp.set_round_pair_threshold(8 if pairs else 1000)
    try:
        _banded_ragged(apsp, dev, whi)
    finally:
        apsp.set_round_pair_threshold(prev)


@pytest.mark.parametrize("whi", [100, 1 << 20])
def test_full_size_ragged_int32(apsp, dev, whi):
    """n = 16461 = 128 * 128 + 77, int32, at the default pair threshold: 129
    rounds, i.e. 64 round pairs then the last (partial) round alone, phase 3
    in two bands; U{1..100} takes the fp32 pipe, U{1..2^20} uint32.  Same
    checks as at n = 8300."""
    _banded_ragged(apsp, dev, whi, n=16461, rounds=129)


def _banded_ragged(apsp, dev, whi, n=8300, rounds=65):
    import torch

    rng = gg.rng_for(gg.CFG_TEST, 1600 + whi + (n != 8300) * n)
    u, v, w = gg.er_edges(n, 6.0 / n, 1, whi, rng)
    D = gg.device_dense_from_edges(n, u, v, w, np.int32, dev)
    assert apsp.num_rounds(n) == rounds
    apsp.solve(D)
    torch.cuda.synchronize()
    csr = gg.csr_from_edges(n, u, v, w)
    src = np.unique(np.concatenate([rng.choice(n, size=23, replace=False), [n - 1]]))
    ref = oracle.dijkstra(csr, n, src, threads=16, integer=True)
    tsrc = torch.as_tensor(src, device=dev)
    assert np.array_equal(D[tsrc].cpu().numpy().astype(np.int64), ref)
    assert np.array_equal(D[:, tsrc].cpu().numpy().T.astype(np.int64), ref)
    brows = rng.choice(n, size=1500, replace=False)
    assert oracle.bellman_violations_i32(D.cpu().numpy(), csr, brows, threads=16) == 0


# ------------------------------------------------------------ round pairs
# From 72 rounds on (by default), phase 3 runs in pairs of rounds, with round
# r+1's update of the pair's first block row/column deferred.  The threshold
# is lowered to 8 rounds here so small matrices take that schedule.  These
# cases cross every boundary of it: odd and even round counts, calls that
# stop after either round of a pair or resume in the middle of one, and the
# next pair's blocks being absent or half present.  fp32 results must equal
# the blocked model bit for bit.

@pytest.fixture
def width128(apsp):
    """Every n in rounds of 128 (round pairs exist only at that width)."""
    prev = apsp.set_width64_max_n(0)
    yield
    apsp.set_width64_max_n(prev)


@pytest.fixture
def pairs_from_8(apsp, width128):
    prev = apsp.set_round_pair_threshold(8)
    yield
    apsp.set_round_pair_threshold(prev)


@pytest.mark.parametrize("n", [1024, 1100, 1300, 2100])
def test_pair_schedule_fp32_bitexact(apsp, dev, pairs_from_8, n):
    """q = 8, 9, 11, 17 rounds: the whole solve equals the blocked model."""
    W, _ = _swiss(n, 40 + n)
    assert apsp.num_rounds(n) >= 8
    assert np.array_equal(_solve(apsp, W, dev), oracle.blocked(W, 128))


@pytest.mark.parametrize("r0,r1", [(0, 3), (0, 4), (0, 7), (1, 6), (3, 10), (5, 12), (2, 11),
                                   (10, 12), (4, 12)])
def test_pair_schedule_slices_fp32(apsp, dev, pairs_from_8, r0, r1):
    """n = 1500 (12 rounds): rounds r0..r1-1, started from the blocked model's
    state after r0 rounds, leave the model's state after r1 rounds."""
    import torch

    n = 1500
    W, _ = _swiss(n, 60)
    start = W if r0 == 0 else oracle.blocked(W, 128, 0, r0)
    view, _ = _to_dev(start, dev)
    apsp.solve_rounds(view, r0, r1)
    torch.cuda.synchronize()
    assert np.array_equal(view.cpu().numpy(), oracle.blocked(start, 128, r0, r1))


@pytest.mark.parametrize("whi", [100, 1 << 20])
def test_pair_schedule_int32(apsp, dev, pairs_from_8, whi):
    """int32, n = 1200 (10 rounds), on either pipe: a solve split after
    rounds 3 and 8 passes through Floyd-Warshall's states after 3*128 and
    8*128 pivots and ends at the oracle's result."""
    import torch

    n = 1200
    W, _ = _er(n, 5.0 / n, 70 + whi, 1, whi)
    view, _ = _to_dev(W, dev)
    for r0, r1 in ((0, 3), (3, 8), (8, 10)):
        apsp.solve_rounds(view, r0, r1)
        torch.cuda.synchronize()
        ref = oracle.fw_steps(oracle.prepare(W), 0, min(r1 * 128, n), threads=8)
        assert np.array_equal(view.cpu().numpy().astype(np.int64), np.minimum(ref, INF)), r1


@pytest.mark.parametrize("ld_extra,offset", [(3, 1), (212, 0)])
def test_pair_schedule_layout(apsp, dev, pairs_from_8, ld_extra, offset):
    """Round pairs on a padded or misaligned matrix (ld = n + 3 with a 4-byte
    offset: the unaligned load path; ld = n + 212): the result equals the
    oracle (int32) and the blocked model (fp32), and nothing outside the
    n x n view is written."""
    import torch

    n = 1100
    Wi, _ = _er(n, 5.0 / n, 90)
    Wf, _ = _swiss(n, 91)
    for W in (Wi, Wf):
        view, buf = _to_dev(W, dev, ld=n + ld_extra, offset=offset)
        before = buf.clone()
        apsp.solve(view)
        torch.cuda.synchronize()
        got = view.cpu().numpy()
        if W.dtype == np.int32:
            assert np.array_equal(got.astype(np.int64), oracle.fw(W, threads=8))
        else:
            assert np.array_equal(got, oracle.blocked(W, 128))
        mask = torch.ones_like(buf, dtype=torch.bool)
        mask[offset:offset + n * (n + ld_extra)].view(n, n + ld_extra)[:, :n] = False
        assert torch.equal(buf[mask], before[mask])


def test_pair_schedule_random_slices(apsp, dev, pairs_from_8):
    """Eight seeded cases: n in [900, 2600), int32 or fp32, the solve cut into
    slices at random rounds; equal to the oracle (int32) and the blocked model
    (fp32)."""
    import torch

    rng = np.random.default_rng(2024)
    for case in range(8):
        n = int(rng.integers(900, 2600))
        q = apsp.num_rounds(n)
        if case % 2:
            W, _ = _swiss(n, 500 + case)
        else:
            W, _ = _er(n, 5.0 / n, 500 + case, 1, int(rng.choice([100, 1 << 20])))
        cuts = sorted({0, q, *(int(x) for x in rng.integers(1, q, size=int(rng.integers(0, 3))))})
        view, _ = _to_dev(W, dev)
        for a, b in zip(cuts[:-1], cuts[1:]):
            apsp.solve_rounds(view, a, b)
        torch.cuda.synchronize()
        got = view.cpu().numpy()
        if W.dtype == np.int32:
            assert np.array_equal(got.astype(np.int64), oracle.fw(W, threads=8)), (n, cuts)
        else:
            assert np.array_equal(got, oracle.blocked(W, 128)), (n, cuts)


@pytest.mark.parametrize("n", [129, 256, 300, 384])
def test_pair_threshold_two_small_matrices(apsp, dev, width128, n):
    """Threshold 2 on matrices of 2 and 3 rounds, int32 and fp32, in one call
    and in calls of two rounds.  Pairs need the helper streams, which fp32
    matrices of 2 rounds do not get: those run single rounds (a pair would
    have no rest set), 3 rounds run a pair and the last round alone.
    Results equal the oracle (int32) and the blocked model (fp32)."""
    import torch

    prev = apsp.set_round_pair_threshold(2)
    try:
        for W in (_er(n, 8.0 / n, 700 + n)[0], _swiss(n, 700 + n)[0]):
            want = (oracle.fw(W, threads=4) if W.dtype == np.int32 else oracle.blocked(W, 128))
            q = apsp.num_rounds(n)
            for cuts in ([0, q], sorted({0, min(2, q), q})):
                view, _ = _to_dev(W, dev)
                for a, b in zip(cuts[:-1], cuts[1:]):
                    apsp.solve_rounds(view, a, b)
                torch.cuda.synchronize()
                got = view.cpu().numpy()
                if W.dtype == np.int32:
                    assert np.array_equal(got.astype(np.int64), want), (n, cuts)
                else:
                    assert np.array_equal(got, want), (n, cuts)
    finally:
        apsp.set_round_pair_threshold(prev)


@pytest.mark.parametrize("shared_stream", [True, False])
def test_host_threads(apsp, dev, pairs_from_8, shared_stream):
    """Six host threads solve at once (round pairs, 7 to 17 rounds), all on one
    stream (the library serialises them on its helper for that stream and
    grows the panel copies between them) or each on a stream of its own
    (separate helpers).  Every result equals the same solve run alone."""
    import threading

    import torch

    sizes = [1100, 2100, 1300, 900, 2100, 1100]
    mats = [(_swiss(n, 900 + i)[0] if i % 2 else _er(n, 6.0 / n, 900 + i, 1, 1 << 20)[0])
            for i, n in enumerate(sizes)]
    want = [_solve(apsp, W, dev) for W in mats]
    shared = torch.cuda.Stream()
    got = [None] * len(mats)
    errors = []

    def work(i):
        try:
            st = shared if shared_stream else torch.cuda.Stream()
            with torch.cuda.stream(st):
                view, _ = _to_dev(mats[i], dev)
                apsp.solve(view)
                out = view.cpu()  # stream-ordered after the solve
            got[i] = out.numpy()
        except Exception as e:  # surfaced below
            errors.append(e)

    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(mats))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for i, W in enumerate(mats):
        assert np.array_equal(got[i], want[i]), (i, sizes[i])


def test_pair_schedule_profiled(apsp, dev, pairs_from_8):
    """The profiled solve runs the same schedule (one rest launch group per
    pair of rounds) and gives the same result as single rounds."""
    n = 1200
    W, _ = _swiss(n, 75)
    a = _solve(apsp, W, dev)
    view, _ = _to_dev(W, dev)
    t = apsp.solve_profiled(view)
    assert np.array_equal(view.cpu().numpy(), a)
    assert t["phase3_rest_launches"] == apsp.num_rounds(n) // 2
    assert t["phase3_rest"] > 0 and t["total"] > 0
    prev = apsp.set_round_pair_threshold(1000)  # single rounds
    try:
        assert np.array_equal(_solve(apsp, W, dev), a)
    finally:
        apsp.set_round_pair_threshold(prev)


# --------------------------------------------------- width-64 rounds (small n)

@pytest.mark.parametrize("n", [65, 129, 200, 257, 640, 1000, 1024])
def test_width64_rounds(apsp, dev, n):
    """Small matrices run rounds of width 64 (with the one-round lookahead from
    3 rounds on): int32 equals the oracle and fp32 the blocked model at width
    64 bit for bit (and fp64 Floyd-Warshall within 1e-5); an int32 solve cut
    into slices passes through Floyd-Warshall's state after 64 r pivots."""
    import torch

    assert apsp.round_width(n) == 64
    Wi, _ = _er(n, min(1.0, 4.0 / n), 3100 + n, 1, 1000)
    Wf, _ = _swiss(n, 3200 + n)
    assert np.array_equal(_solve(apsp, Wi, dev).astype(np.int64), oracle.fw(Wi, threads=8))
    got = _solve(apsp, Wf, dev)
    assert np.array_equal(got, oracle.blocked(Wf, 64))
    _assert_f32_close(got, oracle.fw(Wf, threads=8))
    q = apsp.num_rounds(n)
    assert q == -(-n // 64)
    cuts = sorted({0, 1, q // 2, q - 1, q})
    view, _ = _to_dev(Wi, dev, ld=n + 5)
    for a, b in zip(cuts[:-1], cuts[1:]):
        apsp.solve_rounds(view, a, b)
        torch.cuda.synchronize()
        ref = oracle.fw_steps(oracle.prepare(Wi), 0, min(b * 64, n), threads=8)
        assert np.array_equal(view.cpu().numpy().astype(np.int64), np.minimum(ref, INF)), b


def test_width64_bands(apsp, dev):
    """With the limit raised to 4096, n = 4050 takes 64 rounds of 64: the rest
    of phase 3 then runs in two bands of block rows.  int32 (both pipes)
    equals the oracle; fp32 matches fp64 Dijkstra on sampled rows."""
    import torch

    n = 4050
    prev = apsp.set_width64_max_n(4096)
    try:
        assert apsp.num_rounds(n) == 64
        for whi in (100, 1 << 20):
            Wi, _ = _er(n, 6.0 / n, 3300 + whi, 1, whi)
            assert np.array_equal(_solve(apsp, Wi, dev).astype(np.int64),
                                  oracle.fw(Wi, threads=16)), whi
        Wf, (u, v, w) = _swiss(n, 3400)
        view, _ = _to_dev(Wf, dev)
        t = apsp.solve_profiled(view)
        assert t["phase3_rest_launches"] == 63
        got = view.cpu().numpy()
        rows = gg.rng_for(gg.CFG_TEST, 3401).choice(n, size=24, replace=False)
        csr = oracle.csr_from_dense(Wf)
        ref = oracle.dijkstra(csr, n, rows, threads=8)
        _assert_f32_close(got[rows], ref)
    finally:
        apsp.set_width64_max_n(prev)


# --------------------------------------------------------------- batched

def _batched_case_sizes():
    return [1, 2, 31, 63, 64, 65, 127, 128, 129, 200, 333, 512]


def test_batched_int32_small_cases(apsp, dev):
    import torch

    Ws = [_er(n, min(1.0, 8.0 / n), 500 + n, 1, 1000)[0] for n in _batched_case_sizes()]
    views = [_to_dev(W, dev)[0] for W in Ws]
    apsp.solve_batched(views)
    torch.cuda.synchronize()
    for W, v in zip(Ws, views):
        assert np.array_equal(v.cpu().numpy().astype(np.int64), oracle.fw(W)), W.shape


def test_batched_fp32_with_ld(apsp, dev):
    import torch

    Ws = [_swiss(n, 600 + n)[0] if n > 11 else np.zeros((n, n), np.float32)
          for n in _batched_case_sizes()]
    views = [_to_dev(W, dev, ld=W.shape[0] + 3)[0] for W in Ws]
    apsp.solve_batched(views)
    torch.cuda.synchronize()
    for W, v in zip(Ws, views):
        n = W.shape[0]
        got = v.cpu().numpy()
        assert np.array_equal(got, oracle.blocked(W, apsp.batched_round_width(n, apsp.APSP_F32)))
        _assert_f32_close(got, oracle.fw(W))


def test_batched_config_4096_graphs(apsp, dev):
    """4096 ER graphs, n log-uniform in [32, 512], p = 8/n, int32 U{1..1000}."""
    import torch

    Ws = gg.batched_graphs(4096, item=0)
    views = [torch.from_numpy(W).to(dev) for W in Ws]
    apsp.solve_batched(views)
    # the same graphs one by one through the single-graph path
    singles = [torch.from_numpy(W).to(dev) for W in Ws]
    for s in singles:
        apsp.solve(s)
    torch.cuda.synchronize()
    for v, s in zip(views, singles):
        assert torch.equal(v, s)
    sample = gg.rng_for(gg.CFG_TEST, 4096).choice(len(Ws), size=96, replace=False)
    for g in sample:
        assert np.array_equal(views[g].cpu().numpy().astype(np.int64), oracle.fw(Ws[g])), g


def test_batched_plan_reuse(apsp, dev):
    """A plan is built once and run repeatedly on fresh inputs at the same pointers."""
    import torch

    sizes = [1, 40, 128, 129, 300, 512]
    Ws = [_er(n, min(1.0, 8.0 / n), 700 + n, 1, 1000)[0] for n in sizes]
    mats = [torch.from_numpy(W).to(dev) for W in Ws]
    plan = apsp.BatchPlan(mats)
    info = plan.info()
    # launches: phase 1 of round 0, then phases 2 and 3 of each of the 4 rounds
    assert info["launches"] == 1 + 2 * 4
    for rep in range(2):
        for m, W in zip(mats, Ws):
            m.copy_(torch.from_numpy(W).to(dev))
        plan.run()
        torch.cuda.synchronize()
        for m, W in zip(mats, Ws):
            assert np.array_equal(m.cpu().numpy().astype(np.int64), oracle.fw(W)), (rep, W.shape)
    plan.close()


@pytest.fixture
def default_tuning(apsp):
    """Leave the device's batched tuning table as every other test expects it."""
    apsp.set_batched_tuning([128] * apsp.TUNE_BUCKETS)
    yield
    apsp.set_batched_tuning([128] * apsp.TUNE_BUCKETS)


def _directed_int(n, seed):
    """Directed ER graph with a nonzero diagonal and some 'no edge' entries above 2^30."""
    rng = gg.rng_for(gg.CFG_TEST, seed)
    W = rng.integers(1, 1000, size=(n, n)).astype(np.int32)
    W[rng.random((n, n)) > min(1.0, 6.0 / max(n, 1))] = INF + 5
    np.fill_diagonal(W, rng.integers(1, 50, size=n).astype(np.int32))
    return W


@pytest.mark.parametrize("tile", [64, 128])
def test_batched_forced_width_int32_exact(apsp, dev, tile):
    import torch

    sizes = _batched_case_sizes() + [1000]
    Ws = [_directed_int(n, 800 + n) for n in sizes]
    mats = [_to_dev(W, dev, ld=W.shape[0] + (n % 3))[0] for W, n in zip(Ws, sizes)]
    plan = apsp.BatchPlan(mats, tile=tile)
    # launches: phase 1 of round 0, then phases 2 and 3 of every round of the largest graph
    assert plan.info()["launches"] == 1 + 2 * (-(-1000 // tile))
    plan.run()
    torch.cuda.synchronize()
    for W, m in zip(Ws, mats):
        assert np.array_equal(m.cpu().numpy().astype(np.int64), oracle.fw(W)), W.shape
    plan.close()


def _weighted_int(n, seed, wlo, whi, p=None, diag=0):
    rng = gg.rng_for(gg.CFG_TEST, seed)
    W = rng.integers(wlo, whi + 1, size=(n, n), dtype=np.int64)
    W[rng.random((n, n)) > (p if p is not None else min(1.0, 6.0 / max(n, 1)))] = INF
    np.fill_diagonal(W, diag)
    return W.astype(np.int32)


@pytest.mark.parametrize("tile", [64, 128])
def test_batched_int32_fp32_pipe_boundary(apsp, dev, tile):
    """int32 graphs run on the fp32 pipe only when 2 (n-1) wmax < 2^24; results
    are exact on both sides of that bound, with saturation at 2^30."""
    import torch

    cases = [
        (65, 131071, 0),            # 2*64*131071 = 2^24 - 128: fp32 pipe
        (65, 131072, 0),            # 2*64*131072 = 2^24: uint32
        (300, 1 << 21, 0),          # far above the bound: uint32
        (200, 1000, 1 << 29),       # huge diagonal entries are not weights
        (150, 1 << 29, 0),          # sums reach 2^30: saturate to "no edge"
        (129, 1, 0),                # unit weights
        (2, (1 << 30) - 1, 0),      # largest finite weight
    ]
    Ws = [_weighted_int(n, 1000 + i, max(1, whi // 2), whi, diag=d)
          for i, (n, whi, d) in enumerate(cases)]
    mats = [_to_dev(W, dev)[0] for W in Ws]
    plan = apsp.BatchPlan(mats, tile=tile)
    plan.run()
    torch.cuda.synchronize()
    for (n, whi, _), W, m in zip(cases, Ws, mats):
        assert np.array_equal(m.cpu().numpy().astype(np.int64), oracle.fw(W)), (n, whi)
    plan.close()


def test_batched_width64_fp32_bitexact(apsp, dev):
    import torch

    Ws = [_swiss(n, 900 + n)[0] if n > 11 else np.zeros((n, n), np.float32)
          for n in _batched_case_sizes()]
    mats = [_to_dev(W, dev, ld=W.shape[0] + 1)[0] for W in Ws]  # unaligned rows
    plan = apsp.BatchPlan(mats, tile=64)
    plan.run()
    torch.cuda.synchronize()
    for W, m in zip(Ws, mats):
        got = m.cpu().numpy()
        assert np.array_equal(got, oracle.blocked(W, 64)), W.shape
        _assert_f32_close(got, oracle.fw(W))
    plan.close()


def test_batched_mixed_width_table(apsp, dev, default_tuning):
    """Graphs of one batch split over both widths by the tuning table."""
    import torch

    table = [64, 128, 64, 128, 64, 128, 64, 128, 64]
    apsp.set_batched_tuning(table)
    assert apsp.batched_tuning() == table
    sizes = [1, 50, 64, 65, 100, 128, 129, 190, 256, 300, 400, 450, 512, 513, 700]
    for n in sizes:
        b = 0 if n <= 64 else (min(n, 513) - 1) // 64 if n <= 512 else 8
        assert apsp.batched_round_width(n, apsp.APSP_F32) == table[b], n
    Ws = [_swiss(n, 950 + n)[0] if n > 11 else np.zeros((n, n), np.float32) for n in sizes]
    views = [_to_dev(W, dev)[0] for W in Ws]
    apsp.solve_batched(views)  # one-shot plan
    Wi = [_directed_int(n, 960 + n) for n in sizes]
    vi = [_to_dev(W, dev)[0] for W in Wi]
    apsp.solve_batched(vi)
    torch.cuda.synchronize()
    for W, v, n in zip(Ws, views, sizes):
        assert np.array_equal(v.cpu().numpy(),
                              oracle.blocked(W, apsp.batched_round_width(n, apsp.APSP_F32))), n
    for W, v in zip(Wi, vi):
        assert np.array_equal(v.cpu().numpy().astype(np.int64), oracle.fw(W)), W.shape


def test_batched_autotune(apsp, dev, default_tuning):
    import torch

    res = apsp.batched_autotune(apsp.APSP_I32, batch_elems=1 << 22)
    print(f"autotune widths {res['widths']} ms {res['ms']}")
    assert len(res["widths"]) == apsp.TUNE_BUCKETS
    assert all(w in (64, 128) for w in res["widths"])
    assert all(a > 0 and b > 0 for a, b in res["ms"])
    assert apsp.batched_tuning() == res["widths"]
    # the tuned table is what plans now use, and results stay exact
    Ws = gg.batched_graphs(64, item=3)
    views = [torch.from_numpy(W).to(dev) for W in Ws]
    apsp.solve_batched(views)
    torch.cuda.synchronize()
    for W, v in zip(Ws, views):
        assert np.array_equal(v.cpu().numpy().astype(np.int64), oracle.fw(W)), W.shape


@pytest.mark.parametrize("dtype", [np.int32, np.float32])
def test_batched_plan_in_hip_graph(apsp, dev, dtype):
    """A plan's run() only launches kernels, so it can be captured in a HIP
    graph; every replay (with eager resets between them) gives the eager result."""
    import torch

    sizes = [40, 64, 130, 257, 300]
    if dtype == np.int32:
        Ws = [_directed_int(n, 1200 + n) for n in sizes]
    else:
        Ws = [_swiss(n, 1300 + n)[0] for n in sizes]
    pristine = [torch.from_numpy(W).to(dev) for W in Ws]
    mats = [p.clone() for p in pristine]
    plan = apsp.BatchPlan(mats)
    plan.run()
    torch.cuda.synchronize()
    expect = [m.clone() for m in mats]
    for W, e in zip(Ws, expect):
        ref = oracle.fw(W) if dtype == np.int32 else oracle.blocked(W, apsp.batched_round_width(W.shape[0], 1))
        assert np.array_equal(e.cpu().numpy().astype(ref.dtype), ref)
    for m, p in zip(mats, pristine):
        m.copy_(p)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.run()
    for rep in range(3):
        for m, p in zip(mats, pristine):
            m.copy_(p)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for m, e in zip(mats, expect):
            assert torch.equal(m, e), rep
    plan.close()


def test_batched_autotune_batch(apsp, dev, default_tuning):
    """The whole-batch tuner reads the batch only, and plans built after it
    use its table with exact results."""
    import torch

    Ws = gg.batched_graphs(256, item=5)
    views = [torch.from_numpy(W).to(dev) for W in Ws]
    before = [v.clone() for v in views]
    res = apsp.batched_autotune_batch(views)
    torch.cuda.synchronize()
    print(f"batch autotune {res}")
    assert all(torch.equal(a, b) for a, b in zip(before, views))
    assert all(w in (64, 128) for w in res["widths"])
    assert res["ms_all_128"] > 0 and 0 < res["ms_tuned"] <= res["ms_all_128"]
    assert apsp.batched_tuning() == res["widths"]
    apsp.solve_batched(views)
    torch.cuda.synchronize()
    for W, v in zip(Ws, views):
        assert np.array_equal(v.cpu().numpy().astype(np.int64), oracle.fw(W)), W.shape


# -------------------------------------------------- min-plus product, squaring

def _rand_operand(shape, dtype, seed, p_inf=0.3):
    rng = gg.rng_for(gg.CFG_TEST, seed)
    if dtype == np.int32:
        X = rng.integers(0, 1000, size=shape).astype(np.int32)
        X[rng.random(shape) < p_inf] = INF
    else:
        X = (rng.random(shape) * 10).astype(np.float32)
        X[rng.random(shape) < p_inf] = np.inf
    return X


@pytest.mark.parametrize("dtype", [np.int32, np.float32])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (5, 7, 3), (128, 128, 128), (130, 257, 200),
                                   (300, 100, 513), (64, 1000, 17)])
@pytest.mark.parametrize("accumulate", [False, True])
def test_minplus_product(apsp, dev, dtype, m, n, k, accumulate):
    import torch

    A = _rand_operand((m, k), dtype, m * 7 + k)
    B = _rand_operand((k, n), dtype, n * 11 + k)
    C0 = _rand_operand((m, n), dtype, m + n)
    tA, tB = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
    # C with a padded leading dimension
    buf = torch.full((m, n + 5), 7, dtype=tA.dtype, device=dev)
    tC = buf[:, :n]
    tC.copy_(torch.from_numpy(C0).to(dev))
    apsp.minplus(tC, tA, tB, accumulate=accumulate)
    torch.cuda.synchronize()
    start = C0 if accumulate else np.full_like(C0, INF if dtype == np.int32 else np.inf)
    ref = oracle.minplus_acc(start, A, B)
    assert np.array_equal(tC.cpu().numpy(), ref)
    assert (buf[:, n:] == 7).all()


@pytest.mark.parametrize("n", [2, 3, 100, 300])
def test_repeated_squaring(apsp, dev, n):
    import torch

    Wi, _ = _er(n, min(1.0, 3.0 / n), 9000 + n)
    Wf, _ = _swiss(n, 9100 + n) if n > 11 else (np.zeros((n, n), np.float32), None)
    for W in (Wi, Wf):
        D = torch.from_numpy(W).to(dev)
        work = torch.empty_like(D)
        apsp.solve_squaring(D, work)
        torch.cuda.synchronize()
        got = D.cpu().numpy()
        assert np.array_equal(got, oracle.squaring(W)), (n, W.dtype)
        if W.dtype == np.int32:
            assert np.array_equal(got.astype(np.int64), oracle.fw(W))


def test_minplus_rejects_overlap(apsp, dev):
    import torch

    A = torch.zeros((64, 64), dtype=torch.float32, device=dev)
    with pytest.raises(apsp.ApspError):
        apsp.minplus(A, A, A)


# ------------------------------------------------------------ symmetric variant

@pytest.mark.parametrize("n", [1, 2, 100, 129, 300, 700, 1000])
def test_symmetric_variant_vs_oracle(apsp, dev, n):
    """Upper-triangle solve of an undirected graph (Sec. 4 storage) against the
    oracle: int32 equals Floyd-Warshall exactly; fp32 equals the oracle's
    blocked fp32 model at width 128 bit for bit and lies within 1e-5 of fp64
    Floyd-Warshall.  The input's lower triangle holds junk and its diagonal
    nonzero values: the variant must read neither."""
    import torch

    Wi, _ = _er(n, min(1.0, 4.0 / n), 9500 + n)
    Wf, _ = _swiss(n, 9600 + n) if n > 11 else (np.zeros((n, n), np.float32), None)
    for W in (Wi, Wf):
        junk = W.copy()
        low = np.tril_indices(n, -1)
        if W.dtype == np.int32:
            junk[low] = 3
            np.fill_diagonal(junk, 7)
        else:
            junk[low] = np.float32(0.125)
            np.fill_diagonal(junk, np.float32(2.5e3))
        view, buf = _to_dev(junk, dev, ld=n + 4)
        before = buf.clone()
        apsp.solve_symmetric(view)
        torch.cuda.synchronize()
        got = view.cpu().numpy()
        if W.dtype == np.int32:
            assert np.array_equal(got.astype(np.int64), oracle.fw(W)), n
        else:
            assert np.array_equal(got, oracle.blocked(W, 128)), n
            _assert_f32_close(got, oracle.fw(W))
        # nothing outside the n x n view was written
        mask = torch.ones_like(buf, dtype=torch.bool)
        mask[:n * (n + 4)].view(n, n + 4)[:, :n] = False
        assert torch.equal(buf[mask], before[mask])


@pytest.mark.parametrize("n,pad", [(256, 0), (384, 0), (384, 4), (384, 1), (1024, 0), (1280, 0)])
def test_symmetric_variant_direct_and_lookahead_vs_oracle(apsp, dev, n, pad):
    """Sizes that are multiples of 128 take the direct-staged phase 3 (with
    16-byte aligned rows: pad 0 or 4; pad 1 takes the register-staged one),
    and from 3 rounds on the rest set runs on the helper stream one round
    ahead.  int32 equals Floyd-Warshall, fp32 the oracle's blocked model at
    width 128, bit for bit."""
    import torch

    Wi, _ = _er(n, min(1.0, 4.0 / n), 9800 + n)
    Wf, _ = _swiss(n, 9900 + n)
    for W in (Wi, Wf):
        view, _ = _to_dev(W, dev, ld=n + pad)
        apsp.solve_symmetric(view)
        torch.cuda.synchronize()
        got = view.cpu().numpy()
        if W.dtype == np.int32:
            assert np.array_equal(got.astype(np.int64), oracle.fw(W, threads=8)), n
        else:
            assert np.array_equal(got, oracle.blocked(W, 128)), n


@pytest.mark.parametrize("n", [384, 1024, 2048])
def test_single_rounds_direct_rest_vs_oracle(apsp, dev, n):
    """fp32, rounds of 128 below the pair threshold, n % 128 == 0 and aligned
    rows: phase 2 writes the transposed column copy and the rest set and the
    next-row/column set read it (direct staging).  Whole solves, and a solve
    split into slices (a slice that stops after round r does not fuse block
    r+1's closure), equal the oracle's blocked model at width 128 bit for bit;
    unaligned rows (register-staged) too."""
    import torch

    W, _ = _swiss(n, 9300 + n)
    ref = oracle.blocked(W, 128)
    prev = apsp.set_width64_max_n(0)
    try:
        q = apsp.num_rounds(n)
        for pad in (0, 1):
            view, _ = _to_dev(W, dev, ld=n + pad)
            apsp.solve(view)
            torch.cuda.synchronize()
            assert np.array_equal(view.cpu().numpy(), ref), (n, pad)
        view, _ = _to_dev(W, dev)
        cuts = sorted({0, 1, q // 2, q - 1, q})
        for a, b in zip(cuts[:-1], cuts[1:]):
            apsp.solve_rounds(view, a, b)
        torch.cuda.synchronize()
        assert np.array_equal(view.cpu().numpy(), ref), (n, "slices")
    finally:
        apsp.set_width64_max_n(prev)


def test_symmetric_variant_equals_full_solve_large(apsp, dev):
    """n = 4096 (32 rounds, direct staging, lookahead): the upper-triangle
    solve gives the full solve's bits at width 128 (checked against the
    oracle at the sizes above)."""
    import torch

    n = 4096
    Wf, _ = _swiss(n, 9990)
    a, _ = _to_dev(Wf, dev)
    b, _ = _to_dev(Wf, dev)
    prev = apsp.set_width64_max_n(0)
    try:
        apsp.solve(a)
        apsp.solve_symmetric(b)
        torch.cuda.synchronize()
    finally:
        apsp.set_width64_max_n(prev)
    assert torch.equal(a, b)


# ------------------------------------------------- fp32 input with a diagonal

def _f32_with_diagonal(n, seed):
    """Swiss-roll kNN matrix whose diagonal holds nonzero weights, some huge
    (3e38) and some +inf: the empty path must still give D_ii = 0."""
    W, _ = _swiss(n, seed) if n > 11 else (np.zeros((n, n), np.float32), None)
    rng = gg.rng_for(gg.CFG_TEST, seed + 1)
    d = (rng.random(n) * 5 + 0.5).astype(np.float32)
    d[::3] = np.float32(3e38)
    d[1::3] = np.inf
    W = W.copy()
    np.fill_diagonal(W, d)
    return W


@pytest.mark.parametrize("n", [1, 2, 129, 300, 513])
def test_fp32_nonzero_diagonal(apsp, dev, n):
    """fp32 inputs with a nonzero diagonal through every fp32 entry point, each
    against the oracle (which takes the diagonal as the empty path)."""
    import torch

    W = _f32_with_diagonal(n, 9700 + n)
    ref = oracle.blocked(W, apsp.round_width(n))
    ref128 = oracle.blocked(W, 128)
    ref64 = oracle.fw(W)
    assert (np.diag(ref) == 0).all()
    # apsp_solve
    got = _solve(apsp, W, dev)
    assert np.array_equal(got, ref), "apsp_solve"
    _assert_f32_close(got, ref64)
    # apsp_solve_rounds from round 0, in two slices
    q = apsp.num_rounds(n)
    view, _ = _to_dev(W, dev)
    apsp.solve_rounds(view, 0, 1)
    apsp.solve_rounds(view, 1, q)
    torch.cuda.synchronize()
    assert np.array_equal(view.cpu().numpy(), ref), "apsp_solve_rounds"
    # apsp_solve_symmetric (W is symmetric off the diagonal)
    view, _ = _to_dev(W, dev, ld=n + 2)
    apsp.solve_symmetric(view)
    torch.cuda.synchronize()
    assert np.array_equal(view.cpu().numpy(), ref128), "apsp_solve_symmetric"
    # batched, one-shot call and both forced widths
    views = [_to_dev(W, dev)[0] for _ in range(3)]
    apsp.solve_batched([views[0]])
    plans = [apsp.BatchPlan([views[1]], tile=64), apsp.BatchPlan([views[2]], tile=128)]
    for p in plans:
        p.run()
    torch.cuda.synchronize()
    assert np.array_equal(views[0].cpu().numpy(),
                          oracle.blocked(W, apsp.batched_round_width(n, apsp.APSP_F32)))
    assert np.array_equal(views[1].cpu().numpy(), oracle.blocked(W, 64)), "batched width 64"
    assert np.array_equal(views[2].cpu().numpy(), ref128), "batched width 128"
    for p in plans:
        p.close()


# ------------------------------------------- rows that are not 16-byte aligned

@pytest.fixture
def aligned_copy_threshold(apsp):
    prev = apsp.set_aligned_copy_min_n(256)
    yield apsp
    apsp.set_aligned_copy_min_n(prev)


def _solve_with_copy(apsp, W, dev, copy, fn=None, **kw):
    import torch

    prev = apsp.set_aligned_copy_min_n(256 if copy else 1 << 40)
    try:
        view, buf = _to_dev(W, dev, **kw)
        (fn or apsp.solve)(view)
        torch.cuda.synchronize()
        return view.cpu().numpy(), buf
    finally:
        apsp.set_aligned_copy_min_n(prev)


@pytest.mark.parametrize("n,dtype", [(300, np.int32), (1001, np.float32), (2047, np.int32),
                                     (6001, np.float32), (9219, np.float32)])
def test_aligned_working_copy(aligned_copy_threshold, dev, n, dtype):
    """A matrix whose rows are off 16 bytes (ld = n with n % 4 != 0, or a base
    4 bytes off) is solved in an aligned working copy: the result equals the
    in-place solve on the word-by-word path bit for bit, the padding around
    the matrix is untouched, and (small n) the result equals the oracle.
    9219 vertices take round pairs, 6001 single rounds of 128, 2047 and below
    rounds of 64."""
    import torch

    apsp = aligned_copy_threshold
    W = _er(n, 8.0 / n, 9800 + n)[0] if dtype == np.int32 else _swiss(n, 9800 + n)[0]
    ref, _ = _solve_with_copy(apsp, W, dev, copy=False)
    got, buf = _solve_with_copy(apsp, W, dev, copy=True)
    assert np.array_equal(got, ref)
    # base 4 bytes off 16, leading dimension a multiple of 4
    got_off, buf_off = _solve_with_copy(apsp, W, dev, copy=True, ld=n + (4 - n % 4) % 4 + 4,
                                        offset=1)
    assert np.array_equal(got_off, ref)
    ld = n + (4 - n % 4) % 4 + 4
    pad = buf_off[1:1 + n * ld].view(n, ld)[:, n:]
    assert (pad.cpu().numpy() == (-7 if dtype == np.int32 else -3.5)).all()
    if n <= 1001:
        exp = oracle.fw(W) if dtype == np.int32 else oracle.blocked(W, apsp.round_width(n))
        assert np.array_equal(got, exp)
    # round slices, each call through its own working copy
    q = apsp.num_rounds(n)
    view, _ = _to_dev(W, dev)
    cuts = [0, 1, q // 3, q]
    for r0, r1 in zip(cuts[:-1], cuts[1:]):
        apsp.solve_rounds(view, r0, r1)
    torch.cuda.synchronize()
    assert np.array_equal(view.cpu().numpy(), ref), "round slices"
    # profiled: synchronous, the same bits
    view, _ = _to_dev(W, dev)
    apsp.solve_profiled(view)
    assert np.array_equal(view.cpu().numpy(), ref), "profiled"


@pytest.mark.parametrize("n", [301, 1001])
def test_aligned_working_copy_symmetric(aligned_copy_threshold, dev, n):
    """The symmetric solver on rows off 16 bytes, through the working copy
    (junk in the lower triangle, which it overwrites), against the oracle."""
    apsp = aligned_copy_threshold
    W = _swiss(n, 9900 + n)[0]
    junk = W.copy()
    junk[np.tril_indices(n, -1)] = np.float32(7.0)
    got, _ = _solve_with_copy(apsp, junk, dev, copy=True, fn=apsp.solve_symmetric)
    assert np.array_equal(got, oracle.blocked(W, 128))


@pytest.mark.parametrize("n,dtype", [(8250, np.float32), (8300, np.int32), (9300, np.float32)])
def test_padded_working_copy(aligned_copy_threshold, dev, n, dtype):
    """Rounds of 128 with n not a multiple of 128 (64 or more rounds), rows
    aligned: a call of 16 or more rounds runs on a copy padded to a multiple
    of 128 with vertices that have no edges; the result equals the in-place
    solve bit for bit and the caller's padding columns are untouched.  Round
    slices mix padded calls (>= 16 rounds) and in-place ones.  8250 runs
    single rounds of 128, 9300 round pairs, 8300 (int32) the fp32 pipe."""
    import torch

    apsp = aligned_copy_threshold
    ld = n + (4 - n % 4) % 4 + 4
    W = _er(n, 8.0 / n, 9850 + n)[0] if dtype == np.int32 else _swiss(n, 9850 + n)[0]
    ref, _ = _solve_with_copy(apsp, W, dev, copy=False, ld=ld)
    got, buf = _solve_with_copy(apsp, W, dev, copy=True, ld=ld)
    assert np.array_equal(got, ref)
    pad = buf[:n * ld].view(n, ld)[:, n:]
    assert (pad.cpu().numpy() == (-7 if dtype == np.int32 else -3.5)).all()
    q = apsp.num_rounds(n)
    view, _ = _to_dev(W, dev, ld=ld)
    cuts = [0, 20, 27, q]  # 20 rounds padded, 7 in place, the rest padded
    for r0, r1 in zip(cuts[:-1], cuts[1:]):
        apsp.solve_rounds(view, r0, r1)
    torch.cuda.synchronize()
    assert np.array_equal(view.cpu().numpy(), ref), "round slices"
    if dtype == np.float32 and n == 8250:
        sym, _ = _solve_with_copy(apsp, W, dev, copy=True, fn=apsp.solve_symmetric, ld=ld)
        sym_ref, _ = _solve_with_copy(apsp, W, dev, copy=False, fn=apsp.solve_symmetric, ld=ld)
        assert np.array_equal(sym, sym_ref), "symmetric"


@pytest.mark.parametrize("dtype", [np.int32, np.float32])
def test_batched_working_copies(aligned_copy_threshold, dev, dtype):
    """Batched graphs whose rows are off 16 bytes (ld = n with n % 4 != 0, a
    base 4 bytes off) run on working copies: plan runs (twice), the one-shot
    call and the allocation-free call (which runs them in place) all equal the
    in-place plan bit for bit, and the int32 results equal the oracle."""
    import torch

    apsp = aligned_copy_threshold
    sizes = [40, 63, 130, 257, 301, 513, 64, 200]
    if dtype == np.int32:
        Ws = [_directed_int(n, 9950 + n) for n in sizes]
    else:
        Ws = [_swiss(n, 9950 + n)[0] for n in sizes]

    def fresh():
        out = []
        for k, W in enumerate(Ws):
            offset = 1 if k == 3 else 0
            ld = W.shape[0] + (4 if k == 3 else 0)
            out.append(_to_dev(W, dev, ld=ld, offset=offset)[0])
        return out

    prev = apsp.set_aligned_copy_min_n(1 << 40)  # copies off: everything in place
    try:
        ref = fresh()
        p = apsp.BatchPlan(ref)
        p.run()
        torch.cuda.synchronize()
        p.close()
    finally:
        apsp.set_aligned_copy_min_n(prev)
    ref = [r.cpu().numpy() for r in ref]
    if dtype == np.int32:
        for W, r in zip(Ws, ref):
            assert np.array_equal(r.astype(np.int64), oracle.fw(W)), W.shape
    mats = fresh()
    plan = apsp.BatchPlan(mats)
    for rep in range(2):
        for m, W in zip(mats, Ws):
            m.copy_(torch.from_numpy(W).to(dev))
        plan.run()
        torch.cuda.synchronize()
        for m, r in zip(mats, ref):
            assert np.array_equal(m.cpu().numpy(), r), rep
    plan.close()
    mats = fresh()
    apsp.solve_batched(mats)
    torch.cuda.synchronize()
    for m, r in zip(mats, ref):
        assert np.array_equal(m.cpu().numpy(), r), "one-shot"
    mats = fresh()
    apsp.solve_batched_noalloc(mats)
    torch.cuda.synchronize()
    for m, r in zip(mats, ref):
        assert np.array_equal(m.cpu().numpy(), r), "allocation-free"


@pytest.mark.parametrize("n,whi", [(8192, 100), (8192, 1 << 20), (9216, 100), (9216, 1 << 20)])
def test_int32_held_as_fp32(apsp, dev, n, whi):
    """int32 calls of 16 or more rounds on matrices of 64 or more rounds of
    128 hold the matrix as OpI32F's fp32 bits (when the weight scan allows
    the fp32 pipe) and run the direct-staged kernels; calls of fewer rounds
    run the int32 kernels on the integers.  A whole solve (one call) equals
    the same solve in slices of 8 rounds bit for bit, and sampled rows and
    columns equal integer Dijkstra.  8192 runs single rounds of 128, 9216
    round pairs; U{1..100} takes the fp32 pipe, U{1..2^20} uint32."""
    import torch

    rng = gg.rng_for(gg.CFG_TEST, 1700 + whi + n)
    u, v, w = gg.er_edges(n, 6.0 / n, 1, whi, rng)
    full = gg.device_dense_from_edges(n, u, v, w, np.int32, dev)
    sliced = full.clone()
    apsp.solve(full)
    q = apsp.num_rounds(n)
    for r0 in range(0, q, 8):
        apsp.solve_rounds(sliced, r0, r0 + 8)
    torch.cuda.synchronize()
    assert torch.equal(full, sliced)
    csr = gg.csr_from_edges(n, u, v, w)
    src = np.unique(np.concatenate([rng.choice(n, size=12, replace=False), [n - 1]]))
    ref = oracle.dijkstra(csr, n, src, threads=16, integer=True)
    tsrc = torch.as_tensor(src, device=dev)
    assert np.array_equal(full[tsrc].cpu().numpy().astype(np.int64), ref)
    assert np.array_equal(full[:, tsrc].cpu().numpy().T.astype(np.int64), ref)

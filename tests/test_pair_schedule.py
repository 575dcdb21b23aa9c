"""Host-side checks of the round-pair schedule of the single-graph solver.

Phase 3 of rounds r and r+1 runs as one pass over each tile, with round
r+1's update of block row/column r deferred (paper Sec. 4.4/4.5: the three
phases of Algorithms 3 and 4 on two consecutive rounds).  Two things are
checked here without a GPU:

* the workgroup -> tile maps of the pair launches, re-derived, are
  bijections onto the tile sets the schedule needs;
* a model of the schedule (the same launches, streams and event waits as the
  runtime) gives the blocked model's result bit for bit in fp32, whatever
  order the tiles of concurrently running launches take, each tile reading
  its operands before writing its result.
"""
import random

import numpy as np
import pytest

import oracle


# --------------------------------------------------------------------------
# Workgroup -> tile maps of the pair launches, re-derived.
# --------------------------------------------------------------------------

def _nxt(q, r):
    return max(0, min(2, q - (r + 2)))


def _next2_tile(t, r, q):
    nx, m = _nxt(q, r), q - 2
    if t < nx * m:
        c = t % m
        return r + 2 + t // m, (c if c < r else c + 2)
    t -= nx * m
    m2 = m - nx
    c = t % m2
    return (c if c < r else c + 2 + nx), r + 2 + t // m2


def _next2_count(r, q):
    nx, m = _nxt(q, r), q - 2
    return nx * m + nx * (m - nx)


def _rest2_count(r, q, lo, hi):
    e1 = r + 2 + _nxt(q, r)
    x0, x1 = max(r, lo), min(e1, hi)
    rows = hi - lo - max(0, x1 - x0)
    return max(rows, 0) * (q - (e1 - r))


def _rest2_tile(wg, r, q, lo, hi):
    e1 = r + 2 + _nxt(q, r)
    ex = e1 - r
    x0, x1 = max(r, lo), min(e1, hi)
    skipped = max(0, x1 - x0)
    rows = hi - lo - skipped
    mc = q - ex
    T = rows * mc
    x, s = wg & 7, wg >> 3
    per, rem = T >> 3, T & 7
    tl = x * per + min(x, rem) + s
    ti, tj = divmod(tl, mc)
    i = lo + ti
    if skipped and i >= x0:
        i += skipped
    return i, (tj if tj < r else tj + ex)


def _fix_tiles(r, q, final):
    nx = _nxt(q, r)
    if not final:
        out = []
        for t in range(2 * nx):
            x = r + 2 + (t >> 1)
            out.append((r, x) if t & 1 else (x, r))
        return out
    rowpart = q - 1 - nx
    out = []
    for t in range(rowpart + (q - 2 - nx)):
        if t < rowpart:
            out.append((r, t if t < r + 1 else t + 1 + nx))
        else:
            u = t - rowpart
            out.append((u if u < r else u + 2 + nx, r))
    return out


def _panel_tiles(pr, q):
    return ([(pr, j if j < pr else j + 1) for j in range(q - 1)] +
            [(i if i < pr else i + 1, pr) for i in range(q - 1)])


def _next_tiles(r, q):
    # round r's phase 3 on block row/column r+1 (the single-round lookahead set)
    return ([(r + 1, t if t < r else t + 1) for t in range(q - 1)] +
            [(t if t < r else t + 2, r + 1) for t in range(q - 2)])


def _pending(i, j, prev):
    return prev >= 0 and (i == prev or j == prev) and i != prev + 1 and j != prev + 1


@pytest.mark.parametrize("q", [2, 3, 4, 5, 6, 7, 8, 9, 10, 13, 17, 33])
def test_pair_tile_maps(q):
    for r in range(q - 1):
        S = {r, r + 1}
        nx = _nxt(q, r)
        nxt = set(range(r + 2, r + 2 + nx))
        n2 = [_next2_tile(t, r, q) for t in range(_next2_count(r, q))]
        want2 = {(i, j) for i in range(q) for j in range(q)
                 if i not in S and j not in S and (i in nxt or j in nxt)}
        assert len(n2) == len(set(n2)) and set(n2) == want2
        for bands in (1, 2, 3):
            got = []
            for g in range(bands):
                lo, hi = q * g // bands, q * (g + 1) // bands
                band = [_rest2_tile(w, r, q, lo, hi) for w in range(_rest2_count(r, q, lo, hi))]
                assert all(lo <= i < hi for i, _ in band)
                got += band
            wantr = {(i, j) for i in range(q) for j in range(q)
                     if i not in S | nxt and j not in S | nxt}
            assert len(got) == len(set(got)) and set(got) == wantr
        fn, ff = _fix_tiles(r, q, False), _fix_tiles(r, q, True)
        assert set(fn) == {(x, r) for x in nxt} | {(r, x) for x in nxt}
        assert len(ff) == len(set(ff)) and not set(ff) & set(fn)
        # every tile of block row/column r but the pair's own off-diagonal ones
        assert set(ff) | set(fn) == ({(r, j) for j in range(q)} | {(i, r) for i in range(q)}) - \
            {(r, r + 1), (r + 1, r)}


# --------------------------------------------------------------------------
# Model of the schedule.  Tiles of b x b on an n = q*b matrix; a task reads
# its operands (one phase) and later writes its tile (another phase).
# --------------------------------------------------------------------------

def _blk(D, b, i, j):
    return D[i * b:(i + 1) * b, j * b:(j + 1) * b]


def _mp(C, A, B):
    return np.minimum(C, (A[:, :, None] + B[None, :, :]).astype(np.float32).min(axis=1))


def _closure(T):
    T = T.copy()
    for k in range(T.shape[0]):
        T = np.minimum(T, (T[:, k:k + 1] + T[k:k + 1, :]).astype(np.float32))
    return T


class _Model:
    def __init__(self, D, b, nstreams, seed):
        self.D, self.b = D, b
        self.q = [[] for _ in range(nstreams)]
        self.tok = 0
        self.last = {}
        self.rng = random.Random(seed)

    # tasks: closures returning a writer
    def upd(self, i, j, kblocks, pend=None, close=False, acopy=None):
        """acopy: {k: copy} takes block (i, k) of the left operand from that
        copy of block column k (the direct-staged rest pass) instead of the
        matrix."""
        D, b = self.D, self.b

        def read():
            acc = _blk(D, b, i, j).copy()
            if pend is not None:
                row, col = pend
                acc = _mp(acc, col[("c", i)].copy(), row[("r", j)].copy())
            for k in kblocks:
                left = acopy[k][("c", i)] if acopy is not None else _blk(D, b, i, k)
                acc = _mp(acc, left.copy(), _blk(D, b, k, j).copy())
            if close:
                acc = _closure(acc)

            def write():
                _blk(D, b, i, j)[:] = acc
            return write
        return read

    def panel(self, r, i, j, copy=None, colcopy=None):
        """copy: block-row and block-column copy slot (the second round of a
        pair); colcopy: block-column copy slot only (the first round).  A slot
        is one buffer, overwritten in place when it is used again: block row
        tiles at ("r", j), block column tiles at ("c", i)."""
        D, b = self.D, self.b

        def read():
            T, X = _blk(D, b, r, r).copy(), _blk(D, b, i, j).copy()
            out = _mp(X, T, X) if i == r else _mp(X, X, T)

            def write():
                _blk(D, b, i, j)[:] = out
                if copy is not None:
                    copy[("r", j) if i == r else ("c", i)] = out.copy()
                if colcopy is not None and j == r:
                    colcopy[("c", i)] = out.copy()
            return write
        return read

    def close_task(self, r):
        D, b = self.D, self.b

        def read():
            T = _closure(_blk(D, b, r, r).copy())

            def write():
                _blk(D, b, r, r)[:] = T
            return write
        return read

    def launch(self, s, tasks):
        if tasks:
            self.q[s].append(["L", list(tasks)])

    def record(self, s, ev):
        self.tok += 1
        self.last[ev] = self.tok
        self.q[s].append(["R", self.tok])

    def wait(self, s, ev):
        if ev in self.last:
            self.q[s].append(["W", self.last[ev]])

    def run(self):
        done, started = set(), []
        heads = [0] * len(self.q)
        todo = [None] * len(self.q)
        busy = [0] * len(self.q)
        weights, step = None, 0

        def advance(s):
            while heads[s] < len(self.q[s]):
                it = self.q[s][heads[s]]
                if it[0] == "R":
                    if busy[s] or todo[s] is not None:
                        return
                    done.add(it[1])
                elif it[0] == "W":
                    if it[1] not in done:
                        return
                else:
                    if todo[s] is None and not busy[s]:
                        todo[s] = list(it[1])
                    if todo[s] or busy[s]:
                        return
                    todo[s] = None
                heads[s] += 1
        while True:
            before = None
            while before != heads:
                before = list(heads)
                for s in range(len(self.q)):
                    advance(s)
            if step % 40 == 0:  # long stalls of random streams
                weights = [self.rng.choice((0.001, 1.0, 1000.0)) for _ in self.q]
            step += 1
            cand = []
            for s in range(len(self.q)):
                acts = ([("s", s)] if todo[s] else []) + \
                       [("f", k) for k, (ss, _) in enumerate(started) if ss == s]
                if acts:
                    cand.append((s, acts))
            if not cand:
                break
            s, acts = self.rng.choices(cand, weights=[weights[c[0]] for c in cand])[0]
            kind, x = self.rng.choice(acts)
            if kind == "s":
                task = todo[s].pop(self.rng.randrange(len(todo[s])))
                started.append((s, task()))
                busy[s] += 1
            else:
                s, w = started.pop(x)
                w()
                busy[s] -= 1
        assert all(heads[s] == len(self.q[s]) for s in range(len(self.q)))


def _pair_schedule(m, q, r0, r1, bands, direct=True, ring=3, first_ring=2):
    """The runtime's enqueue order for rounds r0..r1-1 in pairs (stream 0 is
    the caller's stream, 1.. the band streams).  direct: the rest pass takes
    the column panels of its rounds from their copies (the direct-staged
    kernel), as the runtime does for aligned fp32 matrices of full tiles.
    ring / first_ring: copy slots of a pair's second / first round (3 / 2 in
    the runtime; the tests shorten them to see that the model notices)."""
    S, H = 0, list(range(1, bands + 1))
    copies = [{} for _ in range(ring)]
    firsts = [{} for _ in range(first_ring)]
    prev, prev_slot, slot, first = -1, 0, 0, 0
    rest_pending, diag_closed = False, False

    def band(g):
        return q * g // bands, q * (g + 1) // bands

    def wait_rest(st):
        if rest_pending:
            for g in range(bands):
                m.wait(st, ("rest", g))

    def phases12(r, colcopy=None):
        nonlocal diag_closed
        if not diag_closed:
            m.launch(S, [m.close_task(r)])
        diag_closed = False
        m.launch(S, [m.panel(r, i, j, colcopy=colcopy) for i, j in _panel_tiles(r, q)])

    def pend(i, j):
        if _pending(i, j, prev):
            c = copies[prev_slot]
            return (c, c)
        return None

    def fix(r, final):
        m.launch(S, [m.upd(i, j, [r + 1]) for i, j in _fix_tiles(r, q, final)])

    r = r0
    while r < r1:
        if r + 1 >= r1:
            wait_rest(S)
            rest_pending = False
            if prev >= 0:
                fix(prev, True)
                prev = -1
            phases12(r)
            m.launch(S, [m.upd(i, j, [r]) for i in range(q) for j in range(q)
                         if i != r and j != r])
            r += 1
            break
        nx = _nxt(q, r)
        phases12(r, firsts[first])
        m.launch(S, [m.upd(i, j, [r], close=(i == j == r + 1)) for i, j in _next_tiles(r, q)])
        m.launch(S, [m.panel(r + 1, i, j, copies[slot]) for i, j in _panel_tiles(r + 1, q)])
        acopy = {r: firsts[first], r + 1: copies[slot]} if direct else None
        m.record(S, "p2")
        wait_rest(S)
        close_next = nx > 0 and r + 2 < r1
        if nx:
            m.launch(S, [m.upd(i, j, [r, r + 1], pend(i, j), close_next and i == j == r + 2)
                         for i, j in (_next2_tile(t, r, q) for t in range(_next2_count(r, q)))])
            fix(r, False)
        diag_closed = close_next
        for g in range(bands):
            lo, hi = band(g)
            if rest_pending and prev >= 0 and (lo <= prev < hi or lo <= prev + 1 < hi):
                for o in range(bands):
                    if o != g:
                        m.wait(H[g], ("rest", o))
        for g in range(bands):
            lo, hi = band(g)
            m.wait(H[g], "p2")
            m.launch(H[g], [m.upd(i, j, [r, r + 1], pend(i, j), acopy=acopy)
                            for i, j in (_rest2_tile(w, r, q, lo, hi)
                                         for w in range(_rest2_count(r, q, lo, hi)))])
            m.record(H[g], ("rest", g))
        rest_pending = True
        prev, prev_slot, slot, first = r, slot, (slot + 1) % ring, (first + 1) % first_ring
        r += 2
    wait_rest(S)
    if prev >= 0:
        fix(prev, True)


@pytest.mark.parametrize("q,r0,r1", [(2, 0, 2), (3, 0, 3), (3, 1, 3), (4, 0, 4), (5, 0, 5),
                                     (5, 2, 5), (6, 0, 6), (7, 1, 7),
                                     (8, 0, 8), (9, 0, 9), (10, 0, 7), (10, 3, 10), (11, 1, 11),
                                     (12, 2, 4), (13, 0, 13), (12, 5, 12)])
@pytest.mark.parametrize("bands", [1, 2, 3])
@pytest.mark.parametrize("direct", [False, True])
def test_pair_schedule_model_is_bit_exact(q, r0, r1, bands, direct):
    b = 3
    n = q * b
    rng = np.random.default_rng(1000 * q + 10 * r0 + r1)
    W = rng.uniform(0.5, 10.0, size=(n, n)).astype(np.float32)
    W[rng.random((n, n)) > 0.3] = np.inf
    np.fill_diagonal(W, 0.0)
    start = oracle.blocked(W, b, 0, r0) if r0 else W.copy()
    ref = oracle.blocked(start, b, r0, r1)
    for seed in range(3):
        D = start.copy()
        m = _Model(D, b, 1 + bands, seed * 97 + q)
        _pair_schedule(m, q, r0, r1, bands, direct)
        m.run()
        assert np.array_equal(D.view(np.int32), ref.view(np.int32)), seed


@pytest.mark.parametrize("ring,first_ring", [(2, 2), (3, 1)])
def test_pair_schedule_model_catches_a_short_copy_ring(ring, first_ring):
    """One copy slot fewer than the runtime uses (for either round of a pair)
    lets a pair overwrite a copy that a running band still reads: the model
    sees it in some interleavings."""
    b, q, bands = 3, 14, 2
    n = q * b
    rng = np.random.default_rng(11)
    W = rng.uniform(0.5, 10.0, size=(n, n)).astype(np.float32)
    W[rng.random((n, n)) > 0.3] = np.inf
    np.fill_diagonal(W, 0.0)
    ref = oracle.blocked(W, b)
    differs = 0
    for seed in range(24):
        D = W.copy()
        m = _Model(D, b, 1 + bands, seed)
        _pair_schedule(m, q, 0, q, bands, True, ring, first_ring)
        m.run()
        differs += not np.array_equal(D.view(np.int32), ref.view(np.int32))
    assert differs > 0


def test_pair_schedule_model_catches_a_missing_wait():
    """Without the previous pair's rest set before the next pair's first
    tiles, some interleavings give a different result: the model sees it."""
    b, q, bands = 3, 12, 2
    n = q * b
    rng = np.random.default_rng(7)
    W = rng.uniform(0.5, 10.0, size=(n, n)).astype(np.float32)
    W[rng.random((n, n)) > 0.3] = np.inf
    np.fill_diagonal(W, 0.0)
    ref = oracle.blocked(W, b)
    orig = _Model.wait
    differs = 0
    for seed in range(12):
        D = W.copy()
        m = _Model(D, b, 1 + bands, seed)
        # drop the caller stream's waits for the band streams
        m.wait = lambda s, ev, _m=m: None if s == 0 and isinstance(ev, tuple) else orig(_m, s, ev)
        _pair_schedule(m, q, 0, q, bands)
        m.run()
        differs += not np.array_equal(D.view(np.int32), ref.view(np.int32))
    assert differs > 0


@pytest.mark.parametrize("n", [1024, 1100, 2100, 5000, 16384])
def test_bench_pair_update_count(n):
    """bench.py's algorithmic update count of the pair rest launches (the
    roofline numerator) equals a count over the tiles the maps above assign,
    with their widths, including the deferred updates."""
    import importlib.util
    import os

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    b = 128
    q = -(-n // b)

    def w(x):
        return min(b, n - x * b)

    total, pairs, r, prev = 0, 0, 0, -1
    while r + 1 < q:
        for g in range(2):
            lo, hi = q * g // 2, q * (g + 1) // 2
            for wg in range(_rest2_count(r, q, lo, hi)):
                i, j = _rest2_tile(wg, r, q, lo, hi)
                total += w(i) * w(j) * (w(r) + w(r + 1))
                if _pending(i, j, prev):
                    total += w(i) * w(j) * w(prev + 1)
        pairs += 1
        prev, r = r, r + 2
    assert bench.phase3_pair_updates(n, b) == (total, pairs)

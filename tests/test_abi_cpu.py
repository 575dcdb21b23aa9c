"""C-ABI checks that need no GPU: exported symbols, argument validation
(performed on the host before any HIP call), status strings, and the
workgroup -> tile index maps of the phase kernels, re-derived here and checked
for being bijections onto the tiles each phase must cover."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "apsp.h")


@pytest.fixture(scope="module")
def lib():
    import paper_1902_04446_amd as apsp

    return apsp.library()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(apsp_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("apsp_solve", "apsp_solve_batched", "apsp_solve_batched_ex",
                     "apsp_solve_rounds", "apsp_status_string", "apsp_validate"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    import paper_1902_04446_amd as apsp

    out = subprocess.run(["nm", "-D", "--defined-only", apsp.lib_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (apsp_\w+)", out))
    missing = [f for f in _declared_functions() if f not in exported]
    assert not missing, missing
    for f in _declared_functions():
        getattr(lib, f)


def test_library_is_built_for_gfx950():
    import paper_1902_04446_amd as apsp

    out = subprocess.run(["strings", apsp.lib_path()], capture_output=True, text=True).stdout
    assert "gfx950" in out


def test_host_side_argument_validation(lib):
    vp = ctypes.c_void_p
    fake = vp(0x1000)  # never dereferenced: every call below fails validation first
    assert lib.apsp_solve(fake, -1, 4, 0, None) == 1
    assert lib.apsp_solve(fake, 8, 7, 0, None) == 1          # ld < n
    assert lib.apsp_solve(None, 8, 8, 0, None) == 1          # NULL with n > 0
    assert lib.apsp_solve(fake, 8, 8, 7, None) == 1          # bad dtype
    assert lib.apsp_solve(fake, 1 << 31, 1 << 31, 0, None) == 1
    assert lib.apsp_solve(None, 0, 1, 0, None) == 0          # n == 0 is a no-op
    assert lib.apsp_solve(None, 0, 0, 1, None) == 1          # ld >= 1 always
    assert lib.apsp_solve_rounds(fake, 8, 8, 0, -1, 2, None) == 1
    assert lib.apsp_solve_rounds(fake, 8, 8, 0, 3, 3, None) == 0   # empty range: no-op
    assert lib.apsp_solve_rounds(fake, 8, 8, 0, 5, 9, None) == 0   # r0 beyond q: no-op
    ms = (ctypes.c_double * 8)()
    assert lib.apsp_solve_profiled(fake, 8, 8, 0, None, None) == 1
    assert lib.apsp_solve_profiled(None, 0, 1, 0, None, ms) == 0
    assert lib.apsp_validate(None, 3, 3, 0, None) == 1
    assert lib.apsp_validate(None, 0, 1, 0, None) == 0


def test_batched_argument_validation(lib):
    vp = ctypes.c_void_p
    ptrs = (vp * 2)(0x1000, 0x2000)
    ns = (ctypes.c_int32 * 2)(4, 5)
    assert lib.apsp_solve_batched(None, None, 0, None) == 0
    assert lib.apsp_solve_batched(ptrs, ns, -1, None) == 1
    assert lib.apsp_solve_batched(None, ns, 2, None) == 1
    bad_n = (ctypes.c_int32 * 2)(4, 5000)
    assert lib.apsp_solve_batched(ptrs, bad_n, 2, None) == 1
    neg_n = (ctypes.c_int32 * 2)(4, -1)
    assert lib.apsp_solve_batched(ptrs, neg_n, 2, None) == 1
    null_ptrs = (vp * 2)(0x1000, None)
    assert lib.apsp_solve_batched(null_ptrs, ns, 2, None) == 1
    lds = (ctypes.c_int64 * 2)(4, 4)  # second ld < n
    assert lib.apsp_solve_batched_ex(ptrs, ns, lds, 2, 0, None) == 1
    assert lib.apsp_solve_batched_ex(ptrs, ns, None, 2, 9, None) == 1
    zero_n = (ctypes.c_int32 * 2)(0, 0)
    assert lib.apsp_solve_batched(null_ptrs, zero_n, 2, None) == 0  # all empty: no-op


def test_batched_plan_argument_validation(lib):
    vp = ctypes.c_void_p
    plan = vp(None)
    ns = (ctypes.c_int32 * 2)(4, 5)
    ptrs = (vp * 2)(0x1000, 0x2000)
    assert lib.apsp_batched_plan_create(ptrs, ns, None, 2, 0, None, None) == 1
    assert lib.apsp_batched_plan_create(ptrs, ns, None, -1, 0, None, ctypes.byref(plan)) == 1
    assert lib.apsp_batched_plan_create(None, ns, None, 2, 0, None, ctypes.byref(plan)) == 1
    assert lib.apsp_batched_plan_create(ptrs, ns, None, 2, 3, None, ctypes.byref(plan)) == 1
    assert not plan
    # an empty batch needs no device at all
    assert lib.apsp_batched_plan_create(None, None, None, 0, 0, None, ctypes.byref(plan)) == 0
    assert plan
    info = (ctypes.c_int64 * 3)()
    assert lib.apsp_batched_plan_info(plan, info) == 0 and list(info) == [0, 0, 0]
    assert lib.apsp_batched_plan_run(plan, None) == 0
    assert lib.apsp_batched_plan_destroy(plan) == 0
    assert lib.apsp_batched_plan_run(None, None) == 1
    assert lib.apsp_batched_plan_destroy(None) == 0


def test_tiled_plan_and_tuning_argument_validation(lib):
    vp = ctypes.c_void_p
    plan = vp(None)
    ns = (ctypes.c_int32 * 2)(4, 5)
    ptrs = (vp * 2)(0x1000, 0x2000)
    for bad_tile in (-1, 1, 32, 96, 256):
        assert lib.apsp_batched_plan_create_tiled(ptrs, ns, None, 2, 0, bad_tile, None,
                                                  ctypes.byref(plan)) == 1
    assert lib.apsp_batched_plan_create_tiled(ptrs, ns, None, 2, 0, 64, None, None) == 1
    assert not plan
    for tile in (0, 64, 128):  # an empty batch needs no device, whatever the width
        assert lib.apsp_batched_plan_create_tiled(None, None, None, 0, 1, tile, None,
                                                  ctypes.byref(plan)) == 0
        assert plan
        assert lib.apsp_batched_plan_destroy(plan) == 0
        plan = vp(None)
    nb = 9
    good = (ctypes.c_int32 * nb)(*([128] * nb))
    bad = (ctypes.c_int32 * nb)(*([64] * 8 + [100]))
    assert lib.apsp_batched_tuning_set(None, nb) == 1
    assert lib.apsp_batched_tuning_set(good, nb - 1) == 1
    assert lib.apsp_batched_tuning_set(bad, nb) == 1
    assert lib.apsp_batched_tuning_get(None, nb) == 1
    assert lib.apsp_batched_tuning_get(good, 10) == 1
    assert lib.apsp_batched_autotune(2, 1 << 24, None, None, None) == 1      # dtype
    assert lib.apsp_batched_autotune(0, 1 << 19, None, None, None) == 1      # batch too small
    assert lib.apsp_batched_autotune(0, (1 << 30) + 1, None, None, None) == 1
    assert lib.apsp_batched_autotune_batch(ptrs, ns, None, 0, 0, None, None, None) == 1
    assert lib.apsp_batched_autotune_batch(None, ns, None, 2, 0, None, None, None) == 1
    assert lib.apsp_batched_autotune_batch(ptrs, ns, None, 2, 7, None, None, None) == 1
    big = (ctypes.c_int32 * 2)(4, 5000)
    assert lib.apsp_batched_autotune_batch(ptrs, big, None, 2, 0, None, None, None) == 1
    empty = (ctypes.c_int32 * 2)(0, 0)
    assert lib.apsp_batched_autotune_batch(ptrs, empty, None, 2, 0, None, None, None) == 1


def test_minplus_and_squaring_argument_validation(lib):
    vp = ctypes.c_void_p
    a, b, c = vp(0x10000), vp(0x80000), vp(0x100000)
    assert lib.apsp_minplus(c, 8, a, 8, b, 8, 8, 8, 8, 5, 0, None) == 1       # dtype
    assert lib.apsp_minplus(c, 8, a, 8, b, 8, 8, 8, 0, 0, 0, None) == 1       # k == 0
    assert lib.apsp_minplus(c, 8, a, 8, b, 8, 0, 8, 8, 0, 0, None) == 0       # m == 0: no-op
    assert lib.apsp_minplus(c, 7, a, 8, b, 8, 8, 8, 8, 0, 0, None) == 1       # ldc < n
    assert lib.apsp_minplus(c, 8, a, 7, b, 8, 8, 8, 8, 0, 0, None) == 1       # lda < k
    assert lib.apsp_minplus(None, 8, a, 8, b, 8, 8, 8, 8, 0, 0, None) == 1
    assert lib.apsp_minplus(a, 8, a, 8, b, 8, 8, 8, 8, 0, 0, None) == 1       # C overlaps A
    assert lib.apsp_minplus(vp(0x80000 + 64), 8, a, 8, b, 8, 8, 8, 8, 0, 0, None) == 1  # C in B
    assert lib.apsp_squarings(0) == 0 and lib.apsp_squarings(2) == 0
    assert lib.apsp_squarings(3) == 1 and lib.apsp_squarings(5) == 2 and lib.apsp_squarings(6) == 3
    assert lib.apsp_squarings(16385) == 14
    assert lib.apsp_solve_squaring(a, 8, 8, 0, None, 8, None) == 1           # no work buffer
    assert lib.apsp_solve_squaring(a, 8, 8, 0, vp(0x10000 + 16), 8, None) == 1  # overlapping
    assert lib.apsp_solve_squaring(a, 8, 8, 0, b, 7, None) == 1              # ldw < n
    assert lib.apsp_solve_squaring(None, 0, 1, 0, None, 1, None) == 0


def test_status_strings_and_widths(lib):
    for code in range(6):
        s = lib.apsp_status_string(code)
        assert s and s.startswith(b"APSP")
    assert lib.apsp_status_string(99) == b"APSP: unknown status"
    assert lib.apsp_round_width(100, 0) == 64 and lib.apsp_round_width(5120, 1) == 64
    assert lib.apsp_round_width(5121, 0) == 128 and lib.apsp_round_width(16384, 1) == 128
    assert lib.apsp_round_width(100, 5) == 0
    assert lib.apsp_batched_round_width(300, 0) == 128
    assert b"gfx950" in lib.apsp_version()


def test_width64_limit_setter(lib):
    """No HIP call: the width-64 limit is process-wide, in [0, 8192]."""
    prev = lib.apsp_set_width64_max_n(300)
    try:
        assert prev >= 0
        assert lib.apsp_round_width(300, 1) == 64 and lib.apsp_round_width(301, 1) == 128
        assert lib.apsp_set_width64_max_n(-1) == -1
        assert lib.apsp_set_width64_max_n(8193) == -1
        assert lib.apsp_set_width64_max_n(0) == 300
        assert lib.apsp_round_width(1, 0) == 128
    finally:
        lib.apsp_set_width64_max_n(prev)


def test_aligned_copy_threshold_setter(lib):
    """No HIP call: the threshold of the aligned working copy is a
    process-wide vertex count >= 0 (default 512)."""
    prev = lib.apsp_set_aligned_copy_min_n(1000)
    try:
        assert prev >= 0
        assert lib.apsp_set_aligned_copy_min_n(-1) == -1
        assert lib.apsp_set_aligned_copy_min_n(1 << 40) == 1000
        assert lib.apsp_set_aligned_copy_min_n(0) == 1 << 40
    finally:
        lib.apsp_set_aligned_copy_min_n(prev)
    # n == 0 with an ld off 4 is still a no-op that touches no device
    assert lib.apsp_solve(None, 0, 3, 0, None) == 0
    assert lib.apsp_solve_rounds(None, 0, 3, 1, 0, 5, None) == 0


def test_round_pair_threshold_setter(lib):
    """No HIP call: the setter swaps a process-wide value and rejects < 2."""
    prev = lib.apsp_set_round_pair_threshold(9)
    try:
        assert prev >= 2
        assert lib.apsp_set_round_pair_threshold(1) == -1
        assert lib.apsp_set_round_pair_threshold(10) == 9
    finally:
        lib.apsp_set_round_pair_threshold(prev)


def test_stream_state_bytes(lib):
    """No HIP call: the per-stream state a full solve creates.  fp32 solves
    below the lookahead (16 rounds of 64) keep none; int32 solves keep the
    256-byte scan word; from 72 rounds of 128 the pair copies, 8 x 128 x 128q
    words, come on top, and so do they for single rounds of 128 with
    n % 128 == 0 (the direct-staged rest set reads their transposed column
    slots) in fp32, and in int32 from 64 rounds (held as fp32 bits); from 64
    rounds a ragged n is solved padded to a multiple of 128."""
    f32, i32 = 1, 0
    assert lib.apsp_stream_state_bytes(0, f32) == 0
    assert lib.apsp_stream_state_bytes(1000, f32) == 0
    assert lib.apsp_stream_state_bytes(1000, i32) == 256
    # 64 rounds of 128, single rounds with the direct-staged rest set: the
    # transposed column copies come with the state (fp32, n % 128 == 0)
    assert lib.apsp_stream_state_bytes(8192, f32) == 256 + 8 * 128 * 8192 * 4
    # 64 rounds with n % 128 != 0: solved padded to a multiple of 128 when that
    # adds at most 1 % to n (8150 -> 8192), in place otherwise (8100)
    assert lib.apsp_stream_state_bytes(8150, f32) == 256 + 8 * 128 * 8192 * 4
    assert lib.apsp_stream_state_bytes(8100, f32) == 256
    assert lib.apsp_stream_state_bytes(8000, f32) == 256       # 63 rounds: register-staged
    # int32 from 64 rounds is held as fp32 bits and runs the direct-staged kernels
    assert lib.apsp_stream_state_bytes(8192, i32) == 256 + 8 * 128 * 8192 * 4
    assert lib.apsp_stream_state_bytes(8064, i32) == 256       # 63 rounds: int32 kernels
    assert lib.apsp_stream_state_bytes(16384, f32) == 256 + 8 * 128 * 16384 * 4
    assert lib.apsp_stream_state_bytes(16385, i32) == 256 + 8 * 128 * 16512 * 4
    assert lib.apsp_stream_state_bytes(100, 7) == -1
    assert lib.apsp_stream_state_bytes(-1, f32) == -1
    prev = lib.apsp_set_round_pair_threshold(1 << 20)  # no pairs at any size
    try:
        assert lib.apsp_stream_state_bytes(16385, i32) == 256 + 8 * 128 * 16512 * 4
        assert lib.apsp_stream_state_bytes(16384, f32) == 256 + 8 * 128 * 16384 * 4
        prev_copy = lib.apsp_set_aligned_copy_min_n(1 << 40)  # no working copies
        try:
            assert lib.apsp_stream_state_bytes(16385, i32) == 256   # ragged: int32 kernels
            assert lib.apsp_stream_state_bytes(8150, f32) == 256
        finally:
            lib.apsp_set_aligned_copy_min_n(prev_copy)
    finally:
        lib.apsp_set_round_pair_threshold(prev)
    assert lib.apsp_stream_state_count() >= 0


def test_binding_rejects_host_tensors():
    import torch

    import paper_1902_04446_amd as apsp

    with pytest.raises(ValueError):
        apsp.solve(torch.zeros(4, 4, dtype=torch.int32))
    with pytest.raises((TypeError, ValueError)):
        apsp.solve(torch.zeros(4, 4, dtype=torch.float64))


# --------------------------------------------------------------------------
# Workgroup -> tile maps of the phase-2 and phase-3 launches, re-derived.
# --------------------------------------------------------------------------

def _phase2_tile(wg, r, q):
    if wg < q - 1:
        return r, (wg if wg < r else wg + 1)
    t = wg - (q - 1)
    return (t if t < r else t + 1), r


def _phase3_tile(wg, r, q, skip=1):
    # skip = 1: every tile outside block row/column r;
    # skip = 2: every tile outside block rows/columns r and r+1
    m = q - skip
    T = m * m
    x, s = wg & 7, wg >> 3
    per, rem = T >> 3, T & 7
    tile = x * per + min(x, rem) + s
    ti, tj = divmod(tile, m)
    return (ti if ti < r else ti + skip), (tj if tj < r else tj + skip)


def _rest_band_tile(wg, r, q, lo, hi):
    # phase-3 tiles outside rows/columns r, r+1 whose block row is in [lo, hi)
    m = q - 2
    rows = hi - lo - (lo <= r < hi) - (lo <= r + 1 < hi)
    T = rows * m
    x, s = wg & 7, wg >> 3
    per, rem = T >> 3, T & 7
    tile = x * per + min(x, rem) + s
    ti, tj = divmod(tile, m)
    i = lo + ti
    if r >= lo and i >= r:
        i += 1
    if r + 1 >= lo and i >= r + 1:
        i += 1
    return i, (tj if tj < r else tj + 2)


def _band_count(r, q, lo, hi):
    rows = hi - lo - (lo <= r < hi) - (lo <= r + 1 < hi)
    return max(rows, 0) * (q - 2) if r + 1 < q else 0


def _next_tile(wg, r, q):
    # block row r+1 (all columns but r), then block column r+1 (rows but r, r+1)
    if wg < q - 1:
        return r + 1, (wg if wg < r else wg + 1)
    t = wg - (q - 1)
    return (t if t < r else t + 2), r + 1


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5, 9, 17, 33])
def test_phase_tile_maps_are_bijections(q):
    for r in range(q):
        p2 = [_phase2_tile(w, r, q) for w in range(2 * (q - 1))]
        expect2 = {(r, j) for j in range(q) if j != r} | {(i, r) for i in range(q) if i != r}
        assert len(set(p2)) == len(p2) and set(p2) == expect2
        p3 = [_phase3_tile(w, r, q) for w in range((q - 1) ** 2)]
        expect3 = {(i, j) for i in range(q) for j in range(q) if i != r and j != r}
        assert len(set(p3)) == len(p3) and set(p3) == expect3
        # each XCD (wg % 8) receives one contiguous run of tiles
        for x in range(8):
            ids = [(_phase3_tile(w, r, q)) for w in range(x, (q - 1) ** 2, 8)]
            assert len(ids) == len(set(ids))
        if r + 1 < q:
            # lookahead split of phase 3: next set + rest set = the whole phase
            nxt = [_next_tile(w, r, q) for w in range(2 * q - 3)]
            rest = [_phase3_tile(w, r, q, skip=2) for w in range((q - 2) ** 2)]
            assert len(set(nxt)) == len(nxt) and len(set(rest)) == len(rest)
            assert set(nxt) | set(rest) == expect3 and not set(nxt) & set(rest)
            assert set(nxt) == {t for t in expect3 if r + 1 in t}
            # the rest set split in bands of block rows: disjoint, covering it,
            # the full band [0, q) being the rest set itself
            full = [_rest_band_tile(w, r, q, 0, q) for w in range(_band_count(r, q, 0, q))]
            assert full == rest
            for bands in (2, 3):
                got = []
                for g in range(bands):
                    lo, hi = q * g // bands, q * (g + 1) // bands
                    band = [_rest_band_tile(w, r, q, lo, hi)
                            for w in range(_band_count(r, q, lo, hi))]
                    assert all(lo <= i < hi for i, _ in band)
                    got += band
                assert len(got) == len(set(got)) and set(got) == set(rest)


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU; asked for more it says so and exits 2 before
    touching any device."""
    out = subprocess.run(["python3", os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr and out.stdout == ""


def test_binding_rejects_overlapping_row_views():
    """A broadcast or overlapping view would make the library write one element
    through several indices; the binding rejects it before any HIP call (the
    tensors here are host tensors, so a HIP call would fail differently)."""
    import torch

    import paper_1902_04446_amd as apsp

    bad = [torch.full((5,), 1.0).expand(5, 5),
           torch.zeros(40, dtype=torch.int32).as_strided((5, 5), (3, 1)),
           torch.zeros(40).as_strided((5, 5), (0, 1))]
    for t in bad:
        with pytest.raises(ValueError, match="rows overlap"):
            apsp._matrix_args(t)
        with pytest.raises(ValueError, match="rows overlap"):
            apsp.solve(t)
        with pytest.raises(ValueError, match="rows overlap"):
            apsp._batch_arrays([torch.zeros((3, 3), dtype=t.dtype), t])
        with pytest.raises(ValueError, match="rows overlap"):
            apsp.minplus(torch.zeros((5, 5), dtype=t.dtype), t, torch.zeros((5, 5), dtype=t.dtype))
    # non-unit column stride (a transposed view)
    with pytest.raises(ValueError, match="contiguous"):
        apsp._matrix_args(torch.zeros((4, 4)).t()[:, :3][:3])
    # padded rows are fine (the check reaches the device test only)
    padded = torch.zeros((4, 7))[:, :4]
    with pytest.raises(ValueError, match="device"):
        apsp._matrix_args(padded)
    # single rows: no row stride to check
    with pytest.raises(ValueError, match="device"):
        apsp._matrix_args(torch.zeros((1, 1)))

"""The kernels' own workgroup -> tile maps (apsp_tilemap.h, the code the
phase kernels call with their workgroup index), compiled for the host and
compared with the independent derivations of the CPU tests, which those
tests check to be bijections onto each phase's tile set.  The symmetric
solver's maps are checked directly."""
import os
import subprocess

import pytest

import test_abi_cpu as single
import test_pair_schedule as pair

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def maps(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("tilemap") / "tilemap_dump")
    subprocess.run([HIPCC, "-x", "hip", "--cuda-host-only", "-O1", "-std=c++17",
                    os.path.join(ROOT, "tests", "tilemap_dump.cpp"), "-o", exe],
                   check=True, capture_output=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    table = {}
    for line in out.splitlines():
        head, _, tiles = line.partition(":")
        name, q, r, a, b = head.split()
        key = (name, int(q), int(r), int(a), int(b))
        table[key] = [tuple(int(v) for v in t.split(",")) for t in tiles.split()]
    return table


def _qr(table, name):
    return sorted({(k[1], k[2]) for k in table if k[0] == name})


def test_single_round_maps_match(maps):
    assert _qr(maps, "all")
    for q, r in _qr(maps, "all"):
        assert maps[("panels", q, r, 0, 0)] == [single._phase2_tile(w, r, q)
                                                for w in range(2 * (q - 1))]
        assert maps[("all", q, r, 0, 0)] == [single._phase3_tile(w, r, q)
                                             for w in range((q - 1) ** 2)]
        if r + 1 < q:
            assert maps[("next", q, r, 0, 0)] == [single._next_tile(w, r, q)
                                                  for w in range(2 * q - 3)]
        for bands in (1, 2, 3):
            for g in range(bands):
                lo, hi = q * g // bands, q * (g + 1) // bands
                want = [single._rest_band_tile(w, r, q, lo, hi)
                        for w in range(single._band_count(r, q, lo, hi))]
                assert maps[("rest", q, r, lo, hi)] == want, (q, r, lo, hi)


def test_round_pair_maps_match(maps):
    for q, r in _qr(maps, "pnextr"):
        assert maps[("psnap", q, r, 0, 0)] == pair._panel_tiles(r, q)
        assert maps[("pnextr", q, r, 0, 0)] == pair._next_tiles(r, q)
        assert maps[("pnext2", q, r, 0, 0)] == [pair._next2_tile(t, r, q)
                                                for t in range(pair._next2_count(r, q))]
        for bands in (1, 2):
            for g in range(bands):
                lo, hi = q * g // bands, q * (g + 1) // bands
                want = [pair._rest2_tile(w, r, q, lo, hi)
                        for w in range(pair._rest2_count(r, q, lo, hi))]
                assert maps[("prest2", q, r, lo, hi)] == want, (q, r, lo, hi)
        assert maps[("pfix", q, r, 0, 0)] == pair._fix_tiles(r, q, False)
        assert maps[("pfix", q, r, 1, 0)] == pair._fix_tiles(r, q, True)


def _upper(q, skip):
    return [(i, j) for i in range(q) for j in range(i, q) if i not in skip and j not in skip]


def test_symmetric_maps_are_bijections_with_xcd_runs(maps):
    for q, r in _qr(maps, "sall"):
        for name, skip in (("sall", {r}), ("srest", {r, r + 1})):
            if name == "srest" and r + 1 >= q:
                continue
            got = maps[(name, q, r, 0, 0)]
            want = _upper(q, skip)
            assert sorted(got) == sorted(want) and len(set(got)) == len(got), (name, q, r)
            # the workgroups of each XCD (wg % 8) take one contiguous run of
            # the upper triangle in row-major order
            pos = {t: k for k, t in enumerate(want)}
            for x in range(8):
                run = [pos[t] for t in got[x::8]]
                assert run == list(range(run[0], run[0] + len(run))) if run else True
        if r + 1 < q:
            nxt = maps[("snext", q, r, 0, 0)]
            assert nxt[0] == (r + 1, r + 1)
            assert sorted(nxt) == sorted(t for t in _upper(q, {r}) if r + 1 in t)
            # next + rest = all, disjoint
            rest = maps[("srest", q, r, 0, 0)]
            assert sorted(nxt + rest) == sorted(maps[("sall", q, r, 0, 0)])

// Workgroup -> tile maps of the single-graph phase launches (round r of q
// rounds; tile (I, J) is block row I, block column J).  Host-and-device code:
// the kernels call them with their workgroup index, and a host-side check
// builds them on the CPU to show that each map is a bijection onto its tile
// set (tests/test_abi_cpu.py).
//
//   kPanels  phase 2: block row r (every column but r), then block column r
//            (every row but r), 2(q-1) tiles;
//   kNext    phase 3 on block row r+1 (every column but r), then block column
//            r+1 (every row but r, r+1): the tiles the next round's phases 1
//            and 2 read, 2q-3 tiles;
//   kAll     phase 3: every tile outside block row/column r, (q-1)^2;
//   kRest    phase 3 outside block rows/columns r, r+1, restricted to the
//            block rows in [row_lo, row_hi) (a band), (rows) (q-2) tiles.
//
// kAll and kRest deal tiles so that each XCD (workgroup w runs on XCD w % 8)
// gets one contiguous range of them in row-major order: the tiles sharing
// panel blocks then share that XCD's L2.
#pragma once

#include "apsp_common.h"

namespace apsp {
namespace tilemap {

template <int MODE>
__host__ __device__ inline void tile_of(int wg, int r, int q, int row_lo, int row_hi, int &I,
                                        int &J) {
    if (MODE == kPanels) {
        int tt = wg;
        if (tt < q - 1) {
            I = r;
            J = tt < r ? tt : tt + 1;
        } else {
            tt -= q - 1;
            J = r;
            I = tt < r ? tt : tt + 1;
        }
    } else if (MODE == kNext) {
        int tt = wg;
        if (tt < q - 1) {
            I = r + 1;
            J = tt < r ? tt : tt + 1;
        } else {
            tt -= q - 1;
            J = r + 1;
            I = tt < r ? tt : tt + 2;
        }
    } else {
        const int skip = (MODE == kRest) ? 2 : 1;
        const int m = q - skip;
        const int rows = (MODE == kRest)
                             ? row_hi - row_lo - (r >= row_lo && r < row_hi ? 1 : 0) -
                                   (r + 1 >= row_lo && r + 1 < row_hi ? 1 : 0)
                             : m;
        const int T = rows * m;
        const int x = wg & 7, s = wg >> 3;
        const int per = T >> 3, rem = T & 7;
        const int tile = x * per + (x < rem ? x : rem) + s;
        const int ti = tile / m, tj = tile - ti * m;
        if (MODE == kRest) {
            I = row_lo + ti;
            if (r >= row_lo && I >= r) ++I;
            if (r + 1 >= row_lo && I >= r + 1) ++I;
        } else {
            I = ti < r ? ti : ti + skip;
        }
        J = tj < r ? tj : tj + skip;
    }
}

// Tiles in a launch of set MODE (kRest: over block rows [row_lo, row_hi)).
__host__ __device__ inline int64_t tile_count(int64_t q, int64_t r, int set, int64_t row_lo,
                                              int64_t row_hi) {
    if (r < 0 || r >= q) return 0;
    switch (set) {
    case kPanels: return 2 * (q - 1);
    case kAll: return (q - 1) * (q - 1);
    case kNext: return (r + 1 < q) ? 2 * q - 3 : 0;
    case kRest: {
        if (r + 1 >= q || row_lo >= row_hi) return 0;
        const int64_t rows = row_hi - row_lo - (r >= row_lo && r < row_hi ? 1 : 0) -
                             (r + 1 >= row_lo && r + 1 < row_hi ? 1 : 0);
        return rows > 0 ? rows * (q - 2) : 0;
    }
    default: return 0;
    }
}

}  // namespace tilemap
}  // namespace apsp

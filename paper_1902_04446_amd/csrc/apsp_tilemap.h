// Workgroup -> tile maps of the single-graph phase launches (round r of q
// rounds; tile (I, J) is block row I, block column J), the single rounds'
// and the round pairs'.  Host-and-device code: the kernels call them with
// their workgroup index, and a host-side check compiles this header into a
// small CPU program that prints the maps (tests/tilemap_dump.cpp), to show
// that each map is a bijection onto its tile set.
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

// Tile sets of the round-pair launches (apsp_pair.hip), pair (r, r+1):
//   kPanelsSnap  phase 2 of round r (its order: block row r, then block
//                column r), its panels also copied;
//   kNext2       the pass on block rows r+2 .. r+1+nxt (every column outside
//                r, r+1), then block columns r+2 .. r+1+nxt (every row outside
//                r .. r+1+nxt), nxt = min(2, q - r - 2);
//   kRest2       the pass on block rows [lo, hi) and columns outside the
//                blocks [r, r+2+nxt), each XCD one contiguous run of tiles;
//   kFix         round r+1's deferred update on block row/column r: final_ 0
//                tiles (x, r), (r, x) for x = r+2 .. r+1+nxt; final_ 1 block
//                row r but columns r+1 and those x, then block column r but
//                rows r, r+1 and those x;
//   kNextR       round r's phase 3 on block row r+1 (every column but r),
//                then block column r+1 (every row but r, r+1).
//   kRest1       a single round's phase 3 on block rows [lo, hi) outside block
//                rows/columns r, r+1: the band map of kRest above.
constexpr int kPanelsSnap = 0;
constexpr int kNext2 = 1;
constexpr int kRest2 = 2;
constexpr int kFix = 3;
constexpr int kNextR = 4;
constexpr int kRest1 = 5;

template <int MODE>
__host__ __device__ inline void pair_tile_of(int t, int r, int q, int nxt, int lo, int hi,
                                             int final_, int &I, int &J) {
    if (MODE == kRest1) {
        tile_of<kRest>(t, r, q, lo, hi, I, J);
    } else if (MODE == kPanelsSnap) {
        if (t < q - 1) {
            I = r;
            J = t < r ? t : t + 1;
        } else {
            t -= q - 1;
            J = r;
            I = t < r ? t : t + 1;
        }
    } else if (MODE == kFix) {
        if (!final_) {
            const int x = r + 2 + (t >> 1);
            I = (t & 1) ? r : x;
            J = (t & 1) ? x : r;
        } else {
            const int rowpart = q - 1 - nxt;
            if (t < rowpart) {
                I = r;
                J = t < r + 1 ? t : t + 1 + nxt;
            } else {
                t -= rowpart;
                J = r;
                I = t < r ? t : t + 2 + nxt;
            }
        }
    } else if (MODE == kNextR) {
        if (t < q - 1) {
            I = r + 1;
            J = t < r ? t : t + 1;
        } else {
            t -= q - 1;
            J = r + 1;
            I = t < r ? t : t + 2;
        }
    } else if (MODE == kNext2) {
        const int m = q - 2;  // blocks outside r, r+1
        if (t < nxt * m) {
            I = r + 2 + t / m;
            const int c = t % m;
            J = c < r ? c : c + 2;
        } else {
            t -= nxt * m;
            const int m2 = m - nxt;
            J = r + 2 + t / m2;
            const int c = t % m2;
            I = c < r ? c : c + 2 + nxt;
        }
    } else {  // kRest2
        const int e1 = r + 2 + nxt;
        const int ex = e1 - r;
        const int x0 = r > lo ? r : lo, x1 = e1 < hi ? e1 : hi;
        const int skipped = x1 > x0 ? x1 - x0 : 0;
        const int rows = hi - lo - skipped;
        const int mc = q - ex;
        const int T = rows * mc;
        const int x = t & 7, s = t >> 3;
        const int per = T >> 3, rem = T & 7;
        const int tl = x * per + (x < rem ? x : rem) + s;  // one contiguous run per XCD
        const int ti = tl / mc, tj = tl - ti * mc;
        I = lo + ti;
        if (skipped && I >= x0) I += skipped;
        J = tj < r ? tj : tj + ex;
    }
}

// Tile sets of the symmetric solver's phase 3 (apsp_symmetric.hip), upper
// tiles (I <= J) only:
//   kSymAll   every upper tile outside block row/column r, (q-1) q / 2;
//   kSymRest  outside block rows/columns r and r+1, (q-2) (q-1) / 2;
//   kSymNext  the upper tiles in block row/column r+1, q-1: (r+1, r+1 ..
//             q-1), diagonal first, then (0 .. r-1, r+1).
// kSymAll and kSymRest take the a <= b entries of the m x m grid of block
// indices without r (and r+1), row-major, each XCD one contiguous run.
constexpr int kSymAll = 0;
constexpr int kSymRest = 1;
constexpr int kSymNext = 2;

__host__ __device__ inline void upper_tile(int wg, int r, int q, int skip, int &I, int &J) {
    const int m = q - skip;
    const int T = m * (m + 1) / 2;
    const int x = wg & 7, s = wg >> 3;
    const int per = T >> 3, rem = T & 7;
    const int id = x * per + (x < rem ? x : rem) + s;
    // rows before row a hold start(a) = a m - a (a - 1) / 2 entries; a from
    // the quadratic's root, then corrected by whole rows
    auto start = [&](int a) { return a * m - a * (a - 1) / 2; };
    const double w = 2.0 * m + 1.0;
    int a = (int)((w - sqrt(w * w - 8.0 * id)) * 0.5);
    a = a < 0 ? 0 : (a > m - 1 ? m - 1 : a);
    while (a + 1 < m && start(a + 1) <= id) ++a;
    while (a > 0 && start(a) > id) --a;
    const int b = a + (id - start(a));
    I = a < r ? a : a + skip;
    J = b < r ? b : b + skip;
}

template <int SET>
__host__ __device__ inline void sym_tile_of(int wg, int r, int q, int &I, int &J) {
    if (SET == kSymNext) {
        if (wg < q - 1 - r) {  // (r+1, r+1) first: its closure is the chain
            I = r + 1;
            J = r + 1 + wg;
        } else {
            I = wg - (q - 1 - r);
            J = r + 1;
        }
    } else {
        upper_tile(wg, r, q, SET == kSymRest ? 2 : 1, I, J);
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

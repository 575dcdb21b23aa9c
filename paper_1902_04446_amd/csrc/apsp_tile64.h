// Device building blocks of the 64 x 64-tile form of the batched solver:
// one workgroup of 256 threads per 64 x 64 tile, thread (tx, ty) =
// (t % 16, t / 16) keeping rows 4ty .. 4ty+3, columns 4tx .. 4tx+3 in
// registers for the whole item.
//   update    the 64-wide k range of A (stored as k-pairs) and B is staged in
//             LDS in full, then c = min3(c, a0 + b0, a1 + b1) per k-pair
//             (arXiv:1902.04446, Table 1: MinPlus);
//   closure   plain Floyd-Warshall over the register tile, pivots ascending:
//             the owners of pivot row and column k put them in LDS (double
//             buffered), one barrier per pivot (Table 1: FloydWarshall).
// Round width 64 wastes less work on padding than 128 for graphs just above
// a multiple of 128 and runs a quarter of the closure work per vertex; its
// 4 x 4 register block does more LDS traffic per update than the 128-wide
// tile.  Tiles are normalised as they are loaded (Op::norm, zero diagonal on
// diagonal tiles) and converted back as they are stored (Op::out).
#pragma once

#include "apsp_common.h"

namespace apsp {
namespace tile64 {

constexpr int T64 = 64;
constexpr int NT64 = 256;

struct Lds64 {
    uint2 As[T64 / 2][T64];   // As[p][i] = (A[i][2p], A[i][2p+1])
    uint4 Bs[T64][T64 / 4];   // Bs[k][c] = B[k][4c .. 4c+3]
    uint32_t rowbuf[2][T64];  // pivot row (closure)
    uint32_t colbuf[2][T64];  // pivot column (closure)
};

__device__ __forceinline__ uint4 ld4_64(const uint32_t *p) {
    return *reinterpret_cast<const uint4 *>(p);
}

// acc = normalised tile (i0, j0) of D, padded outside mr x nc; zero diagonal
// when the tile is a diagonal one.
template <class Op>
__device__ __forceinline__ void load64(uint32_t (&acc)[4][4], const uint32_t *D, int64_t ld,
                                       int i0, int j0, int mr, int nc, bool vec) {
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const uint32_t PAD = Op::pad();
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int row = ty * 4 + m;
        const uint32_t *crow = D + (int64_t)(i0 + (row < mr ? row : mr - 1)) * ld + j0;
        uint32_t x[4];
        if (vec && tx * 4 + 4 <= nc) {
            const uint4 v = ld4_64(crow + tx * 4);
            x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int c = tx * 4 + e;
                x[e] = crow[c < nc ? c : nc - 1];
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int c = tx * 4 + e;
            const uint32_t y = (row < mr && c < nc) ? Op::norm(x[e]) : PAD;
            acc[m][e] = (i0 == j0 && row == c) ? 0u : y;
        }
    }
}

template <class Op>
__device__ __forceinline__ void store64(const uint32_t (&acc)[4][4], uint32_t *D, int64_t ld,
                                        int i0, int j0, int mr, int nc, bool vec) {
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int row = ty * 4 + m;
        if (row >= mr) continue;
        uint32_t *crow = D + (int64_t)(i0 + row) * ld + j0 + tx * 4;
        if (vec && tx * 4 + 4 <= nc) {
            *reinterpret_cast<uint4 *>(crow) = make_uint4(Op::out(acc[m][0]), Op::out(acc[m][1]),
                                                          Op::out(acc[m][2]), Op::out(acc[m][3]));
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (tx * 4 + e < nc) crow[e] = Op::out(acc[m][e]);
        }
    }
}

// acc = min(acc, A (x) B) with A = D[i0 .., kb .. kb+kw), B = D[kb .. kb+kw, j0 ..]
// (mr x kw and kw x nc valid).  Both operands are staged in full before the
// caller stores acc, so the output tile may be one of them (phase 2).
template <class Op>
__device__ __forceinline__ void update64(uint32_t (&acc)[4][4], const uint32_t *D, int64_t ld, int i0, int j0,
                         int kb, int mr, int nc, int kw, bool vec, Lds64 &L) {
    const int t = threadIdx.x;
    const uint32_t PAD = Op::pad();
    {   // A: row t/4, k offset (t%4)*16 .. +15
        const int ar = t >> 2, ak = (t & 3) * 16;
        const uint32_t *src = D + (int64_t)(i0 + (ar < mr ? ar : mr - 1)) * ld + kb;
        uint32_t a[16];
        if (vec && ar < mr && ak + 16 <= kw) {
#pragma unroll
            for (int w = 0; w < 16; w += 4) {
                const uint4 x = ld4_64(src + ak + w);
                a[w] = x.x; a[w + 1] = x.y; a[w + 2] = x.z; a[w + 3] = x.w;
            }
        } else {
#pragma unroll
            for (int w = 0; w < 16; ++w) {
                const uint32_t x = src[ak + w < kw ? ak + w : kw - 1];
                a[w] = (ar < mr && ak + w < kw) ? x : PAD;
            }
        }
#pragma unroll
        for (int p = 0; p < 8; ++p)
            L.As[(ak >> 1) + p][ar] = make_uint2(Op::norm(a[2 * p]), Op::norm(a[2 * p + 1]));
    }
    {   // B: k row t/4, columns (t%4)*16 .. +15
        const int br = t >> 2, bc = (t & 3) * 16;
        const uint32_t *src = D + (int64_t)(kb + (br < kw ? br : kw - 1)) * ld + j0;
        uint32_t b[16];
        if (vec && br < kw && bc + 16 <= nc) {
#pragma unroll
            for (int w = 0; w < 16; w += 4) {
                const uint4 x = ld4_64(src + bc + w);
                b[w] = x.x; b[w + 1] = x.y; b[w + 2] = x.z; b[w + 3] = x.w;
            }
        } else {
#pragma unroll
            for (int w = 0; w < 16; ++w) {
                const uint32_t x = src[bc + w < nc ? bc + w : nc - 1];
                b[w] = (br < kw && bc + w < nc) ? x : PAD;
            }
        }
#pragma unroll
        for (int w = 0; w < 4; ++w)
            L.Bs[br][(bc >> 2) + w] = make_uint4(Op::norm(b[4 * w]), Op::norm(b[4 * w + 1]),
                                                 Op::norm(b[4 * w + 2]), Op::norm(b[4 * w + 3]));
    }
    __syncthreads();
    const int tx = t & 15, ty = t >> 4;
    const int np = (kw + 1) >> 1;  // an odd kw pairs its last k with a padded one
#pragma unroll 4
    for (int p = 0; p < np; ++p) {
        uint32_t a0[4], a1[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const uint2 av = L.As[p][ty * 4 + m];
            a0[m] = av.x;
            a1[m] = av.y;
        }
        const uint4 b0 = L.Bs[2 * p][tx], b1 = L.Bs[2 * p + 1][tx];
        const uint32_t bb0[4] = {b0.x, b0.y, b0.z, b0.w};
        const uint32_t bb1[4] = {b1.x, b1.y, b1.z, b1.w};
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                acc[m][e] = Op::min3(acc[m][e], Op::add(a0[m], bb0[e]), Op::add(a1[m], bb1[e]));
    }
    __syncthreads();  // every read of the staged operands done before LDS is reused
}

// Floyd-Warshall closure of the register tile over pivots 0 .. kw-1 (kw <=
// 64), ascending.  Pivot row and column do not change under their own pivot
// (zero diagonal), so publishing them before the update is exact.
template <class Op>
__device__ __forceinline__ void close64(uint32_t (&acc)[4][4], int kw, Lds64 &L) {
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    for (int kq = 0; kq < kw; kq += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = kq + u;
            if (k < kw) {  // kw is uniform over the workgroup
                const int s = k & 1;
                if (ty == (kq >> 2)) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) L.rowbuf[s][tx * 4 + e] = acc[u][e];
                }
                if (tx == (kq >> 2)) {
#pragma unroll
                    for (int m = 0; m < 4; ++m) L.colbuf[s][ty * 4 + m] = acc[m][u];
                }
                __syncthreads();
                uint32_t col[4], row[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) col[m] = L.colbuf[s][ty * 4 + m];
#pragma unroll
                for (int e = 0; e < 4; ++e) row[e] = L.rowbuf[s][tx * 4 + e];
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        acc[m][e] = Op::min2(acc[m][e], Op::add(col[m], row[e]));
            }
        }
    }
}

// The same closure with one barrier per two pivots.  For pivots k, k+1 the
// owners publish the rows and columns k and k+1 as they stand before pivot
// k; every thread then forms, for its own rows i and columns j, the entries
// pivot k gives column k+1 and row k+1,
//     c'_i = min(d_i,k+1, d_ik + d_k,k+1)     r'_j = min(d_k+1,j, d_k+1,k + d_kj)
// (the sequential loop's operations on those entries, so its bits; pivot k
// changes neither row k nor column k, d_kk being 0), and applies both pivots
// with one three-input minimum:
//     d_ij = min3(d_ij, d_ik + d_kj, c'_i + r'_j).
// Sequential Floyd-Warshall reaches min(min(d_ij, d_ik + d_kj), c'_i + r'_j)
// from the same two sums; the minimum is exact, so the bits are the same.
// Half the barriers of close64 for the same VALU work.  A trailing odd pivot
// runs alone.  The LDS staging area of update64 is free during a closure and
// holds the published rows and columns (double-buffered).
template <class Op>
__device__ __forceinline__ void close64_pairs(uint32_t (&acc)[4][4], int kw, Lds64 &L) {
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    uint32_t *buf = reinterpret_cast<uint32_t *>(&L.As[0][0]);  // [2][4][64]
    // pivots k = 4 kq + u, u unrolled: the register row/column u of a pivot is
    // a compile-time index
    for (int kq = 0; kq < 16; ++kq) {
#pragma unroll
        for (int u = 0; u < 4; u += 2) {
            const int k = kq * 4 + u;
            if (k < kw) {  // uniform over the workgroup
                const bool pair = k + 1 < kw;
                uint32_t *b = buf + ((k >> 1) & 1) * 256;
                uint32_t *r0 = b, *r1 = b + 64, *c0 = b + 128, *c1 = b + 192;
                if (ty == kq) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        r0[tx * 4 + e] = acc[u][e];
                        r1[tx * 4 + e] = acc[u + 1][e];
                    }
                }
                if (tx == kq) {
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        c0[ty * 4 + m] = acc[m][u];
                        c1[ty * 4 + m] = acc[m][u + 1];
                    }
                }
                __syncthreads();
                uint32_t ck[4], ck1[4], rk[4], rk1[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) ck[m] = c0[ty * 4 + m];
#pragma unroll
                for (int e = 0; e < 4; ++e) rk[e] = r0[tx * 4 + e];
                if (pair) {
                    const uint32_t dk_k1 = r0[k + 1], dk1_k = r1[k];
#pragma unroll
                    for (int m = 0; m < 4; ++m)
                        ck1[m] = Op::min2(c1[ty * 4 + m], Op::add(ck[m], dk_k1));
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        rk1[e] = Op::min2(r1[tx * 4 + e], Op::add(dk1_k, rk[e]));
#pragma unroll
                    for (int m = 0; m < 4; ++m)
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            acc[m][e] = Op::min3(acc[m][e], Op::add(ck[m], rk[e]),
                                                 Op::add(ck1[m], rk1[e]));
                } else {  // the last pivot of an odd kw
#pragma unroll
                    for (int m = 0; m < 4; ++m)
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            acc[m][e] = Op::min2(acc[m][e], Op::add(ck[m], rk[e]));
                }
            }
        }
    }
    __syncthreads();  // every read of the published rows done before the LDS is reused
}

}  // namespace tile64
}  // namespace apsp

// 64 x 64-tile form of the round-synchronous batched solver (the schedule is
// the one of apsp_batched.hip: phase 1 of round 0, then per round r a phase-2
// launch and a phase-3 launch whose diagonal block r+1 is also closed).
// Round width 64 wastes less work on padding for graphs just above a multiple
// of 128 (n = 130 needs two 128-wide rounds, mostly empty, or three 64-wide
// ones); its tile update keeps a 4 x 4 block per thread, so it does more LDS
// traffic per update than the 128-wide form.  Which form a graph gets is
// decided per size bucket by the batched tuning table (apsp_autotune.hip).
//
// One workgroup of 256 threads per 64 x 64 tile; thread (tx, ty) =
// (t % 16, t / 16) keeps rows 4ty .. 4ty+3, columns 4tx .. 4tx+3 in
// registers for the whole item:
//   update    the 64-wide k range of A (stored as k-pairs) and B is staged in
//             LDS in full, then c = min3(c, a0 + b0, a1 + b1) per k-pair;
//   closure   plain Floyd-Warshall over the register tile, pivots ascending:
//             the owners of pivot row and column k put them in LDS (double
//             buffered), one barrier per pivot.
// Tiles are normalised as they are loaded (int32 clamp at 2^30, zero
// diagonal on diagonal tiles), as in the 128-wide form.
#include "apsp_common.h"

namespace apsp {

namespace {

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
            *reinterpret_cast<uint4 *>(crow) = make_uint4(acc[m][0], acc[m][1], acc[m][2], acc[m][3]);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (tx * 4 + e < nc) crow[e] = acc[m][e];
        }
    }
}

// acc = min(acc, A (x) B) with A = D[i0 .., kb .. kb+kw), B = D[kb .. kb+kw, j0 ..]
// (mr x kw and kw x nc valid).  Both operands are staged in full before the
// caller stores acc, so the output tile may be one of them (phase 2).
template <class Op>
__device__ void update64(uint32_t (&acc)[4][4], const uint32_t *D, int64_t ld, int i0, int j0,
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
__device__ void close64(uint32_t (&acc)[4][4], int kw, Lds64 &L) {
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

template <class Op, bool CLOSE_ONLY>
__global__ __launch_bounds__(NT64) void k_batched64(const BatchDesc *__restrict__ descs,
                                                    const BatchItem *__restrict__ items,
                                                    XcdRanges ranges, int r) {
    __shared__ Lds64 L;
    const int x = blockIdx.x & 7, slot = blockIdx.x >> 3;
    if (slot >= ranges.count[x]) return;  // this XCD's list is shorter
    const BatchItem it = items[ranges.offset[x] + slot];
    const BatchDesc g = descs[it.graph];
    uint32_t *D = g.ptr;
    const int n = g.n;
    const int64_t ld = g.ld;
    const bool vec = ((reinterpret_cast<uintptr_t>(D) & 15u) == 0) && ((ld & 3) == 0);
    const int I = it.ij >> 16, J = it.ij & 0xffff;
    const int kb = r * T64, i0 = I * T64, j0 = J * T64;
    const int kw = (n - kb) < T64 ? (n - kb) : T64;
    const int mr = (n - i0) < T64 ? (n - i0) : T64;
    const int nc = (n - j0) < T64 ? (n - j0) : T64;
    uint32_t acc[4][4];
    load64<Op>(acc, D, ld, i0, j0, mr, nc, vec);
    if (CLOSE_ONLY) {
        close64<Op>(acc, kw, L);
    } else {
        update64<Op>(acc, D, ld, i0, j0, kb, mr, nc, kw, vec, L);
        if (I == r + 1 && J == r + 1)  // phase 1 of round r+1, fused
            close64<Op>(acc, mr, L);
    }
    store64<Op>(acc, D, ld, i0, j0, mr, nc, vec);
}

}  // namespace

hipError_t launch_batched64_items(const BatchDesc *descs, const BatchItem *items,
                                  const XcdRanges &ranges, int r, bool close_only, int dtype,
                                  hipStream_t s) {
    int longest = 0;
    for (int x = 0; x < 8; ++x) longest = ranges.count[x] > longest ? ranges.count[x] : longest;
    if (longest == 0) return hipSuccess;
    const dim3 grid((unsigned)longest * 8u);
    if (dtype == 0) {
        if (close_only)
            hipLaunchKernelGGL((k_batched64<OpI32, true>), grid, dim3(NT64), 0, s, descs, items, ranges, r);
        else
            hipLaunchKernelGGL((k_batched64<OpI32, false>), grid, dim3(NT64), 0, s, descs, items, ranges, r);
    } else {
        if (close_only)
            hipLaunchKernelGGL((k_batched64<OpF32, true>), grid, dim3(NT64), 0, s, descs, items, ranges, r);
        else
            hipLaunchKernelGGL((k_batched64<OpF32, false>), grid, dim3(NT64), 0, s, descs, items, ranges, r);
    }
    return hipGetLastError();
}

}  // namespace apsp

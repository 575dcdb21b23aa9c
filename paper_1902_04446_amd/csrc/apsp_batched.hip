// Many independent graphs in one launch: one workgroup per graph runs the
// whole blocked Floyd-Warshall (arXiv:1902.04446, Sec. 4.4/4.5, Algorithms 3
// and 4) on its own matrix with round width 64.  The graph stays in device
// memory (at most 1 MiB for n = 512, so it lives in L2 while its workgroup
// works on it); each phase step stages 64 x 64 blocks through LDS.
//
// Graphs arrive sorted by decreasing n (longest job first), so the hardware's
// in-order workgroup dispatch hands the largest solves out first and the
// small ones fill in behind them.
//
// Within a workgroup the phases are separated by barriers; the memory model
// of a workgroup (one CU, one L1) makes global writes of one wave visible to
// the others after the barrier.
#include "apsp_common.h"

namespace apsp {

namespace {

constexpr int BT = 64;   // batched round width and tile edge
constexpr int BNT = 256; // threads per workgroup

__device__ __forceinline__ uint4 bld4(const uint32_t *p) {
    return *reinterpret_cast<const uint4 *>(p);
}

// Normalise the input of one graph: zero diagonal, int32 clamp at 2^30.
template <class Op, bool IS_I32>
__device__ void batched_prologue(uint32_t *D, int n, int64_t ld) {
    if (IS_I32) {
        // 64 consecutive threads sweep one row segment (coalesced)
        for (int i = threadIdx.x >> 6; i < n; i += BNT / 64) {
            for (int j = threadIdx.x & 63; j < n; j += 64) {
                uint32_t *p = D + i * ld + j;
                const uint32_t v = *p;
                const uint32_t nv = (i == j) ? 0u : (v > kInfI32 ? kInfI32 : v);
                if (nv != v) *p = nv;
            }
        }
    } else {
        for (int i = threadIdx.x; i < n; i += BNT) D[i * ld + i] = 0u;
    }
}

// Phase 1 on the (kw x kw, kw <= 64) diagonal block at (kb, kb).  Thread t
// owns row t/4 and columns (t%4)*16 .. +15, in registers; the pivot row and
// column go through LDS, one barrier per pivot (double-buffered).
template <class Op>
__device__ void batched_phase1(uint32_t *D, int64_t ld, int kb, int kw, uint32_t (*rowbuf)[BT],
                               uint32_t (*colbuf)[BT]) {
    const int t = threadIdx.x;
    const int i = t >> 2;
    const int cg = t & 3;
    const int c0 = cg * 16;
    uint32_t *rowp = D + (int64_t)(kb + (i < kw ? i : kw - 1)) * ld + kb;
    uint32_t v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const uint32_t x = rowp[c0 + u < kw ? c0 + u : kw - 1];
        v[u] = (i < kw && c0 + u < kw) ? x : Op::pad();
    }
    for (int kk = 0; kk < kw; kk += 16) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int k = kk + u;
            if (k < kw) {
                const int s = k & 1;
                if (i == k) {
#pragma unroll
                    for (int w = 0; w < 16; ++w) rowbuf[s][c0 + w] = v[w];
                }
                if (cg == (kk >> 4)) colbuf[s][i] = v[u];
                __syncthreads();
                const uint32_t dik = colbuf[s][i];
#pragma unroll
                for (int w = 0; w < 16; ++w) v[w] = Op::min2(v[w], Op::add(dik, rowbuf[s][c0 + w]));
            }
        }
    }
    __syncthreads();  // every pivot read done before the buffers are reused
    if (i < kw) {
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (c0 + u < kw) rowp[c0 + u] = v[u];
    }
}

// C = min(C, A (x) B) for one 64 x 64 tile: C at (i0, j0) with mr x nc valid
// entries, A = D[i0.., kb..kb+kw), B = D[kb..kb+kw, j0..].  Thread (tx, ty)
// = (t % 16, t / 16) holds the 4 x 4 block rows ty*4.., columns tx*4...
// Operands are read into LDS in full before any output is written, so C may
// overlap A or B (phase 2).
template <class Op>
__device__ void batched_tile(uint32_t *D, int64_t ld, int i0, int j0, int kb, int mr, int nc,
                             int kw, bool vec, uint2 (*As)[BT], uint4 (*Bs)[BT / 4]) {
    const int t = threadIdx.x;
    const uint32_t PAD = Op::pad();
    // A: row t/4, k offset (t%4)*16 .. +15  -> pairs As[k/2][row]
    {
        const int ar = t >> 2, ak = (t & 3) * 16;
        const uint32_t *src = D + (int64_t)(i0 + (ar < mr ? ar : mr - 1)) * ld + kb;
        uint32_t a[16];
        if (vec && ar < mr && ak + 16 <= kw) {
#pragma unroll
            for (int w = 0; w < 16; w += 4) {
                const uint4 x = bld4(src + ak + w);
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
        for (int p = 0; p < 8; ++p) As[(ak >> 1) + p][ar] = make_uint2(a[2 * p], a[2 * p + 1]);
    }
    // B: k row t/4, columns (t%4)*16 .. +15
    {
        const int br = t >> 2, bc = (t & 3) * 16;
        const uint32_t *src = D + (int64_t)(kb + (br < kw ? br : kw - 1)) * ld + j0;
        uint32_t b[16];
        if (vec && br < kw && bc + 16 <= nc) {
#pragma unroll
            for (int w = 0; w < 16; w += 4) {
                const uint4 x = bld4(src + bc + w);
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
            Bs[br][(bc >> 2) + w] = make_uint4(b[4 * w], b[4 * w + 1], b[4 * w + 2], b[4 * w + 3]);
    }
    const int tx = t & 15, ty = t >> 4;
    uint32_t acc[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int row = ty * 4 + m;
        const uint32_t *crow = D + (int64_t)(i0 + (row < mr ? row : mr - 1)) * ld + j0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int c = tx * 4 + e;
            const uint32_t x = crow[c < nc ? c : nc - 1];
            acc[m][e] = (row < mr && c < nc) ? x : PAD;
        }
    }
    __syncthreads();
    const int np = (kw + 1) >> 1;  // an odd kw pairs its last k with a padded one
#pragma unroll 4
    for (int p = 0; p < np; ++p) {
        uint32_t a0[4], a1[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const uint2 av = As[p][ty * 4 + m];
            a0[m] = av.x;
            a1[m] = av.y;
        }
        const uint4 b0 = Bs[2 * p][tx], b1 = Bs[2 * p + 1][tx];
        const uint32_t bb0[4] = {b0.x, b0.y, b0.z, b0.w};
        const uint32_t bb1[4] = {b1.x, b1.y, b1.z, b1.w};
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                acc[m][e] = Op::min3(acc[m][e], Op::add(a0[m], bb0[e]), Op::add(a1[m], bb1[e]));
    }
    __syncthreads();  // all reads of A/B (which may include C) done
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int row = ty * 4 + m;
        if (row >= mr) continue;
        uint32_t *crow = D + (int64_t)(i0 + row) * ld + j0 + tx * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (tx * 4 + e < nc) crow[e] = acc[m][e];
    }
}

template <class Op, bool IS_I32>
__global__ __launch_bounds__(BNT) void k_batched(const BatchDesc *__restrict__ descs) {
    __shared__ uint2 As[BT / 2][BT];
    __shared__ uint4 Bs[BT][BT / 4];
    __shared__ uint32_t rowbuf[2][BT];
    __shared__ uint32_t colbuf[2][BT];

    const BatchDesc g = descs[blockIdx.x];
    uint32_t *D = g.ptr;
    const int n = g.n;
    const int64_t ld = g.ld;
    if (n <= 0) return;
    const bool vec = ((reinterpret_cast<uintptr_t>(D) & 15u) == 0) && ((ld & 3) == 0);

    batched_prologue<Op, IS_I32>(D, n, ld);
    __syncthreads();

    const int q = (n + BT - 1) / BT;
    for (int r = 0; r < q; ++r) {
        const int kb = r * BT;
        const int kw = (n - kb) < BT ? (n - kb) : BT;
        batched_phase1<Op>(D, ld, kb, kw, rowbuf, colbuf);
        __syncthreads();
        // phase 2: block row r, then block column r
        for (int J = 0; J < q; ++J) {
            if (J == r) continue;
            const int j0 = J * BT;
            batched_tile<Op>(D, ld, kb, j0, kb, kw, (n - j0) < BT ? (n - j0) : BT, kw, vec, As, Bs);
        }
        for (int I = 0; I < q; ++I) {
            if (I == r) continue;
            const int i0 = I * BT;
            batched_tile<Op>(D, ld, i0, kb, kb, (n - i0) < BT ? (n - i0) : BT, kw, kw, vec, As, Bs);
        }
        __syncthreads();
        // phase 3: every other block
        for (int I = 0; I < q; ++I) {
            if (I == r) continue;
            const int i0 = I * BT;
            const int mr = (n - i0) < BT ? (n - i0) : BT;
            for (int J = 0; J < q; ++J) {
                if (J == r) continue;
                const int j0 = J * BT;
                batched_tile<Op>(D, ld, i0, j0, kb, mr, (n - j0) < BT ? (n - j0) : BT, kw, vec, As,
                                 Bs);
            }
        }
        __syncthreads();
    }
}

}  // namespace

int batched_tile(int64_t) { return BT; }

hipError_t launch_batched(const BatchDesc *descs_dev, int32_t count, int, int dtype,
                          hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (dtype == 0)
        hipLaunchKernelGGL((k_batched<OpI32, true>), dim3((unsigned)count), dim3(BNT), 0, s,
                           descs_dev);
    else
        hipLaunchKernelGGL((k_batched<OpF32, false>), dim3((unsigned)count), dim3(BNT), 0, s,
                           descs_dev);
    return hipGetLastError();
}

}  // namespace apsp
